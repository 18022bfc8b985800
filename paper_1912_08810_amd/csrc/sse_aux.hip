// sse_aux.hip -- small kernels around the self-energy launch: status word
// reset and the device-side neighbour-table check (every neigh[a, b] must be
// an atom index in [0, NA), the indirection f(a, b) of Sec. 4.1).
#include <hip/hip_runtime.h>

#include "sse_internal.h"

namespace sse {

namespace {

__global__ void k_clear_status(uint32_t *status) { status[0] = 0u; }

__global__ void k_clear_u64(unsigned long long *p, int n)
{
    if ((int)threadIdx.x < n)
        p[threadIdx.x] = 0ULL;
}

__global__ void k_validate_neigh(const int32_t *__restrict__ neigh, int64_t n, int32_t NA,
                                 uint32_t *status)
{
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t f = neigh[i];
        bad |= (f < 0 || f >= NA);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0)
        atomicOr(status, kStatusBadNeigh);
}

}  // namespace

hipError_t launch_clear_status(uint32_t *status, hipStream_t s)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, status);
    return hipGetLastError();
}

hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_clear_u64, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_validate_neigh(const int32_t *neigh, int64_t n, int32_t NA, uint32_t *status,
                                 hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    if (g > 1024)
        g = 1024;
    if (g < 1)
        g = 1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_validate_neigh, dim3((unsigned)g), dim3(256), 0, s, neigh, n, NA, status);
    return hipGetLastError();
}

}  // namespace sse
