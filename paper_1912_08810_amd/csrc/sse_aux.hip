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

// The tables of a batch: blockIdx.y selects the table.
struct NeighBatch {
    const int32_t *neigh[kMaxBatch];
    int64_t n[kMaxBatch];
    int32_t NA[kMaxBatch];
};

__global__ void k_validate_neigh_batch(const NeighBatch nb, uint32_t *status)
{
    const int t = blockIdx.y;
    const int32_t *__restrict__ neigh = nb.neigh[t];
    const int64_t n = nb.n[t];
    const int32_t NA = nb.NA[t];
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

hipError_t launch_validate_neigh_batch(const int32_t *const *neigh, const int64_t *n,
                                       const int32_t *NA, int count, uint32_t *status,
                                       hipStream_t s)
{
    if (count < 1 || count > kMaxBatch)
        return hipErrorInvalidValue;
    NeighBatch nb{};
    int64_t nmax = 1;
    for (int t = 0; t < count; ++t) {
        nb.neigh[t] = neigh[t];
        nb.n[t] = n[t];
        nb.NA[t] = NA[t];
        nmax = n[t] > nmax ? n[t] : nmax;
    }
    int64_t g = (nmax + 255) / 256;
    if (g > 1024)
        g = 1024;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_validate_neigh_batch, dim3((unsigned)g, (unsigned)count), dim3(256), 0,
                       s, nb, status);
    return hipGetLastError();
}

}  // namespace sse
