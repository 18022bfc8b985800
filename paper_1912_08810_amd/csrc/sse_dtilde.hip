// sse_dtilde.hip -- the steps either side of the self-energy kernels:
//   * the phonon Green's function blocks combined as Eq. (3) consumes them,
//       Dt[q, w, a, b] = D_ba - D_bb - D_aa + D_ab   (each 3 x 3, entry by entry),
//     from D [Nqz, Nw, NA, NB + 1, 3, 3] (neighbour blocks D_a,neigh[a, b] in
//     slots b < NB, the diagonal block D_aa in slot NB), through the reverse
//     neighbour map r(a, b) = the slot of a in the row of f = neigh[a, b];
//   * the retarded component (X> - X<) / 2 of Sigma or Pi (Sec. 2, after Eq. (5)).
// Both are memory-bound elementwise passes: one thread per complex element,
// consecutive threads on consecutive elements of the output.
#include <hip/hip_runtime.h>

#include "sse_internal.h"

namespace sse {

namespace {

__device__ __forceinline__ double2 ld(const double2 *p, size_t i) { return p[i]; }
__device__ __forceinline__ double2 ld(const float2 *p, size_t i)
{
    const float2 v = p[i];
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st(double2 *p, size_t i, double x, double y)
{
    p[i] = make_double2(x, y);
}
__device__ __forceinline__ void st(float2 *p, size_t i, double x, double y)
{
    p[i] = make_float2((float)x, (float)y);
}

// rmap[a NB + b] = first slot r with neigh[f, r] == a (f = neigh[a, b]); -1 and
// a status bit when f is out of range or does not list a.
__global__ void k_reverse_map(const int32_t *neigh, int32_t NA, int32_t NB, int32_t *rmap,
                              uint32_t *status)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (int64_t)NA * NB)
        return;
    const int a = (int)(x / NB);
    const int f = neigh[x];
    int r = -1;
    if (f < 0 || f >= NA) {
        atomicOr(status, kStatusBadNeigh);
    } else {
        for (int s = NB - 1; s >= 0; --s)
            if (neigh[(size_t)f * NB + s] == a)
                r = s;
        if (r < 0)
            atomicOr(status, kStatusAsymNeigh);
    }
    rmap[x] = r;
}

// One thread per (q w, a, b, i j) element of Dt; the sum is formed left to right
// as written above, in binary64 (complex64 storage is promoted on load and
// rounded once on store).  Entries whose neighbour has no reverse slot are 0.
template <typename T>
__global__ void k_dtilde(const T *D, T *Dt, const int32_t *neigh, const int32_t *rmap,
                         int64_t nqw, int32_t NA, int32_t NB)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = nqw * NA * NB * kNF;
    if (x >= n)
        return;
    const int ij = (int)(x % kNF);
    const int64_t ab = x / kNF;             // (q w, a, b)
    const int b = (int)(ab % NB);
    const int64_t qwa = ab / NB;            // (q w, a)
    const int a = (int)(qwa % NA);
    const int64_t qw = qwa / NA;
    const int f = neigh[(size_t)a * NB + b];
    const int r = rmap[(size_t)a * NB + b];
    if (r < 0 || f < 0 || f >= NA) {
        st(Dt, (size_t)x, 0.0, 0.0);
        return;
    }
    const size_t rowa = ((size_t)qw * NA + a) * (NB + 1) * kNF;
    const size_t rowf = ((size_t)qw * NA + f) * (NB + 1) * kNF;
    const double2 d_ba = ld(D, rowf + (size_t)r * kNF + ij);
    const double2 d_bb = ld(D, rowf + (size_t)NB * kNF + ij);
    const double2 d_aa = ld(D, rowa + (size_t)NB * kNF + ij);
    const double2 d_ab = ld(D, rowa + (size_t)b * kNF + ij);
    st(Dt, (size_t)x, ((d_ba.x - d_bb.x) - d_aa.x) + d_ab.x, ((d_ba.y - d_bb.y) - d_aa.y) + d_ab.y);
}

// XR[i] = (X[n + i] - X[i]) / 2 over n complex elements.
template <typename T>
__global__ void k_retarded(const T *X, T *XR, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double2 l = ld(X, (size_t)i), g = ld(X, (size_t)(n + i));
    st(XR, (size_t)i, (g.x - l.x) * 0.5, (g.y - l.y) * 0.5);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t dtilde_launch(const void *D, void *Dt, const int32_t *neigh, int32_t *rmap,
                         uint32_t *status, int64_t nqw, int32_t NA, int32_t NB, bool c64,
                         hipStream_t s)
{
    const int64_t nab = (int64_t)NA * NB;
    const int64_t n = nqw * nab * kNF;
    if (blocks_for(n) > 0x7fffffffu)
        return hipErrorInvalidConfiguration;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_reverse_map, dim3(blocks_for(nab)), dim3(256), 0, s, neigh, NA, NB, rmap,
                       status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0)
        return e;
    if (c64)
        hipLaunchKernelGGL(k_dtilde<float2>, dim3(blocks_for(n)), dim3(256), 0, s,
                           (const float2 *)D, (float2 *)Dt, neigh, (const int32_t *)rmap, nqw, NA,
                           NB);
    else
        hipLaunchKernelGGL(k_dtilde<double2>, dim3(blocks_for(n)), dim3(256), 0, s,
                           (const double2 *)D, (double2 *)Dt, neigh, (const int32_t *)rmap, nqw,
                           NA, NB);
    return hipGetLastError();
}

hipError_t retarded_launch(const void *X, void *XR, int64_t n, bool c64, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    if (blocks_for(n) > 0x7fffffffu)
        return hipErrorInvalidConfiguration;
    (void)hipGetLastError();
    if (c64)
        hipLaunchKernelGGL(k_retarded<float2>, dim3(blocks_for(n)), dim3(256), 0, s,
                           (const float2 *)X, (float2 *)XR, n);
    else
        hipLaunchKernelGGL(k_retarded<double2>, dim3(blocks_for(n)), dim3(256), 0, s,
                           (const double2 *)X, (double2 *)XR, n);
    return hipGetLastError();
}

}  // namespace sse
