// sse_check.hip -- sampled binary64 check of a complex64 self-energy result.
//
// For a list of output blocks (k, e, a) the kernel recomputes Sigma[k, e, a]
// of Eq. (3) (Sec. 2) in binary64 from the same complex64-stored inputs --
// nine tap filters per channel read straight from G and D~ in global memory,
// then the dH sandwich through LDS -- and accumulates, per block,
// |Sigma_stored - Sigma_ref|^2 and |Sigma_ref|^2.  A second one-workgroup
// kernel sums the per-block partials in block order, so the result (and any
// decision taken on it) does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "sse_internal.h"

namespace sse {

namespace {

constexpr int kBlock = 256;
constexpr int kCmax = 2;  // channels per thread: Norb^2 <= 512

__global__ __launch_bounds__(kBlock) void k_check(const CheckParams p)
{
    extern __shared__ double2 sm[];
    const int NN = p.NN, No = p.Norb;
    double2 *S = sm;                                      // [3][NN] scratch
    double *A = reinterpret_cast<double *>(sm + 3 * NN);  // [3][NN] dH of the bond
    __shared__ double red[2][kBlock];

    const int id = blockIdx.x;
    const int k = p.blocks[3 * id], e = p.blocks[3 * id + 1], a = p.blocks[3 * id + 2];
    const int tid = threadIdx.x;
    if (k < 0 || k >= p.Nkz || e < 0 || e >= p.NE || a < 0 || a >= p.NA) {
        if (tid == 0) {
            p.partial[2 * id] = 0.0;
            p.partial[2 * id + 1] = 0.0;
            atomicOr(p.status, kStatusBadBlock);
        }
        return;
    }
    const size_t strideE = (size_t)p.NA * NN;
    const size_t strideD = (size_t)p.NA * p.NB * kNF;

    double sr[kCmax] = {0.0, 0.0}, si[kCmax] = {0.0, 0.0};
    for (int b = 0; b < p.NB; ++b) {
        const int f = p.neigh[(size_t)a * p.NB + b];
        if ((unsigned)f >= (unsigned)p.NA)
            continue;
        double gr[kCmax][kNF], gi[kCmax][kNF];
#pragma unroll
        for (int u = 0; u < kCmax; ++u)
#pragma unroll
            for (int x = 0; x < kNF; ++x)
                gr[u][x] = gi[u][x] = 0.0;
        for (int q = 0; q < p.Nqz; ++q) {
            int kk = k - q;
            if (kk < 0)
                kk += p.Nkz;
            for (int w = 0; w < p.Nw; ++w) {
                const int ee = e - p.shift[w];
                if (ee < 0 || ee >= p.NE)
                    continue;
                const float2 *g = p.G + ((size_t)kk * p.NE + ee) * strideE + (size_t)f * NN;
                const float2 *d =
                    p.D + ((size_t)q * p.Nw + w) * strideD + ((size_t)a * p.NB + b) * kNF;
#pragma unroll
                for (int u = 0; u < kCmax; ++u) {
                    const int c = tid + u * kBlock;
                    if (c >= NN)
                        continue;
                    const double xr = g[c].x, xi = g[c].y;
#pragma unroll
                    for (int x = 0; x < kNF; ++x) {
                        const double dr = d[x].x, di = d[x].y;
                        gr[u][x] += dr * xr - di * xi;
                        gi[u][x] += dr * xi + di * xr;
                    }
                }
            }
        }
        __syncthreads();
        const double *Ag = p.dH + ((size_t)a * p.NB + b) * kN3D * NN;
        for (int x = tid; x < kN3D * NN; x += kBlock)
            A[x] = Ag[x];
        double tr[kCmax][kN3D], ti[kCmax][kN3D];
#pragma unroll
        for (int u = 0; u < kCmax; ++u)
#pragma unroll
            for (int j = 0; j < kN3D; ++j)
                tr[u][j] = ti[u][j] = 0.0;
        for (int i = 0; i < kN3D; ++i) {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kCmax; ++u) {
                const int c = tid + u * kBlock;
                if (c < NN)
#pragma unroll
                    for (int j = 0; j < kN3D; ++j)
                        S[j * NN + c] = make_double2(gr[u][i * kN3D + j], gi[u][i * kN3D + j]);
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kCmax; ++u) {
                const int c = tid + u * kBlock;
                if (c >= NN)
                    continue;
                const int m = c / No, n = c - m * No;
                for (int l = 0; l < No; ++l) {
                    const double am = A[i * NN + m * No + l];
#pragma unroll
                    for (int j = 0; j < kN3D; ++j) {
                        const double2 s = S[j * NN + l * No + n];
                        tr[u][j] += am * s.x;
                        ti[u][j] += am * s.y;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kCmax; ++u) {
            const int c = tid + u * kBlock;
            if (c < NN)
#pragma unroll
                for (int j = 0; j < kN3D; ++j)
                    S[j * NN + c] = make_double2(tr[u][j], ti[u][j]);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kCmax; ++u) {
            const int c = tid + u * kBlock;
            if (c >= NN)
                continue;
            const int m = c / No, n = c - m * No;
            for (int j = 0; j < kN3D; ++j)
                for (int l = 0; l < No; ++l) {
                    const double2 s = S[j * NN + m * No + l];
                    const double am = A[j * NN + n * No + l];
                    sr[u] += s.x * am;
                    si[u] += s.y * am;
                }
        }
    }

    double d2 = 0.0, r2 = 0.0;
    const float2 *got = p.Sigma + ((size_t)k * p.NE + e) * strideE + (size_t)a * NN;
#pragma unroll
    for (int u = 0; u < kCmax; ++u) {
        const int c = tid + u * kBlock;
        if (c >= NN)
            continue;
        const double rr = p.alpha_re * sr[u] - p.alpha_im * si[u];
        const double ri = p.alpha_re * si[u] + p.alpha_im * sr[u];
        const double dx = (double)got[c].x - rr, dy = (double)got[c].y - ri;
        d2 += dx * dx + dy * dy;
        r2 += rr * rr + ri * ri;
    }
    red[0][tid] = d2;
    red[1][tid] = r2;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if (tid < h) {
            red[0][tid] += red[0][tid + h];
            red[1][tid] += red[1][tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
        p.partial[2 * id] = red[0][0];
        p.partial[2 * id + 1] = red[1][0];
    }
}

// Sums the per-block partials in block order: out = (sum |diff|^2, sum |ref|^2).
__global__ void k_check_reduce(const double *partial, int n, double *out)
{
    if (threadIdx.x == 0) {
        double d2 = 0.0, r2 = 0.0;
        for (int t = 0; t < n; ++t) {
            d2 += partial[2 * t];
            r2 += partial[2 * t + 1];
        }
        out[0] = d2;
        out[1] = r2;
    }
}

}  // namespace

hipError_t check_launch(const CheckParams &p, double *out, hipStream_t s)
{
    if (p.nblocks <= 0)
        return hipSuccess;
    const size_t lds = (size_t)3 * p.NN * sizeof(double2) + (size_t)3 * p.NN * sizeof(double);
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_check,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
        if (e != hipSuccess)
            return e;
        attr = true;
    }
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_check, dim3(p.nblocks), dim3(kBlock), lds, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_check_reduce, dim3(1), dim3(64), 0, s, p.partial, p.nblocks, out);
    return hipGetLastError();
}

}  // namespace sse
