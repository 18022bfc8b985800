// sse_pi.hip -- binary64 phonon scattering self-energy kernel for gfx950.
//
// Computes Eqs. (4) and (5) (Sec. 2): for frequency w, momentum q, atom a and
// neighbour slot b (f = neigh[a, b]),
//   P_ij[q, w, a, b] = sum_k sum_e tr( dH_ab,i^T . X[(k + q) mod Nkz, e + s_w, a]
//                                     . dH_ab,j . Y[k, e, f] )
//   Pi[q, w, a, b]  =  beta P[q, w, a, b]            (Eq. (5))
//   Pi[q, w, a, NB] = -beta sum_b P[q, w, a, b]      (Eq. (4), the diagonal block)
// with X, Y the two opposite components of G (Pi<: X = G<, Y = G>).
//
// Order of the sums.  The trace is rewritten as tr(X . Z_ij) with
// Z_ij = dH_j . Y . dH_i^T, so that
//   P_ij[q, w] = sum_k sum_e sum_{n,p} X[k + q, e + s_w][n][p] * Zt_ij[k, e][n][p],
//   Zt_ij[n][p] = Z_ij[p][n] = sum_m dH_i[n][m] (dH_j . Y)[p][m]:
// the two Norb x Norb products run once per (k, e) of the workgroup (not once
// per frequency), and each frequency costs one complex multiply-add per orbital
// pair and (i, j) -- the (q, w) correlation the paper's Sec. 4.2 rewrites into
// one GEMM, here without any Norb x Norb product inside it.
//
// Work decomposition: one 256-thread workgroup per (atom a, neighbour slot b,
// momentum q, tap chunk).  It walks k and then e (one energy per step); per step
// the neighbour's block Y[k, e, f] is staged and sandwiched into Zt (two rounds
// of Norb-long dot products through LDS), and atom a's rows X[k + q, e + s] for
// the chunk's shifts are kept in a ring of R = s_hi - s_lo + 1 rows in LDS that
// advances one row per step (rows outside the energy grid are zero).  Thread
// (g, p) owns the 9 x kNT accumulators of (i, j) and the 4 taps of tap group g
// and sums them over the orbital pairs p, p + P, ... of every step; the P
// partial sums of a group are reduced once at the end, in a fixed order.  The
// next step's two rows are loaded into registers while a step's taps run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "sse_internal.h"

namespace sse {

namespace {

constexpr int kBlock = pik::kBlock;
constexpr int kNT = pik::kNT;

__device__ __forceinline__ void cmac(double &accr, double &acci, double ar, double ai, double br,
                                     double bi)
{
    accr = fma(ar, br, accr);
    accr = fma(-ai, bi, accr);
    acci = fma(ar, bi, acci);
    acci = fma(ai, br, acci);
}

// Logical workgroup of physical workgroup `bid`: workgroups are dispatched
// round-robin over the 8 XCDs, so give each XCD a contiguous range of logical
// indices (the b, q and chunk workgroups of one atom, which read the same rows
// of its G, share an L2).
__device__ __forceinline__ int64_t xcd_logical(int64_t bid, int64_t n)
{
    const int64_t per = n >> 3, rem = n & 7;
    const int64_t x = bid & 7, slot = bid >> 3;
    return x * per + (x < rem ? x : rem) + slot;
}

__device__ __forceinline__ int ring_slot(int row, int R)
{
    const int m = row % R;
    return m < 0 ? m + R : m;
}

// First sandwich round: U_j[p][m] = sum_r dH_j[p][r] Y[r][m], j < 3.
__device__ __forceinline__ void sandwich_first(const double *dHs, const double2 *Ys, double2 *Us,
                                               int NN, int No, int tid)
{
#pragma unroll 1
    for (int o = tid; o < 3 * NN; o += kBlock) {
        const int j = o / NN, rem = o - j * NN, r0 = rem / No, m = rem - r0 * No;
        double ur = 0.0, ui = 0.0;
        for (int r = 0; r < No; ++r) {
            const double h = dHs[j * NN + r0 * No + r];
            const double2 y = Ys[r * No + m];
            ur = fma(h, y.x, ur);
            ui = fma(h, y.y, ui);
        }
        Us[o] = make_double2(ur, ui);
    }
}

// Second round: Zt_ij[n][p] = sum_m dH_i[n][m] U_j[p][m] (= (dH_j Y dH_i^T)[p][n]).
__device__ __forceinline__ void sandwich_second(const double *dHs, const double2 *Us, double2 *Zs,
                                                int NN, int No, int tid)
{
#pragma unroll 1
    for (int o = tid; o < kNF * NN; o += kBlock) {
        const int ij = o / NN, rem = o - ij * NN, n = rem / No, r0 = rem - n * No;
        const int i = ij / 3, j = ij - 3 * i;
        double zr = 0.0, zi = 0.0;
        for (int m = 0; m < No; ++m) {
            const double h = dHs[i * NN + n * No + m];
            const double2 u = Us[j * NN + r0 * No + m];
            zr = fma(h, u.x, zr);
            zi = fma(h, u.y, zi);
        }
        Zs[o] = make_double2(zr, zi);
    }
}

__global__ __launch_bounds__(kBlock, 1) void k_pi_fp64(const PiParams p)
{
    extern __shared__ double2 lds[];
    const int NN = p.NN, No = p.Norb, R = p.R;
    double2 *ring = lds;                 // [R][NN]
    double2 *Zs = ring + (size_t)R * NN; // [9][NN]: Zt_ij[n][p] at ij * NN + n * No + p
    double2 *Us = Zs + 9 * NN;           // [3][NN]: (dH_j . Y)[p][m]
    double2 *Ys = Us + 3 * NN;           // [NN]
    double *dHs = reinterpret_cast<double *>(Ys + NN);  // [3][NN]
    const int tid = threadIdx.x;

    int64_t L = xcd_logical(blockIdx.x, p.n_wg);
    const int chunk = (int)(L % p.nchunk);
    L /= p.nchunk;
    const int q = (int)(L % p.Nqz);
    L /= p.Nqz;
    const int b = (int)(L % p.NB);
    const int a = (int)(L / p.NB);
    const int f = p.neigh[(size_t)a * p.NB + b];
    const int t0 = p.cb[chunk], t1 = p.cb[chunk + 1];
    const int s_lo = p.ts[t0], s_hi = p.ts[t1 - 1];
    const int ngroups = p.cg[chunk];
    const int P = kBlock / ngroups;
    const int g = tid / P, pp = tid % P;
    const size_t out_a = (size_t)a * (p.NB + 1) + b;  // output block (.., a, b) per (q, w)
    const size_t qw_stride = (size_t)p.NA * (p.NB + 1) * kNF;

    if (f < 0 || f >= p.NA) {
        // reported by the neighbour check; the block is left zero
        for (int t = t0 + tid; t < t1; t += kBlock)
            for (int ij = 0; ij < kNF; ++ij)
                p.Pi[((size_t)q * p.Nw + p.tw[t]) * qw_stride + out_a * kNF + ij] =
                    make_double2(0.0, 0.0);
        return;
    }

    for (int x = tid; x < 3 * NN; x += kBlock)
        dHs[x] = p.dH[((size_t)a * p.NB + b) * 3 * NN + x];

    // this thread's taps; unused slots repeat the chunk's first shift
    int su[kNT];
    bool valid[kNT];
#pragma unroll
    for (int u = 0; u < kNT; ++u) {
        const int t = t0 + g * kNT + u;
        valid[u] = g < ngroups && t < t1;
        su[u] = valid[u] ? p.ts[t] : s_lo;
    }
    double accr[kNF][kNT], acci[kNF][kNT];
#pragma unroll
    for (int ij = 0; ij < kNF; ++ij)
#pragma unroll
        for (int u = 0; u < kNT; ++u)
            accr[ij][u] = acci[ij][u] = 0.0;

    const size_t row_stride = (size_t)p.NA * NN;  // one energy step of G
    const double2 zero = make_double2(0.0, 0.0);

    for (int k = 0; k < p.Nkz; ++k) {
        const int kx = (k + q) % p.Nkz;
        const double2 *Xk = p.X + ((size_t)kx * p.NE * p.NA + a) * NN;
        const double2 *Yk = p.Y + ((size_t)k * p.NE * p.NA + f) * NN;
        __syncthreads();  // the previous k's last step is done with the ring, Us and Ys
        // ring rows s_lo .. s_hi - 1 (step 0's rows but its top one); Y[k, 0, f]
        for (int x = tid; x < (s_hi - s_lo) * NN; x += kBlock) {
            const int row = s_lo + x / NN, c = x % NN;
            ring[ring_slot(row, R) * NN + c] =
                (row >= 0 && row < p.NE) ? Xk[(size_t)row * row_stride + c] : zero;
        }
        double2 yv = zero, xv = zero;  // rows in flight: Y of a later step, the ring's next top row
        if (tid < NN) {
            Ys[tid] = Yk[tid];
            if (s_hi >= 0 && s_hi < p.NE)
                xv = Xk[(size_t)s_hi * row_stride + tid];
            if (1 < p.NE)
                yv = Yk[row_stride + tid];
        }
        __syncthreads();
        sandwich_first(dHs, Ys, Us, NN, No, tid);
        __syncthreads();
        for (int es = 0;; ++es) {
            // ---- phase B: second sandwich round of step es; the ring's top row
            // for step es and Y of step es + 1 go to LDS; the next two rows load
            if (es < p.NE) {
                sandwich_second(dHs, Us, Zs, NN, No, tid);
                if (tid < NN) {
                    ring[ring_slot(es + s_hi, R) * NN + tid] = xv;
                    if (es + 1 < p.NE)
                        Ys[tid] = yv;
                    xv = zero;
                    yv = zero;
                    const int row = es + 1 + s_hi;
                    if (row >= 0 && row < p.NE)
                        xv = Xk[(size_t)row * row_stride + tid];
                    if (es + 2 < p.NE)
                        yv = Yk[(size_t)(es + 2) * row_stride + tid];
                }
            }
            __syncthreads();
            if (es >= p.NE)
                break;
            // ---- phase A: the taps of step es, then the first sandwich round of es + 1
            if (g < ngroups) {
                int rs[kNT];
#pragma unroll
                for (int u = 0; u < kNT; ++u)
                    rs[u] = ring_slot(es + su[u], R) * NN;
#pragma unroll 1
                for (int c = pp; c < NN; c += P) {
                    double2 xx[kNT];
#pragma unroll
                    for (int u = 0; u < kNT; ++u)
                        xx[u] = ring[rs[u] + c];
#pragma unroll
                    for (int ij = 0; ij < kNF; ++ij) {
                        const double2 z = Zs[ij * NN + c];
#pragma unroll
                        for (int u = 0; u < kNT; ++u)
                            cmac(accr[ij][u], acci[ij][u], z.x, z.y, xx[u].x, xx[u].y);
                    }
                }
            }
            if (es + 1 < p.NE)
                sandwich_first(dHs, Ys, Us, NN, No, tid);
            __syncthreads();
        }
    }

    // ---- reduce each group's P partial sums in a fixed order, write beta * P
    __syncthreads();
    const int lane = tid & 63;
    const int pw = P < 64 ? P : 64;  // partitions of one group inside a wave
#pragma unroll
    for (int ij = 0; ij < kNF; ++ij)
#pragma unroll
        for (int u = 0; u < kNT; ++u)
            for (int off = pw >> 1; off > 0; off >>= 1) {
                accr[ij][u] += __shfl_xor(accr[ij][u], off);
                acci[ij][u] += __shfl_xor(acci[ij][u], off);
            }
    // waves of one group (P > 64) combine through LDS, lowest wave first
    double2 *red = lds;  // [4 waves][kNF][kNT]
    const int wave = tid >> 6;
    const int wpg = P > 64 ? P / 64 : 1;  // waves per group
    if (wpg > 1 && lane == 0) {
#pragma unroll
        for (int ij = 0; ij < kNF; ++ij)
#pragma unroll
            for (int u = 0; u < kNT; ++u)
                red[(wave * kNF + ij) * kNT + u] = make_double2(accr[ij][u], acci[ij][u]);
    }
    __syncthreads();
    if (g < ngroups && pp == 0) {
        if (wpg > 1) {
#pragma unroll
            for (int ij = 0; ij < kNF; ++ij)
#pragma unroll
                for (int u = 0; u < kNT; ++u) {
                    double sr = 0.0, si = 0.0;
                    for (int v = 0; v < wpg; ++v) {
                        const double2 x = red[((wave + v) * kNF + ij) * kNT + u];
                        sr += x.x;
                        si += x.y;
                    }
                    accr[ij][u] = sr;
                    acci[ij][u] = si;
                }
        }
#pragma unroll
        for (int u = 0; u < kNT; ++u) {
            if (!valid[u])
                continue;
            const int t = t0 + g * kNT + u;
            double2 *o = p.Pi + ((size_t)q * p.Nw + p.tw[t]) * qw_stride + out_a * kNF;
#pragma unroll
            for (int ij = 0; ij < kNF; ++ij)
                o[ij] = make_double2(p.beta_re * accr[ij][u] - p.beta_im * acci[ij][u],
                                     p.beta_re * acci[ij][u] + p.beta_im * accr[ij][u]);
        }
    }
}

// Diagonal blocks (Eq. (4)): Pi[q, w, a, NB] = -sum_b Pi[q, w, a, b], summed
// in b order, one thread per (q, w, a, i, j).
__global__ void k_pi_diag(double2 *Pi, int64_t nqwa, int NB)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nqwa * kNF)
        return;
    const int64_t qwa = x / kNF;
    const int ij = (int)(x - qwa * kNF);
    double2 *blk = Pi + (size_t)qwa * (NB + 1) * kNF;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < NB; ++b) {
        const double2 v = blk[b * kNF + ij];
        sr += v.x;
        si += v.y;
    }
    blk[NB * kNF + ij] = make_double2(-sr, -si);
}

}  // namespace

hipError_t pi_launch(const PiParams &p, size_t lds_bytes, hipStream_t s)
{
    if (p.n_wg <= 0)
        return hipSuccess;
    if (p.n_wg > 0x7fffffffLL)
        return hipErrorInvalidConfiguration;
    static bool done = false;
    if (!done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_pi_fp64,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)pik::kLdsBudgetOne);
        if (e != hipSuccess)
            return e;
        done = true;
    }
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_pi_fp64, dim3((unsigned)p.n_wg), dim3(kBlock), lds_bytes, s, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int64_t nqwa = (int64_t)p.Nqz * p.Nw * p.NA;
    const int64_t n = nqwa * kNF;
    hipLaunchKernelGGL(k_pi_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.Pi, nqwa,
                       p.NB);
    return hipGetLastError();
}

}  // namespace sse
