// sse_fp64.hip -- binary64 scattering self-energy kernel for gfx950.
//
// Computes Eq. (3) (Sec. 2) in a reassociated order that does the same sums:
//   Gh_ij[k, e, a, b] = sum_q sum_w Dt[q, w, a, b, i, j] * G[(k - q) mod Nkz, e - s_w, f]
//   Sigma[k, e, a]    = alpha * sum_b sum_i sum_j dH_i . Gh_ij . dH_j^T
// The (qz, w) sums act on G alone, so they are taken first as nine scalar
// filters over the Norb^2 channels of the neighbour's G block (the redundancy
// the paper removes in Sec. 4.2 by hoisting dH.G out of the (qz, w) loops,
// carried one step further: the Norb x Norb products leave the (qz, w) loop
// entirely); the dH sandwich then runs once per (k, e, a, b).
//
// Work decomposition: one 256-thread workgroup per (energy tile, k, a).  Its
// TE x Norb^2 output positions (energy, orbital pair) are flattened; thread t
// owns positions t + 256 r, r < R.  For each neighbour b and momentum
// transfer q, the workgroup stages the neighbour's G rows for energies
// [e0 - s_max, e0 + TE - s_min) into LDS (the energy window of the tap chunk);
// each tap w is then a uniform offset (s_max - s_w) Norb^2 into that window, so
// every tap is one 16-byte LDS read per position feeding 36 fp64 FMAs (nine
// complex multiply-adds with the wave-uniform D~ values held in SGPRs).  The
// sandwich dH_i Gh_ij dH_j^T goes through LDS (two rounds of Norb-long dot
// products) and is summed over b in registers.  Sigma is written once,
// coalesced.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sse_internal.h"

namespace sse {

namespace {

constexpr int kBlock = 256;
constexpr int kR = 4;
constexpr int kPmax = kBlock * kR;
// LDS per workgroup: two workgroups share one CU's 160 KiB.
constexpr size_t kLdsBudget = 78 * 1024;

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical tiles so tiles that read the same G rows (the
// Nkz momenta and neighbouring energy tiles of one atom) share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t n)
{
    const int64_t per = n >> 3;
    if (bid >= (per << 3))
        return bid;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ void cmac(double &accr, double &acci, double dr, double di, double gr,
                                     double gi)
{
    accr = fma(dr, gr, accr);
    accr = fma(-di, gi, accr);
    acci = fma(dr, gi, acci);
    acci = fma(di, gr, acci);
}

__global__ __launch_bounds__(kBlock, 2) void k_sse_fp64(const Fp64Params p)
{
    extern __shared__ double2 lds[];
    double *ldsA = reinterpret_cast<double *>(lds + p.lds_win);

    int64_t L = xcd_remap(blockIdx.x, p.n_wg);
    const int k = (int)(L % p.Nkz);
    L /= p.Nkz;
    const int et = (int)(L % p.n_etiles);
    const int a = (int)(L / p.n_etiles);
    const int e0 = et * p.TE;
    const int te = min(p.TE, p.NE - e0);
    const int NN = p.NN, No = p.Norb;
    const int P = te * NN;
    const int Pst = p.TE * NN;  // scratch stride between the three filters of a round
    const int tid = threadIdx.x;

    int pos[kR];
    bool valid[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        pos[r] = tid + r * kBlock;
        valid[r] = pos[r] < P;
        if (!valid[r])
            pos[r] = 0;
    }
    // orbital coordinates of each position: energy el, row m, column n
    int pe[kR], pm[kR], pn[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        pe[r] = pos[r] / NN;
        const int c = pos[r] - pe[r] * NN;
        pm[r] = c / No;
        pn[r] = c - pm[r] * No;
    }

    double sr[kR], si[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        sr[r] = 0.0;
        si[r] = 0.0;
    }

    const size_t strideD = (size_t)p.NA * p.NB * kNF;  // one (q, w) slab of D~
    const size_t strideE = (size_t)p.NA * NN;          // one energy row of G

    for (int b = 0; b < p.NB; ++b) {
        const int f = p.neigh[(size_t)a * p.NB + b];
        if ((unsigned)f >= (unsigned)p.NA)
            continue;  // invalid neighbour: reported by the validation kernel

        double ar[kR][kNF], ai[kR][kNF];
#pragma unroll
        for (int r = 0; r < kR; ++r)
#pragma unroll
            for (int x = 0; x < kNF; ++x) {
                ar[r][x] = 0.0;
                ai[r][x] = 0.0;
            }

        const double2 *Dab = p.D + ((size_t)a * p.NB + b) * kNF;
        for (int q = 0; q < p.Nqz; ++q) {
            int kk = k - q;
            if (kk < 0)
                kk += p.Nkz;
            const double2 *Gk = p.G + (size_t)kk * p.NE * strideE + (size_t)f * NN;
            for (int c = 0; c < p.taps.nchunk; ++c) {
                const int t0 = p.taps.cb[c], t1 = p.taps.cb[c + 1];
                const int smax = p.taps.s[t0], smin = p.taps.s[t1 - 1];
                const int wn = (te + smax - smin) * NN;
                const int ebase = e0 - smax;
                __syncthreads();
                for (int idx = tid; idx < wn; idx += kBlock) {
                    const int ew = idx / NN;
                    const int cc = idx - ew * NN;
                    const int e = ebase + ew;
                    double2 v = make_double2(0.0, 0.0);
                    if (e >= 0 && e < p.NE)
                        v = Gk[(size_t)e * strideE + cc];
                    lds[idx] = v;
                }
                __syncthreads();
                for (int t = t0; t < t1; ++t) {
                    const int off = (smax - p.taps.s[t]) * NN;
                    const double2 *dp = Dab + (size_t)(q * p.Nw + p.taps.w[t]) * strideD;
                    double dr[kNF], di[kNF];
#pragma unroll
                    for (int x = 0; x < kNF; ++x) {
                        const double2 d = dp[x];
                        dr[x] = d.x;
                        di[x] = d.y;
                    }
#pragma unroll
                    for (int r = 0; r < kR; ++r) {
                        const double2 g = lds[pos[r] + off];
#pragma unroll
                        for (int x = 0; x < kNF; ++x)
                            cmac(ar[r][x], ai[r][x], dr[x], di[x], g.x, g.y);
                    }
                }
            }
        }

        // ---- sandwich: Sigma += sum_ij dH_i Gh_ij dH_j^T for this neighbour
        __syncthreads();  // window reads done; LDS becomes scratch
        const double *Ag = p.dH + ((size_t)a * p.NB + b) * kN3D * NN;
        for (int idx = tid; idx < kN3D * NN; idx += kBlock)
            ldsA[idx] = Ag[idx];

        // T_j = sum_i dH_i Gh_ij, one i per round
        double tr[kR][kN3D], ti[kR][kN3D];
#pragma unroll
        for (int r = 0; r < kR; ++r)
#pragma unroll
            for (int j = 0; j < kN3D; ++j) {
                tr[r][j] = 0.0;
                ti[r][j] = 0.0;
            }
#pragma unroll
        for (int i = 0; i < kN3D; ++i) {
            if (i > 0)
                __syncthreads();
#pragma unroll
            for (int r = 0; r < kR; ++r)
                if (valid[r])
#pragma unroll
                    for (int j = 0; j < kN3D; ++j)
                        lds[j * Pst + pos[r]] = make_double2(ar[r][i * kN3D + j], ai[r][i * kN3D + j]);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int base = pe[r] * NN + pn[r];
                const double *Arow = ldsA + i * NN + pm[r] * No;
                for (int l = 0; l < No; ++l) {
                    const double am = Arow[l];
#pragma unroll
                    for (int j = 0; j < kN3D; ++j) {
                        const double2 s = lds[j * Pst + base + l * No];
                        tr[r][j] = fma(am, s.x, tr[r][j]);
                        ti[r][j] = fma(am, s.y, ti[r][j]);
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kR; ++r)
            if (valid[r])
#pragma unroll
                for (int j = 0; j < kN3D; ++j)
                    lds[j * Pst + pos[r]] = make_double2(tr[r][j], ti[r][j]);
        __syncthreads();
        // Sigma_mn += sum_j sum_l T_j[m, l] dH_j[n, l]
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int base = pe[r] * NN + pm[r] * No;
#pragma unroll
            for (int j = 0; j < kN3D; ++j) {
                const double *Arow = ldsA + j * NN + pn[r] * No;
                for (int l = 0; l < No; ++l) {
                    const double2 s = lds[j * Pst + base + l];
                    const double am = Arow[l];
                    sr[r] = fma(s.x, am, sr[r]);
                    si[r] = fma(s.y, am, si[r]);
                }
            }
        }
    }

    // ---- Sigma[k, e0 + el, a] = alpha * accumulated sum
    double2 *Sk = p.Sigma + ((size_t)k * p.NE + e0) * strideE + (size_t)a * NN;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        if (!valid[r])
            continue;
        const int c = pos[r] - pe[r] * NN;
        Sk[(size_t)pe[r] * strideE + c] =
            make_double2(p.alpha_re * sr[r] - p.alpha_im * si[r], p.alpha_re * si[r] + p.alpha_im * sr[r]);
    }
}

}  // namespace

TileGeom fp64_geometry(int Norb, int NE, const TapTable &taps, int te_request, TapTable *out)
{
    const int NN = Norb * Norb;
    int TE = kPmax / NN;
    if (te_request > 0)
        TE = std::min(TE, te_request);
    TE = std::max(1, std::min(TE, NE));
    const size_t a_bytes = (size_t)kN3D * NN * sizeof(double);
    const long budget = (long)((kLdsBudget - a_bytes) / sizeof(double2));

    *out = taps;
    out->nchunk = 0;
    int t = 0;
    long win_max = 0;
    while (t < taps.n) {
        int u = t + 1;
        while (u < taps.n && (long)(TE + taps.s[t] - taps.s[u]) * NN <= budget)
            ++u;
        out->cb[out->nchunk++] = t;
        win_max = std::max(win_max, (long)(TE + taps.s[t] - taps.s[u - 1]) * NN);
        t = u;
    }
    out->cb[out->nchunk] = taps.n;
    TileGeom g;
    g.TE = TE;
    g.n_etiles = (NE + TE - 1) / TE;
    g.lds_win = (int)std::max(win_max, (long)kN3D * TE * NN);
    g.lds_bytes = (size_t)g.lds_win * sizeof(double2) + a_bytes;
    return g;
}

hipError_t fp64_launch(const Fp64Params &p, size_t lds_bytes, hipStream_t s)
{
    if (p.n_wg <= 0)
        return hipSuccess;
    if (p.n_wg > 0x7fffffffLL)
        return hipErrorInvalidConfiguration;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_sse_fp64,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kLdsBudget + 4096));
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_sse_fp64, dim3((unsigned)p.n_wg), dim3(kBlock), lds_bytes, s, p);
    return hipGetLastError();
}

}  // namespace sse
