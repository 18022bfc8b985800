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
#include "sse_copy.h"

namespace sse {

namespace {

constexpr int kBlock = fp64k::kBlock;
constexpr int kR = fp64k::kR;
constexpr size_t kLdsBudget = fp64k::kLdsBudget;

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

// One tap's update of the nine filter accumulators of one position.  General
// D~: acc_x += D~_x g for the nine (i, j).  Anti-Hermitian D~ (D~_ji =
// -conj(D~_ij), so D~_ii = i Im D~_ii): slot ij (i < j) gathers U_ij += Re D~_ij g,
// slot ji gathers V_ij += Im D~_ij g, and slot ii gathers V_ii += Im D~_ii g
// -- 18 instead of 36 FMAs; ah_finish turns them into Gh_ij = U + iV,
// Gh_ji = -U + iV, Gh_ii = i V.
template <bool AH>
__device__ __forceinline__ void tap_update(double (&ar)[kNF], double (&ai)[kNF],
                                           const double2 (&d)[kNF], double2 g)
{
    if constexpr (!AH) {
#pragma unroll
        for (int x = 0; x < kNF; ++x)
            cmac(ar[x], ai[x], d[x].x, d[x].y, g.x, g.y);
    } else {
        constexpr int up[3] = {1, 2, 5}, lo[3] = {3, 6, 7}, dg[3] = {0, 4, 8};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ar[up[k]] = fma(d[up[k]].x, g.x, ar[up[k]]);
            ai[up[k]] = fma(d[up[k]].x, g.y, ai[up[k]]);
            ar[lo[k]] = fma(d[up[k]].y, g.x, ar[lo[k]]);
            ai[lo[k]] = fma(d[up[k]].y, g.y, ai[lo[k]]);
            ar[dg[k]] = fma(d[dg[k]].y, g.x, ar[dg[k]]);
            ai[dg[k]] = fma(d[dg[k]].y, g.y, ai[dg[k]]);
        }
    }
}

// Anti-Hermitian mode: (U, V) accumulators -> the nine filtered blocks.
__device__ __forceinline__ void ah_finish(double (&ar)[kNF], double (&ai)[kNF])
{
    constexpr int up[3] = {1, 2, 5}, lo[3] = {3, 6, 7}, dg[3] = {0, 4, 8};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double ur = ar[up[k]], ui = ai[up[k]], vr = ar[lo[k]], vi = ai[lo[k]];
        ar[up[k]] = ur - vi;
        ai[up[k]] = ui + vr;
        ar[lo[k]] = -ur - vi;
        ai[lo[k]] = -ui + vr;
        const double wr = ar[dg[k]], wi = ai[dg[k]];
        ar[dg[k]] = -wi;
        ai[dg[k]] = wr;
    }
}

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return make_double2(v.x, v.y); }
template <typename T> __device__ __forceinline__ T from_d2(double x, double y);
template <> __device__ __forceinline__ double2 from_d2<double2>(double x, double y)
{
    return make_double2(x, y);
}
template <> __device__ __forceinline__ float2 from_d2<float2>(double x, double y)
{
    return make_float2((float)x, (float)y);
}

// Zero source of the window copies (rows outside the energy grid).
__device__ __attribute__((aligned(16))) uint32_t g_zero16[4] = {0u, 0u, 0u, 0u};

// One output tile: energies [et TE, et TE + TE) of (k, a).  pp supplies the
// problem's sizes and tap table (a kernel argument or a batch table in global
// memory), ptr its tensors.
// T is the storage type of G, D~ and Sigma (complex128, or complex64 promoted to
// binary64 on load); all arithmetic is binary64.
template <typename T, bool AH>
__device__ __forceinline__ void fp64_tile(const_ptr<Fp64Params> pp, const TensorPtrs &ptr, int a,
                                          int k, int et, double2 *lds)
{
    const auto &p = *pp;
    double *ldsA = reinterpret_cast<double *>(lds + p.lds_win);
    const int e0 = et * p.TE;
    const int te = min(p.TE, p.NE - e0);
    const int NN = p.NN, No = p.Norb;
    const int P = te * NN;
    const int Pst = p.TE * NN;  // scratch stride between the three filters of a round
    const int tid = threadIdx.x;
    // Thread tid owns positions tid + 256 r.  Positions at or beyond P are
    // computed from in-bounds LDS (the window region is padded to 1024 +
    // spread) and never stored.

    double sr[kR], si[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        sr[r] = 0.0;
        si[r] = 0.0;
    }

    const size_t strideD = (size_t)p.NA * p.NB * kNF;  // one (q, w) slab of D~
    const size_t strideE = (size_t)p.NA * NN;          // one energy row of G
    // staging walk: element idx = tid + 256 it is (energy ew, channel cc)
    // small_div: exact quotients of small integers without the GPU's long
    // integer-division sequence
    const float rNN = 1.0f / (float)NN, rNo = 1.0f / (float)No;
    const int st_e = small_div(kBlock, NN, rNN), st_c = kBlock - st_e * NN;
    const int ew0 = small_div(tid, NN, rNN), cc0 = tid - ew0 * NN;

    for (int b = 0; b < p.NB; ++b) {
        const int f = ro(ptr.neigh)[(size_t)a * p.NB + b];
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

        const_ptr<T> Dab = ro((const T *)ptr.D) + ((size_t)a * p.NB + b) * kNF;
        for (int q = 0; q < p.Nqz; ++q) {
            int kk = k - q;
            if (kk < 0)
                kk += p.Nkz;
            const T *Gk = (const T *)ptr.G + (size_t)kk * p.NE * strideE + (size_t)f * NN;
            const_ptr<T> Dq = Dab + (size_t)q * p.Nw * strideD;
            for (int c = 0; c < p.taps.nchunk; ++c) {
                const int t0 = p.taps.cb[c], t1 = p.taps.cb[c + 1];
                const int smax = p.taps.s[t0], smin = p.taps.s[t1 - 1];
                const int wn = (te + smax - smin) * NN;
                const int ebase = e0 - smax;
                __syncthreads();
                if constexpr (sizeof(T) == sizeof(double2)) {
                    // complex128: the copy engine moves the rows straight into
                    // LDS (16-byte units, rows outside the energy grid from a
                    // zero block); the barrier below waits for it
                    copy_window<4, kBlock>(reinterpret_cast<uint32_t *>(lds),
                                           reinterpret_cast<const uint32_t *>(Gk),
                                           (int64_t)strideE * 4, ebase, p.NE, te + smax - smin,
                                           NN * 4, g_zero16);
                } else {
                    // complex64: promoted to binary64 on the way
                    int ew = ew0, cc = cc0;
                    for (int idx = tid; idx < wn; idx += kBlock) {
                        const int e = ebase + ew;
                        double2 v = make_double2(0.0, 0.0);
                        if (e >= 0 && e < p.NE)
                            v = to_d2(Gk[(size_t)e * strideE + cc]);
                        lds[idx] = v;
                        cc += st_c;
                        ew += st_e;
                        if (cc >= NN) {
                            cc -= NN;
                            ++ew;
                        }
                    }
                }
                __syncthreads();
                int t = t0;
                if constexpr (sizeof(T) == sizeof(double2)) {
                    // complex128: one tap at a time, its D~ (scalar loads) fetched
                    // during the previous tap.  Scalar and LDS loads share one
                    // wait counter and scalar loads complete out of order, so a
                    // wait for window reads also waits for every scalar load in
                    // flight; each tap therefore waits once (its window reads and
                    // its D~, issued a tap earlier), then issues the next tap's
                    // D~ before its 36 FMAs per position.  The scheduling barriers
                    // keep the compiler from hoisting those loads above the wait.
                    double2 dA[kNF], dB[kNF];
                    int sh = p.tws[2 * t + 1], wn = p.tws[2 * t + 2];
                    {
                        const_ptr<T> dp = Dq + (size_t)p.tws[2 * t] * strideD;
#pragma unroll
                        for (int x = 0; x < kNF; ++x)
                            dA[x] = to_d2(dp[x]);
                    }
                    // tap t from cur while the D~ of tap t + 1 is fetched into nxt
                    // (the table is padded, so the last tap fetches a valid block)
                    auto step = [&](double2(&cur)[kNF], double2(&nxt)[kNF]) {
                        const double2 *wp = lds + tid + (smax - sh) * NN;
                        double2 g[kR];
#pragma unroll
                        for (int r = 0; r < kR; ++r)
                            g[r] = wp[r * kBlock];
                        const int sh2 = p.tws[2 * t + 3], wn2 = p.tws[2 * t + 4];
                        __builtin_amdgcn_sched_barrier(0);
                        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
                        __builtin_amdgcn_sched_barrier(0);
                        {
                            const_ptr<T> dp = Dq + (size_t)wn * strideD;
#pragma unroll
                            for (int x = 0; x < kNF; ++x)
                                nxt[x] = to_d2(dp[x]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int r = 0; r < kR; ++r)
                            tap_update<AH>(ar[r], ai[r], cur, g[r]);
                        sh = sh2;
                        wn = wn2;
                        ++t;
                    };
                    while (t + 1 < t1) {
                        step(dA, dB);
                        step(dB, dA);
                    }
                    if (t < t1)
                        step(dA, dB);
                }
                if constexpr (sizeof(T) != sizeof(double2)) {
                    // complex64: the same pipeline, the D~ in flight held as
                    // complex64 (scalar registers) and promoted where it is used
                    T fA[kNF], fB[kNF];
                    int sh = p.tws[2 * t + 1], wn = p.tws[2 * t + 2];
                    {
                        const_ptr<T> dp = Dq + (size_t)p.tws[2 * t] * strideD;
#pragma unroll
                        for (int x = 0; x < kNF; ++x)
                            fA[x] = dp[x];
                    }
                    auto step = [&](T(&cur)[kNF], T(&nxt)[kNF]) {
                        const double2 *wp = lds + tid + (smax - sh) * NN;
                        double2 g[kR];
#pragma unroll
                        for (int r = 0; r < kR; ++r)
                            g[r] = wp[r * kBlock];
                        const int sh2 = p.tws[2 * t + 3], wn2 = p.tws[2 * t + 4];
                        __builtin_amdgcn_sched_barrier(0);
                        __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
                        __builtin_amdgcn_sched_barrier(0);
                        {
                            const_ptr<T> dp = Dq + (size_t)wn * strideD;
#pragma unroll
                            for (int x = 0; x < kNF; ++x)
                                nxt[x] = dp[x];
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        double2 d[kNF];
#pragma unroll
                        for (int x = 0; x < kNF; ++x)
                            d[x] = to_d2(cur[x]);
#pragma unroll
                        for (int r = 0; r < kR; ++r)
                            tap_update<AH>(ar[r], ai[r], d, g[r]);
                        sh = sh2;
                        wn = wn2;
                        ++t;
                    };
                    while (t + 1 < t1) {
                        step(fA, fB);
                        step(fB, fA);
                    }
                    if (t < t1)
                        step(fA, fB);
                }
            }
        }

        if constexpr (AH) {
#pragma unroll
            for (int r = 0; r < kR; ++r)
                ah_finish(ar[r], ai[r]);
        }
        // ---- sandwich: Sigma += sum_ij dH_i Gh_ij dH_j^T for this neighbour
        __syncthreads();  // window reads done; LDS becomes scratch
        const double *Ag = ptr.dH + ((size_t)a * p.NB + b) * kN3D * NN;
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
                if (tid + r * kBlock < P)
#pragma unroll
                    for (int j = 0; j < kN3D; ++j)
                        lds[j * Pst + tid + r * kBlock] =
                            make_double2(ar[r][i * kN3D + j], ai[r][i * kN3D + j]);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kR; ++r) {
                const int pos = tid + r * kBlock < P ? tid + r * kBlock : 0;
                const int el = small_div(pos, NN, rNN), cpos = pos - el * NN;
                const int m = small_div(cpos, No, rNo), n = cpos - m * No;
                const int base = el * NN + n;
                const double *Arow = ldsA + i * NN + m * No;
                // unrolled explicitly: inlined into the persistent kernel's
                // loop the compiler's own heuristics leave it rolled
#pragma unroll 4
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
            if (tid + r * kBlock < P)
#pragma unroll
                for (int j = 0; j < kN3D; ++j)
                    lds[j * Pst + tid + r * kBlock] = make_double2(tr[r][j], ti[r][j]);
        __syncthreads();
        // Sigma_mn += sum_j sum_l T_j[m, l] dH_j[n, l]
#pragma unroll
        for (int r = 0; r < kR; ++r) {
            const int pos = tid + r * kBlock < P ? tid + r * kBlock : 0;
            const int el = small_div(pos, NN, rNN), cpos = pos - el * NN;
            const int m = small_div(cpos, No, rNo), n = cpos - m * No;
            const int base = el * NN + m * No;
#pragma unroll
            for (int j = 0; j < kN3D; ++j) {
                const double *Arow = ldsA + j * NN + n * No;
#pragma unroll 8
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
    T *Sk = (T *)ptr.Sigma + ((size_t)k * p.NE + e0) * strideE + (size_t)a * NN;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int pos = tid + r * kBlock;
        if (pos >= P)
            continue;
        const int el = small_div(pos, NN, rNN);
        const int c = pos - el * NN;
        Sk[(size_t)el * strideE + c] = from_d2<T>(p.alpha_re * sr[r] - p.alpha_im * si[r],
                                                 p.alpha_re * si[r] + p.alpha_im * sr[r]);
    }
}

template <typename T, bool AH>
__global__ __launch_bounds__(kBlock, 2) void k_sse_fp64(const Fp64Params p)
{
    extern __shared__ double2 lds[];
    int64_t L = xcd_remap(blockIdx.x, p.n_wg);
    const int k = (int)(L % p.Nkz);
    L /= p.Nkz;
    const int et = (int)(L % p.n_etiles);
    const int a = (int)(L / p.n_etiles);
    const TensorPtrs ptr{p.neigh, p.dH, p.G, p.D, p.Sigma};
    fp64_tile<T, AH>(ro(&p), ptr, a, k, et, lds);
}

// Persistent form: a fixed grid pulls tiles from the batch's work queues
// (one queue per XCD, then the others) until all are taken; the next tile's
// ticket is taken while the current tile runs.
template <typename T, bool AH>
__global__ __launch_bounds__(kBlock, 2) void k_sse_fp64_persistent(const BatchLaunch bl)
{
    extern __shared__ double2 lds[];
    __shared__ int s_tile[4], s_st[2];
    const int home = blockIdx.x & 7;
    if (threadIdx.x == 0)
        pull_first(bl, home, s_st, s_tile);
    __syncthreads();
    for (;;) {
        const int inst = __builtin_amdgcn_readfirstlane(s_tile[0]);
        const int a = __builtin_amdgcn_readfirstlane(s_tile[1]);
        const int k = __builtin_amdgcn_readfirstlane(s_tile[2]);
        const int et = __builtin_amdgcn_readfirstlane(s_tile[3]);
        __syncthreads();
        if (inst < 0)
            break;
        long long ticket = 0;
        if (threadIdx.x == 0)
            ticket = pull_take(bl, home, s_st);
        fp64_tile<T, AH>(ro(reinterpret_cast<const Fp64Params *>(bl.params)) + inst,
                         bl.ptr[inst], a, k, et, lds);
        if (threadIdx.x == 0)
            pull_resolve(bl, home, ticket, s_st, s_tile);
        __syncthreads();
    }
}

}  // namespace

template <typename K>
static hipError_t set_lds_attr(K kernel, bool &done)
{
    if (done)
        return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void *)kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kLdsBudget + 4096));
    done = e == hipSuccess;
    return e;
}

template <typename T, bool AH>
static hipError_t persistent_launch_as(const BatchLaunch &bl, int grid, size_t lds_bytes,
                                       hipStream_t s)
{
    static bool done = false;
    hipError_t e = set_lds_attr(k_sse_fp64_persistent<T, AH>, done);
    if (e != hipSuccess)
        return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL((k_sse_fp64_persistent<T, AH>), dim3(grid), dim3(kBlock), lds_bytes, s, bl);
    return hipGetLastError();
}

hipError_t fp64_persistent_launch(const BatchLaunch &bl, bool c64, bool ah, int grid,
                                  size_t lds_bytes, hipStream_t s)
{
    if (c64)
        return ah ? persistent_launch_as<float2, true>(bl, grid, lds_bytes, s)
                  : persistent_launch_as<float2, false>(bl, grid, lds_bytes, s);
    return ah ? persistent_launch_as<double2, true>(bl, grid, lds_bytes, s)
              : persistent_launch_as<double2, false>(bl, grid, lds_bytes, s);
}

template <typename T, bool AH>
static hipError_t launch_as(const Fp64Params &p, size_t lds_bytes, hipStream_t s)
{
    static bool done = false;
    hipError_t e = set_lds_attr(k_sse_fp64<T, AH>, done);
    if (e != hipSuccess)
        return e;
    (void)hipGetLastError();
    hipLaunchKernelGGL((k_sse_fp64<T, AH>), dim3((unsigned)p.n_wg), dim3(kBlock), lds_bytes, s, p);
    return hipGetLastError();
}

hipError_t fp64_launch(const Fp64Params &p, bool c64, bool ah, size_t lds_bytes, hipStream_t s)
{
    if (p.n_wg <= 0)
        return hipSuccess;
    if (p.n_wg > 0x7fffffffLL)
        return hipErrorInvalidConfiguration;
    if (c64)
        return ah ? launch_as<float2, true>(p, lds_bytes, s) : launch_as<float2, false>(p, lds_bytes, s);
    return ah ? launch_as<double2, true>(p, lds_bytes, s) : launch_as<double2, false>(p, lds_bytes, s);
}

}  // namespace sse
