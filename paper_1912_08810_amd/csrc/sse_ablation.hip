// sse_ablation.hip -- the electron self-energy in the paper's own final form
// (Sec. 4.2: map fission, redundancy removal, data-layout transformation,
// multiplication fusion, map expansion and nested-map substitution), for
// comparison with the reassociated kernel of sse_fp64.hip.  Binary64.
//
// With A_i = dH[a, b, i] and the reading dH_ba,j = A_j^T, Eq. (3) regroups as
//   Sigma[k, e, a] = alpha sum_b sum_i sum_q sum_w M_i[(k - q) mod Nkz, e - s_w] . N_i[q, w]
//   M_i[k', e'] = A_i . G[k', e', f]             (dH G: one Norb x Norb x Nkz NE Norb GEMM
//                                                 per (a, b, i), precomputed)
//   N_i[q, w]   = sum_j Dt[q, w, a, b, i, j] A_j^T   (dH D, precomputed)
// and for each (a, b, i, k, q) the sum over w is one GEMM of the energy window
// of M_i rows (Norb x Norb Nw, Toeplitz in (e, w)) with the stacked N_i[q, :]
// (Norb Nw x Norb): the paper's "N_orb x N_orb N_w x N_orb GEMM".  Here it runs on
// the matrix cores (v_mfma_f64_16x16x4f64), rows (e, m) of TE energies, columns
// (n, re/im), K = (w, l, re/im), accumulated over (b, i, q) in the MFMA
// registers.  The transients M and N live in the caller's workspace, atoms in
// chunks that fit it.  Per (k, e, q, w, a, b) this form costs 8 N3D Norb^3 flops
// where the reassociated kernel costs 8 N3D^2 Norb^2 -- the comparison this
// file exists for.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sse_internal.h"

namespace sse {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// M[al][b][i][k'][e'] = A_i G[k', e', f]: one thread per element (m, l).
__global__ void k_abl_dhg(AblParams p, int a0, int nat)
{
    const int NN = p.NN, No = p.Norb;
    const int64_t n = (int64_t)nat * p.NB * kN3D * p.Nkz * p.NE * NN;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n)
        return;
    const int c = (int)(x % NN);
    int64_t r = x / NN;
    const int e = (int)(r % p.NE);
    r /= p.NE;
    const int k = (int)(r % p.Nkz);
    r /= p.Nkz;
    const int i = (int)(r % kN3D);
    r /= kN3D;
    const int b = (int)(r % p.NB);
    const int a = a0 + (int)(r / p.NB);
    const int m = c / No, l = c - m * No;
    const int f = p.neigh[(size_t)a * p.NB + b];
    double sr = 0.0, si = 0.0;
    if (f >= 0 && f < p.NA) {
        const double *A = p.dH + (((size_t)a * p.NB + b) * kN3D + i) * NN + (size_t)m * No;
        const double2 *G = p.G + (((size_t)k * p.NE + e) * p.NA + f) * NN + l;
        for (int t = 0; t < No; ++t) {
            const double2 g = G[(size_t)t * No];
            sr = fma(A[t], g.x, sr);
            si = fma(A[t], g.y, si);
        }
    }
    p.M[x] = make_double2(sr, si);
}

// N[al][b][i][q][w][l][n] = sum_j Dt[q, w, a, b, i, j] A_j[n][l].
__global__ void k_abl_dhd(AblParams p, int a0, int nat)
{
    const int NN = p.NN, No = p.Norb;
    const int64_t n = (int64_t)nat * p.NB * kN3D * p.Nqz * p.Nw * NN;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n)
        return;
    const int c = (int)(x % NN);
    int64_t r = x / NN;
    const int w = (int)(r % p.Nw);
    r /= p.Nw;
    const int q = (int)(r % p.Nqz);
    r /= p.Nqz;
    const int i = (int)(r % kN3D);
    r /= kN3D;
    const int b = (int)(r % p.NB);
    const int a = a0 + (int)(r / p.NB);
    const int l = c / No, nn = c - l * No;
    const double2 *D = p.D + ((((size_t)q * p.Nw + w) * p.NA + a) * p.NB + b) * kNF + i * kN3D;
    const double *A = p.dH + ((size_t)a * p.NB + b) * kN3D * NN + (size_t)nn * No + l;
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < kN3D; ++j) {
        const double h = A[(size_t)j * NN];
        sr = fma(D[j].x, h, sr);
        si = fma(D[j].y, h, si);
    }
    p.N[x] = make_double2(sr, si);
}

// One workgroup per (atom of the chunk, k, energy tile): 8 waves, wave t owns
// rows 16 t .. 16 t + 15 of the TE Norb (<= 128) rows (e, m) and both column
// tiles of the 2 Norb columns (n, re/im); two waves per SIMD.  Per (b, i, q)
// the window of M_i rows and the stacked N_i[q, :] are staged into LDS in
// ready-made form: the window with a zero row (the padding rows' operand), N_i
// as binary64 rows of 32 columns (n, re/im) with zero padding, so an operand is
// one 8-byte LDS read and, for the imaginary part of M, a sign flip.  A table of
// each K entry's offset into the window (built once) replaces the per-step
// (w, l) arithmetic, so the operands of the next K step can be read while the
// MFMAs of the current one run.
__global__ __launch_bounds__(pik::kAblBlock, 1) void k_abl_gemm(AblParams p, int a0)
{
    extern __shared__ double2 lds[];
    constexpr int ZC = 16 * pik::kAblNT;           // N row: 2 Norb columns, padded
    const int NN = p.NN, No = p.Norb, TE = p.TE;
    const int nrow = p.win_rows;                   // TE + shift spread
    double2 *win = lds;                            // [nrow + 1][NN]: M_i rows, then a zero row
    double *nb = reinterpret_cast<double *>(win + (size_t)(nrow + 1) * NN);  // [Kp + 2][ZC]
    const int Kcount = p.Nw * No;                  // complex K entries (w, l)
    const int Kp = Kcount + (Kcount & 1);
    // A offset (doubles, from a lane's row base) of complex K entry (w, l):
    // ((smax - s_w) NN + l) 2; entries past Kcount are 0 (their N rows are zero)
    int *aoff = reinterpret_cast<int *>(nb + (size_t)(Kp + 2) * ZC);  // [Kp + 4]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    int64_t L = blockIdx.x;
    const int et = (int)(L % p.n_etiles);
    L /= p.n_etiles;
    const int k = (int)(L % p.Nkz);
    const int al = (int)(L / p.Nkz);
    const int a = a0 + al;
    const int e0 = et * TE;
    const int te = min(TE, p.NE - e0);
    for (int x = tid; x < Kp + 4; x += pik::kAblBlock) {
        const int w = x / No, l = x - w * No;
        aoff[x] = x < Kcount ? ((p.smax - p.shift[w]) * NN + l) * 2 : 0;
    }
    for (int x = tid; x < NN; x += pik::kAblBlock)
        win[(size_t)nrow * NN + x] = make_double2(0.0, 0.0);
    for (int x = tid; x < (Kp + 2) * ZC; x += pik::kAblBlock)
        nb[x] = 0.0;

    // this lane's A row (e, m), K' slot and B column
    const int arow = 16 * wave + (lane & 15);
    const bool arow_ok = arow < TE * No;
    const int ae = arow_ok ? arow / No : 0, am = arow_ok ? arow - ae * No : 0;
    const int kq = lane >> 4, xpart = kq & 1, chalf = kq >> 1;
    // A: M window element (row of e - s_w, m, l), part xpart; padding rows read the zero row
    const int abase = arow_ok ? (ae * NN + am * No) * 2 + xpart : nrow * NN * 2;
    const int arow_step = arow_ok ? 1 : 0;       // padding lanes stay on the zero row
    const int *ao = aoff + chalf;                // this lane's K entries: ao[2 s]
    // B: x re reads (N re, N im) for the columns (re, im); x im reads (-N im, N re)
    int bsrc[pik::kAblNT];
    unsigned bsign[pik::kAblNT];
#pragma unroll
    for (int t = 0; t < pik::kAblNT; ++t) {
        const int col = 16 * t + (lane & 15);
        bsrc[t] = xpart ? (col ^ 1) : col;
        bsign[t] = (xpart && !(col & 1)) ? 0x80000000u : 0u;
    }
    v4d acc[pik::kAblNT];
#pragma unroll
    for (int t = 0; t < pik::kAblNT; ++t)
        acc[t] = (v4d){0.0, 0.0, 0.0, 0.0};
    const double *wind = reinterpret_cast<const double *>(win);
    const int nks = Kp >> 1;

    for (int b = 0; b < p.NB; ++b) {
        for (int i = 0; i < kN3D; ++i) {
            for (int q = 0; q < p.Nqz; ++q) {
                int kk = k - q;
                if (kk < 0)
                    kk += p.Nkz;
                __syncthreads();
                const double2 *Mrow = p.M + ((((size_t)al * p.NB + b) * kN3D + i) * p.Nkz + kk) *
                                                (size_t)p.NE * NN;
                const int ebase = e0 - p.smax;
                for (int x = tid; x < nrow * NN; x += pik::kAblBlock) {
                    const int r = x / NN, c = x - r * NN;
                    const int e = ebase + r;
                    win[x] = (e >= 0 && e < p.NE) ? Mrow[(size_t)e * NN + c] : make_double2(0.0, 0.0);
                }
                const double2 *Nq = p.N + ((((size_t)al * p.NB + b) * kN3D + i) * p.Nqz + q) *
                                              (size_t)p.Nw * NN;
                for (int x = tid; x < Kcount * No; x += pik::kAblBlock) {
                    const int kc = x / No, n = x - kc * No;
                    const double2 v = Nq[x];
                    nb[kc * ZC + 2 * n] = v.x;
                    nb[kc * ZC + 2 * n + 1] = v.y;
                }
                __syncthreads();
                // K loop: step s covers complex K entries 2 s and 2 s + 1 = (w, l).
                // The operands of step s + 1 are read while the MFMAs of step s run
                // (past the last step they come from the padding rows and entries)
                int ib = chalf * ZC;
                double a_cur = wind[abase + arow_step * ao[0]];
                double b_cur[pik::kAblNT];
#pragma unroll
                for (int t = 0; t < pik::kAblNT; ++t)
                    b_cur[t] = nb[ib + bsrc[t]];
                int ao_nx = ao[2];
                for (int s = 0; s < nks; ++s) {
                    const int ao_nn = ao[2 * s + 4];
                    const double a_n = wind[abase + arow_step * ao_nx];
                    double b_n[pik::kAblNT];
#pragma unroll
                    for (int t = 0; t < pik::kAblNT; ++t)
                        b_n[t] = nb[ib + 2 * ZC + bsrc[t]];
#pragma unroll
                    for (int t = 0; t < pik::kAblNT; ++t) {
                        const double bv = __hiloint2double(
                            __double2hiint(b_cur[t]) ^ (int)bsign[t], __double2loint(b_cur[t]));
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_cur, bv, acc[t], 0, 0, 0);
                    }
                    a_cur = a_n;
#pragma unroll
                    for (int t = 0; t < pik::kAblNT; ++t)
                        b_cur[t] = b_n[t];
                    ao_nx = ao_nn;
                    ib += 2 * ZC;
                }
            }
        }
    }
    // C tiles -> LDS [row][col] (doubles; value r of a lane is row lane / 16 + 4 r of
    // its tile, column lane % 16), then alpha (re + i im) -> Sigma, coalesced
    __syncthreads();
    double *cs = reinterpret_cast<double *>(lds);
#pragma unroll
    for (int t = 0; t < pik::kAblNT; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            cs[(16 * wave + (lane >> 4) + 4 * r) * ZC + 16 * t + (lane & 15)] = acc[t][r];
    __syncthreads();
    double2 *S = p.Sigma + (((size_t)k * p.NE + e0) * p.NA + a) * NN;
    for (int x = tid; x < te * NN; x += pik::kAblBlock) {
        const int e = x / NN, c = x - e * NN, m = c / No, n = c - m * No;
        const double cr = cs[(e * No + m) * ZC + 2 * n], ci = cs[(e * No + m) * ZC + 2 * n + 1];
        S[(size_t)e * p.NA * NN + c] = make_double2(p.alpha_re * cr - p.alpha_im * ci,
                                                    p.alpha_re * ci + p.alpha_im * cr);
    }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t ablation_launch(const AblParams &p, size_t lds_bytes, int chunk_atoms, hipStream_t s)
{
    static bool done = false;
    if (!done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_abl_gemm,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)pik::kLdsBudgetOne);
        if (e != hipSuccess)
            return e;
        done = true;
    }
    (void)hipGetLastError();
    for (int a0 = 0; a0 < p.NA; a0 += chunk_atoms) {
        const int nat = std::min(chunk_atoms, p.NA - a0);
        const int64_t nm = (int64_t)nat * p.NB * kN3D * p.Nkz * p.NE * p.NN;
        const int64_t nn = (int64_t)nat * p.NB * kN3D * p.Nqz * p.Nw * p.NN;
        hipLaunchKernelGGL(k_abl_dhg, dim3(nblk(nm)), dim3(256), 0, s, p, a0, nat);
        hipLaunchKernelGGL(k_abl_dhd, dim3(nblk(nn)), dim3(256), 0, s, p, a0, nat);
        const int64_t nwg = (int64_t)nat * p.Nkz * p.n_etiles;
        hipLaunchKernelGGL(k_abl_gemm, dim3((unsigned)nwg), dim3(pik::kAblBlock), lds_bytes, s, p,
                           a0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace sse
