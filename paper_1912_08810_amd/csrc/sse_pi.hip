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
// the two Norb x Norb products run once per (k, e) of a workgroup (not once per
// frequency), and each frequency costs one complex multiply-add per orbital pair
// and (i, j) -- the (q, w) correlation that Sec. 4.2 turns into one GEMM, here
// without any Norb x Norb product inside it.
//
// The correlation is a GEMM on the matrix cores (v_mfma_f64_16x16x4f64):
// rows = the frequencies (taps) of a chunk, columns = (b, i, j, re/im) for the
// nbw neighbours of the workgroup, K = (orbital pair, re/im of X), summed over
// every (k, e).  A = X rows, read from a ring of atom a's rows in LDS (a tap is
// an offset into it); B = Zt in LDS, the complex product folded into the
// operand's sign and part.  One workgroup (8 waves) per (atom a, momentum q,
// group of nbw neighbours, tap chunk) walks k, then e one energy per step; the
// eight waves split the step's K range, each holding every output tile in its
// matrix-core accumulators, and the eight partial sums are added in a fixed
// order at the end.  The nbw neighbours' blocks Y[k, e, f] are sandwiched into
// Zt on the vector units in two rounds of Norb-long dot products through LDS,
// pipelined over the energy steps: while the MFMAs of step e run, each wave
// computes the second round of step e + 1 for exactly the Zt rows its own MFMAs
// read (interleaved with them, so the vector and matrix units work together,
// and no barrier guards Zt); the first round of step e + 2 follows between two
// barriers.  The ring holds one row more than a step reads, so the next step's
// top row is written while the MFMAs read the others.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sse_internal.h"

namespace sse {

namespace {

constexpr int kBlock = pik::kBlock;
constexpr int kS2Terms = 2;  // second-round m terms per MFMA step of the interleave
typedef double v4d __attribute__((ext_vector_type(4)));

// Logical workgroup of physical workgroup `bid`: workgroups are dispatched
// round-robin over the 8 XCDs, so give each XCD a contiguous range of logical
// indices (the q, neighbour-group and chunk workgroups of one atom, which read
// the same rows of its G, share an L2).
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

// Per-thread offsets of the two sandwich rounds and of the Y staging; a
// thread's tasks are the same at every step (at most two each, since
// nbw Norb^2 <= 1024 = 2 kBlock), so their index arithmetic is done once.
// Every loop over a thread's tasks runs over the constant bound 2 with a
// guard: an array indexed by a run-time value would be placed in private
// (scratch) memory and reloaded from it at every step.
struct SandwichTasks {
    int n1, n2, ny;                 // tasks of the first and second rounds, staged Y elements
    int h1[2], y1[2], o1[2];        // first round: dH row, Y column, U output
    int h2[2], u2[2], o2[2];        // second round: dH rows, U rows, Zb output (double index)
    int ys[2], yg[2];               // Y staging: LDS slot, element offset in a G energy row (-1: zero)
};

// First sandwich round: U[b][j][p][m] = sum_r dH_bj[p][r] Y_b[r][m]; a task is
// one (b, p, m) for all three j, sharing the loads of Y's column.
__device__ __forceinline__ void sandwich_first(const SandwichTasks &T, const double *dHs,
                                               const double2 *Ys, double2 *Us, int NN, int No)
{
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        if (u >= T.n1)
            break;
        const double *h = dHs + T.h1[u];
        const double2 *y = Ys + T.y1[u];
        double ur[3] = {0.0, 0.0, 0.0}, ui[3] = {0.0, 0.0, 0.0};
#pragma unroll 5
        for (int r = 0; r < No; ++r) {
            const double2 v = y[r * No];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double hj = h[j * NN + r];
                ur[j] = fma(hj, v.x, ur[j]);
                ui[j] = fma(hj, v.y, ui[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Us[T.o1[u] + j * NN] = make_double2(ur[j], ui[j]);
    }
}

// Second round: Zt_bij[n][p] = sum_m dH_bi[n][m] U[b][j][p][m] into the column
// pair 2 (9 b + 3 i + j) + (re, im) of row c = n Norb + p of Zb (the orbital pair
// of X it multiplies); a task is one (c, b) for all nine (i, j), sharing the
// loads of the three dH rows and the three U rows.  The rows of Zb a wave
// computes are the rows its own MFMA steps read, so Zb needs no barrier: one
// m term of task u is added into (zr, zi) per call.
__device__ __forceinline__ void sandwich_second_term(const SandwichTasks &T, int u, int m,
                                                     const double *dHs, const double2 *Us,
                                                     int NN, double (&zr)[kNF],
                                                     double (&zi)[kNF])
{
    const double *h = dHs + T.h2[u];
    const double2 *us = Us + T.u2[u];
    double hi[3];
    double2 uj[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        hi[t] = h[t * NN + m];
        uj[t] = us[t * NN + m];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            zr[3 * i + j] = fma(hi[i], uj[j].x, zr[3 * i + j]);
            zi[3 * i + j] = fma(hi[i], uj[j].y, zi[3 * i + j]);
        }
}

__device__ __forceinline__ void sandwich_second_store(const SandwichTasks &T, int u, double *Zb,
                                                      const double (&zr)[kNF],
                                                      const double (&zi)[kNF])
{
    if (T.o2[u] < 0)
        return;
    double2 *out = reinterpret_cast<double2 *>(Zb + T.o2[u]);
#pragma unroll
    for (int x = 0; x < kNF; ++x)
        out[x] = make_double2(zr[x], zi[x]);
}

// Task u of the second round in full (every m term, then the store).
__device__ __forceinline__ void sandwich_second(const SandwichTasks &T, int u, const double *dHs,
                                                const double2 *Us, double *Zb, int NN, int No)
{
    double zr[kNF], zi[kNF];
#pragma unroll
    for (int x = 0; x < kNF; ++x)
        zr[x] = zi[x] = 0.0;
#pragma unroll 1
    for (int m = 0; m < No; ++m)
        sandwich_second_term(T, u, m, dHs, Us, NN, zr, zi);
    sandwich_second_store(T, u, Zb, zr, zi);
}

template <int MT, int NTN>
__global__ __launch_bounds__(kBlock, 1) void k_pi_mfma(const PiParams p)
{
    extern __shared__ double2 lds[];
    constexpr int ZC = 16 * NTN;                  // Zb row: 2 (b, i, j) columns, padded
    const int NN = p.NN, No = p.Norb, R = p.R, nbw = p.nbw;
    const int NNp = NN + (NN & 1);                // orbital pairs padded to an even count
    // ring slots: the R rows a step reads plus one, so that the next step's top
    // row can be written while a step's MFMAs read the others
    const int RS = R + 1;
    double2 *ring = lds;                          // [RS + 1][NNp]; row RS and pair NN are zero
    double *Zb = reinterpret_cast<double *>(ring + (size_t)(RS + 1) * NNp);  // [NNp][ZC]
    double2 *Us = reinterpret_cast<double2 *>(Zb + (size_t)NNp * ZC);     // [nbw 3][NN]
    double2 *Ys = Us + (size_t)nbw * 3 * NN;      // [nbw][NN]
    double *dHs = reinterpret_cast<double *>(Ys + (size_t)nbw * NN);  // [nbw 3][NN]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    int64_t L = xcd_logical(blockIdx.x, p.n_wg);
    const int chunk = (int)(L % p.nchunk);
    L /= p.nchunk;
    const int bg = (int)(L % p.nbgroups);
    L /= p.nbgroups;
    const int q = (int)(L % p.Nqz);
    const int a = (int)(L / p.Nqz);
    const int b0 = bg * nbw;
    const int nbv = min(nbw, p.NB - b0);          // neighbours of this workgroup
    const int t0 = p.cb[chunk], t1 = p.cb[chunk + 1];
    const int s_lo = p.ts[t0], s_hi = p.ts[t1 - 1];

    for (int x = tid; x < nbw * 3 * NN; x += kBlock) {
        const int b = x / (3 * NN);
        dHs[x] = b < nbv ? p.dH[((size_t)a * p.NB + b0) * 3 * NN + x] : 0.0;
    }
    // zero once: the ring's zero row and padding pair, Zb's padding row and columns
    for (int x = tid; x < (RS + 1) * NNp; x += kBlock)
        ring[x] = make_double2(0.0, 0.0);
    for (int x = tid; x < NNp * ZC; x += kBlock)
        Zb[x] = 0.0;

    SandwichTasks T;
    T.n1 = T.n2 = T.ny = 0;
    // first-round tasks dealt evenly over the eight waves (the two waves of a SIMD
    // then carry the same number): wave w takes tasks [w per, (w + 1) per)
    const int per_wave = (nbw * NN + pik::kWaves - 1) / pik::kWaves;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int lo = lane + 64 * u;
        const int o = wave * per_wave + lo;
        if (lo < per_wave && o < nbw * NN) {
            // first round and Y staging: o = (b, p, m)
            const int b = o / NN, rem = o - b * NN, r0 = rem / No, m = rem - r0 * No;
            T.h1[u] = b * 3 * NN + r0 * No;
            T.y1[u] = b * NN + m;
            T.o1[u] = b * 3 * NN + rem;
            T.n1 = u + 1;
            const int f = b < nbv ? p.neigh[(size_t)a * p.NB + b0 + b] : -1;
            T.ys[u] = o;
            T.yg[u] = (f >= 0 && f < p.NA) ? f * NN + rem : -1;
            T.ny = u + 1;
        }
        // second round: task t = lane + 64 u of this wave is (row i / nbw of the wave's
        // rows c = 16 (i / 2) + 2 wave + i % 2, neighbour i % nbw); lanes past the
        // wave's tasks compute on row 0 and store nothing
        const int t = lane + 64 * u, ri = t / nbw, b2 = t - ri * nbw;
        const int c = 16 * (ri >> 1) + 2 * wave + (ri & 1);
        const bool ok = c < NN;
        const int n = ok ? c / No : 0, r2 = ok ? c - n * No : 0;
        T.h2[u] = b2 * 3 * NN + n * No;
        T.u2[u] = b2 * 3 * NN + r2 * No;
        T.o2[u] = ok ? c * ZC + 2 * kNF * b2 : -1;
    }
    // tasks of the second round per lane: 2 where some lane of the wave has a second one
    T.n2 = __ballot(T.o2[1] >= 0) != 0 ? 2 : 1;

    // per lane: its tap row in each row tile, its K' slot, its columns
    const int kq = lane >> 4, xpart = kq & 1, chalf = kq >> 1;
    int tap_s[MT];
    bool tap_ok[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int t = t0 + 16 * mt + (lane & 15);
        tap_ok[mt] = t < t1;
        tap_s[mt] = tap_ok[mt] ? p.ts[t] : s_lo;
    }
    // B operand: x re reads (Z re, Z im) for the columns (re, im); x im reads
    // (-Z im, Z re), the neighbouring column of the pair with a sign (applied
    // by flipping the sign bit)
    int bsrc[NTN];
    unsigned bsign[NTN];
#pragma unroll
    for (int nt = 0; nt < NTN; ++nt) {
        const int col = 16 * nt + (lane & 15);
        bsrc[nt] = xpart ? (col ^ 1) : col;
        bsign[nt] = (xpart && !(col & 1)) ? 0x80000000u : 0u;
    }
    v4d acc[MT][NTN];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTN; ++nt)
            acc[mt][nt] = (v4d){0.0, 0.0, 0.0, 0.0};

    const size_t row_stride = (size_t)p.NA * NN;  // one energy step of G
    const int nks = NNp >> 1;                     // MFMA steps (two orbital pairs each) per energy
    const double *ringd = reinterpret_cast<const double *>(ring);

    for (int k = 0; k < p.Nkz; ++k) {
        const int kx = (k + q) % p.Nkz;
        const double2 *Xk = p.X + ((size_t)kx * p.NE * p.NA + a) * NN;
        const double2 *Yk = p.Y + (size_t)k * p.NE * row_stride;
        __syncthreads();  // the previous k's last step is done with the ring, Us and Ys
        // ring rows s_lo .. s_hi (step 0's rows); Y of step 0
        for (int x = tid; x < (s_hi - s_lo + 1) * NN; x += kBlock) {
            const int row = s_lo + x / NN, c = x % NN;
            ring[ring_slot(row, RS) * NNp + c] = (row >= 0 && row < p.NE)
                                                      ? Xk[(size_t)row * row_stride + c]
                                                      : make_double2(0.0, 0.0);
        }
        // Rows in flight: Y elements of a later step (two scalars: an array
        // element written under a branch put the array in private memory) and the
        // ring's next top row.  Every step first stores the rows in flight to LDS
        // and only then requests the next ones, so that no LDS store waits for a
        // global load issued in the same step (the vector-memory counter is
        // waited in order).
        auto load_y = [&](int u, int e) {
            return (u < T.ny && T.yg[u] >= 0 && e < p.NE)
                       ? Yk[(size_t)e * row_stride + T.yg[u]]
                       : make_double2(0.0, 0.0);
        };
        auto put_y = [&](int u, double2 v) {
            if (u < T.ny)
                Ys[T.ys[u]] = v;
        };
        auto load_x = [&](int row) {
            return (tid < NN && row >= 0 && row < p.NE) ? Xk[(size_t)row * row_stride + tid]
                                                        : make_double2(0.0, 0.0);
        };
        put_y(0, load_y(0, 0));
        put_y(1, load_y(1, 0));
        double2 yv0 = load_y(0, 1), yv1 = load_y(1, 1), xv = load_x(1 + s_hi);
        __syncthreads();
        sandwich_first(T, dHs, Ys, Us, NN, No);   // U of step 0
        __syncthreads();
        // Zt of step 0 (each wave its own rows); Y of step 1 to LDS
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (u < T.n2)
                sandwich_second(T, u, dHs, Us, Zb, NN, No);
        if (1 < p.NE) {
            put_y(0, yv0);
            put_y(1, yv1);
        }
        yv0 = load_y(0, 2);
        yv1 = load_y(1, 2);
        __syncthreads();
        if (1 < p.NE)
            sandwich_first(T, dHs, Ys, Us, NN, No);   // U of step 1
        __syncthreads();
        for (int es = 0; es < p.NE; ++es) {
            // ---- phase A: the MFMAs of step es (this wave's share of the orbital
            // pairs), with the second sandwich round of step es + 1 for the Zb rows
            // those MFMAs read interleaved (the vector units work while the matrix
            // cores run); the ring's top row of step es + 1 and Y of step es + 2 go
            // to LDS, the next rows load
            const bool next = es + 1 < p.NE;
            int ia[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                ia[mt] = ((tap_ok[mt] ? ring_slot(es + tap_s[mt], RS) : RS) * NNp +
                          2 * wave + chalf) * 2 + xpart;
            int ib = (2 * wave + chalf) * ZC;
            constexpr int da = 4 * pik::kWaves;   // doubles between a lane's A operands
            const int db = 2 * pik::kWaves * ZC;
            double zr[kNF], zi[kNF];
#pragma unroll
            for (int x = 0; x < kNF; ++x)
                zr[x] = zi[x] = 0.0;
            int m2 = 0;
            for (int s = wave; s < nks; s += pik::kWaves) {
                double av[MT], bv[NTN];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    av[mt] = ringd[ia[mt]];
#pragma unroll
                for (int nt = 0; nt < NTN; ++nt)
                    bv[nt] = __hiloint2double(__double2hiint(Zb[ib + bsrc[nt]]) ^ (int)bsign[nt],
                                              __double2loint(Zb[ib + bsrc[nt]]));
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NTN; ++nt)
                        acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt],
                                                                           acc[mt][nt], 0, 0, 0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    ia[mt] += da;
                ib += db;
                if (next) {
#pragma unroll
                    for (int v = 0; v < kS2Terms; ++v)
                        if (m2 + v < No)
                            sandwich_second_term(T, 0, m2 + v, dHs, Us, NN, zr, zi);
                    m2 += kS2Terms;
                }
            }
            if (next) {
                // this wave's MFMA reads of step es are issued: its Zb rows take step
                // es + 1 (LDS operations of a wave complete in order)
#pragma unroll 1
                for (; m2 < No; ++m2)
                    sandwich_second_term(T, 0, m2, dHs, Us, NN, zr, zi);
                sandwich_second_store(T, 0, Zb, zr, zi);
                if (T.n2 > 1)
                    sandwich_second(T, 1, dHs, Us, Zb, NN, No);
                if (tid < NN)
                    ring[ring_slot(es + 1 + s_hi, RS) * NNp + tid] = xv;
                if (es + 2 < p.NE) {
                    put_y(0, yv0);
                    put_y(1, yv1);
                }
                xv = load_x(es + 2 + s_hi);
                yv0 = load_y(0, es + 3);
                yv1 = load_y(1, es + 3);
            }
            __syncthreads();
            // ---- phase B: the first sandwich round of step es + 2
            if (es + 2 < p.NE) {
                sandwich_first(T, dHs, Ys, Us, NN, No);
                __syncthreads();
            }
        }
    }

    // ---- the waves' partial sums in a fixed order: wave w + 4 is added into
    // wave w, then the four sums are added in wave order; then beta * P.  An
    // MFMA accumulator holds, for lane l, rows l / 16 + 4 r of its tile at
    // column l % 16.
    constexpr int kHalf = pik::kWaves / 2;
    double *red = reinterpret_cast<double *>(lds);  // [kHalf waves][16 MT][16 NTN]
    const int rows = 16 * MT, cols = 16 * NTN;
    auto at = [&](int v, int mt, int nt, int r) -> double & {
        return red[((size_t)v * rows + 16 * mt + (lane >> 4) + 4 * r) * cols + 16 * nt +
                   (lane & 15)];
    };
    __syncthreads();
    if (wave >= kHalf) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NTN; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    at(wave - kHalf, mt, nt, r) = acc[mt][nt][r];
    }
    __syncthreads();
    if (wave < kHalf) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NTN; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[mt][nt][r] += at(wave, mt, nt, r);
    }
    __syncthreads();
    if (wave < kHalf) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NTN; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    at(wave, mt, nt, r) = acc[mt][nt][r];
    }
    __syncthreads();
    const size_t qw_stride = (size_t)p.NA * (p.NB + 1) * kNF;
    for (int x = tid; x < (t1 - t0) * nbv * kNF; x += kBlock) {
        const int tt = x / (nbv * kNF), bij = x - tt * (nbv * kNF);
        double sr = 0.0, si = 0.0;
        for (int v = 0; v < kHalf; ++v) {
            sr += red[((size_t)v * rows + tt) * cols + 2 * bij];
            si += red[((size_t)v * rows + tt) * cols + 2 * bij + 1];
        }
        const int b = b0 + bij / kNF, ij = bij % kNF;
        p.Pi[((size_t)q * p.Nw + p.tw[t0 + tt]) * qw_stride + ((size_t)a * (p.NB + 1) + b) * kNF +
             ij] = make_double2(p.beta_re * sr - p.beta_im * si, p.beta_re * si + p.beta_im * sr);
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

template <int MT, int NTN>
hipError_t launch_as(const PiParams &p, size_t lds_bytes, hipStream_t s)
{
    static bool done = false;
    if (!done) {
        hipError_t e = hipFuncSetAttribute((const void *)k_pi_mfma<MT, NTN>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)pik::kLdsBudgetOne);
        if (e != hipSuccess)
            return e;
        done = true;
    }
    (void)hipGetLastError();
    hipLaunchKernelGGL((k_pi_mfma<MT, NTN>), dim3((unsigned)p.n_wg), dim3(kBlock), lds_bytes, s,
                       p);
    return hipGetLastError();
}

}  // namespace

hipError_t pi_launch(const PiParams &p, size_t lds_bytes, hipStream_t s)
{
    if (p.n_wg <= 0)
        return hipSuccess;
    if (p.n_wg > 0x7fffffffLL)
        return hipErrorInvalidConfiguration;
    const int ntn = (p.nbw * kNF * 2 + 15) / 16;
    hipError_t e;
    if (p.mtiles == 1) {
        e = ntn <= 2 ? launch_as<1, 2>(p, lds_bytes, s)
          : ntn == 3 ? launch_as<1, 3>(p, lds_bytes, s)
          : ntn == 4 ? launch_as<1, 4>(p, lds_bytes, s)
                     : launch_as<1, 5>(p, lds_bytes, s);
    } else {
        e = ntn <= 2 ? launch_as<2, 2>(p, lds_bytes, s)
          : ntn == 3 ? launch_as<2, 3>(p, lds_bytes, s)
          : ntn == 4 ? launch_as<2, 4>(p, lds_bytes, s)
                     : launch_as<2, 5>(p, lds_bytes, s);
    }
    if (e != hipSuccess)
        return e;
    const int64_t nqwa = (int64_t)p.Nqz * p.Nw * p.NA;
    const int64_t n = nqwa * kNF;
    hipLaunchKernelGGL(k_pi_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p.Pi, nqwa,
                       p.NB);
    return hipGetLastError();
}

}  // namespace sse
