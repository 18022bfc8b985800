// sse_mfma.hip -- complex64-storage scattering self-energy on the gfx950
// matrix cores: the (qz, w) tap filters of Eq. (3) (Sec. 2) as a GEMM on
// MFMA, then the dH sandwich as two fp32 GEMMs on MFMA.
//
// For one bond (a, b) with neighbour f, the tap sum
//   Gh_ij[k, e, c] = sum_{q, w} Dt[q, w, a, b, i, j] G[(k - q) mod Nkz, e - s_w, f, c]
// is a real GEMM  C[row, pos] = sum_K A[row, K] B[K, pos]  with
//   row = 2 ij + (re | im)                         (18 of the 32 MFMA rows),
//   K   = 2 tap + (re | im)                         (the complex product written out),
//   pos = (energy, orbital pair) of the output tile (32 MFMA columns per tile),
//   A[(ij, re), (t, re)] = Re D, A[(ij, re), (t, im)] = -Im D,
//   A[(ij, im), (t, re)] = Im D, A[(ij, im), (t, im)] =  Re D,
//   B[(t, x), pos] = component x of G at the tap-shifted window position.
// B is read straight from the LDS window of the neighbour's G rows (a tap is a
// uniform offset, so the im2col matrix is never formed); A depends only on
// (a, b, q) and is pre-arranged per lane by k_prep_afrag.
//
// SSE_FP32:   v_mfma_f32_32x32x2_f32, one tap per instruction.
// SSE_BF16X3: v_mfma_f32_32x32x16_bf16, eight taps per instruction; every fp32
//             operand x is split x = hi + lo (bf16 hi, bf16 lo = x - hi) and the
//             product is hi*hi + hi*lo + lo*hi.
// Accumulation: fp32 inside the MFMA over the taps of one energy window (one
// qz row), binary64 across windows (the sum over qz and the tap chunks); the
// sandwich's Norb x Norb block products and the sum over neighbours are fp32
// (v_mfma_f32_16x16x4f32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sse_internal.h"
#include "sse_mfma.h"
#include "sse_copy.h"

namespace sse {

namespace {

constexpr int kBlock = mfmak::kBlock;
constexpr int kNT = mfmak::kNT;               // 32-column tiles per wave
constexpr int kPwg = mfmak::kPwg;             // output positions per workgroup
constexpr int kGS = mfmak::kGS;               // taps per group
constexpr size_t kPlaneBytes = mfmak::kPlaneBytes;
constexpr size_t kBufBytes = mfmak::kBufBytes;
constexpr size_t kZeroPage = mfmak::kZeroPage;
constexpr size_t kAfragGroupBytes = mfmak::kAfragGroupBytes;
constexpr size_t kSandBytes = mfmak::kSandBytes;
constexpr int kDhR = (kN3D * 484 + kBlock - 1) / kBlock;  // dH values per thread (Norb <= 22)
constexpr int kSandT = mfmak::kSandT;         // sandwich output tiles per wave

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t n)
{
    const int64_t per = n >> 3;
    if (bid >= (per << 3))
        return bid;
    return (bid & 7) * per + (bid >> 3);
}

// Workgroup barrier for data exchanged through LDS by ordinary LDS reads and
// writes only: waits for this wave's LDS operations, not for its vector-memory
// operations, so global -> LDS copies in flight into another buffer stay in
// flight (a __syncthreads() fence would wait for them: they write LDS).  The
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);  // vmcnt and expcnt not waited
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

__device__ __forceinline__ uint32_t bf16_bits(float x)
{
    __bf16 h = (__bf16)x;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float bf16_value(uint32_t bits)
{
    return __builtin_bit_cast(float, bits << 16);
}

// hi and lo bf16 parts of x packed as (hi, lo) bit patterns.
__device__ __forceinline__ void split_bf16(float x, uint32_t &hi, uint32_t &lo)
{
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
}

// A-operand value of MFMA row r for tap t, K component x (0 = re, 1 = im).
__device__ __forceinline__ float a_value(const float2 *D, int NA, int NB, int Nw,
                                         const TapTable &taps, int ab, int q, int row, int t,
                                         int tend, int x)
{
    const int ij = row >> 1, ri = row & 1;
    if (ij >= kNF || t >= tend)
        return 0.0f;
    const float2 d = D[(((size_t)q * Nw + taps.w[t]) * NA * NB + ab) * kNF + ij];
    if (ri == 0)
        return x == 0 ? d.x : -d.y;
    return x == 0 ? d.y : d.x;
}

// Item idx of the A-fragment preparation of one instance: the first
// kZeroPage / 16 items also clear the zero page; item (a, b, q, group, lane)
// writes the lane's 32-byte A fragment.  The tables are the instance's (a
// kernel argument, or a batch's table in global memory).
template <int PREC>
__device__ __forceinline__ void prep_item(int64_t idx, const float2 *D, void *afrag, void *zero,
                                          int NA, int NB, int Nqz, int Nw, const TapTable &taps,
                                          const GroupTable &groups)
{
    if (idx < (int64_t)(kZeroPage / 16))
        reinterpret_cast<uint4 *>(zero)[idx] = make_uint4(0u, 0u, 0u, 0u);
    const int lane = (int)(idx & 63);
    int64_t rest = idx >> 6;
    const int g = (int)(rest % groups.n);
    rest /= groups.n;
    const int q = (int)(rest % Nqz);
    const int64_t ab = rest / Nqz;
    if (ab >= (int64_t)NA * NB)
        return;
    int c = 0;
    while (groups.gb[c + 1] <= g)
        ++c;
    const int tend = taps.cb[c + 1];
    const int t0 = groups.t0[g];
    const int row = lane & 31, h = lane >> 5;
    uint4 *out = reinterpret_cast<uint4 *>(afrag) + (idx << 1);
    if (PREC == SSE_BF16X3) {
        uint32_t hi[8], lo[8];
        for (int u = 0; u < 4; ++u)
            for (int x = 0; x < 2; ++x)
                split_bf16(a_value(D, NA, NB, Nw, taps, (int)ab, q, row, t0 + 4 * h + u, tend, x),
                           hi[2 * u + x], lo[2 * u + x]);
        out[0] = make_uint4(hi[0] | hi[1] << 16, hi[2] | hi[3] << 16, hi[4] | hi[5] << 16,
                            hi[6] | hi[7] << 16);
        out[1] = make_uint4(lo[0] | lo[1] << 16, lo[2] | lo[3] << 16, lo[4] | lo[5] << 16,
                            lo[6] | lo[7] << 16);
    } else {
        float v[8];
        for (int u = 0; u < 8; ++u)
            v[u] = a_value(D, NA, NB, Nw, taps, (int)ab, q, row, t0 + u, tend, h);
        out[0] = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                            __float_as_uint(v[3]));
        out[1] = make_uint4(__float_as_uint(v[4]), __float_as_uint(v[5]), __float_as_uint(v[6]),
                            __float_as_uint(v[7]));
    }
}

// One thread per (a, b, q, group, lane): the lane's 32-byte A fragment.
template <int PREC>
__global__ void k_prep_afrag(const MfmaPrepParams p)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    prep_item<PREC>(idx, p.D, p.afrag, p.zero, p.NA, p.NB, p.Nqz, p.Nw, p.taps, p.groups);
}

// The A fragments of every instance of a batch in one launch: blockIdx.y is
// the instance (sizes and tables from the batch's parameter table, D~ and the
// fragment buffer from the launch's pointers); each instance's items are
// strided over the grid's x extent.
template <int PREC>
__global__ void k_prep_afrag_batch(const BatchLaunch bl)
{
    const int t = blockIdx.y;
    const MfmaParams &mp = reinterpret_cast<const MfmaParams *>(bl.params)[t];
    const int NA = mp.NA, NB = mp.NB, Nqz = mp.Nqz, Nw = mp.Nw;
    const int64_t n = std::max<int64_t>((int64_t)NA * NB * Nqz * mp.groups.n * 64,
                                        (int64_t)(kZeroPage / 16));
    const float2 *D = reinterpret_cast<const float2 *>(bl.ptr[t].D);
    char *aux = reinterpret_cast<char *>(const_cast<void *>(bl.ptr[t].aux));
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x)
        prep_item<PREC>(idx, D, aux + kZeroPage, aux, NA, NB, Nqz, Nw, mp.taps, mp.groups);
}

// One output tile (energies [et TE, et TE + TE) of (k, a)); pp supplies sizes and
// tap/group tables (a kernel argument or a batch table in global memory), ptr
// the tensors (aux = zero page, then A fragments).
//
// The tile walks its windows (neighbour b, momentum transfer q, tap chunk c)
// through two LDS buffers: while the MFMAs consume window n from one buffer,
// the copy engine fills the other with window n + 1 (G rows and A fragments),
// so one barrier per window separates them.  After the last window of a
// neighbour the sandwich runs on the matrix cores in its own LDS region.
// bufA and bufB are distinct __shared__ arrays and the window loop alternates
// them by name, so the compiler can see that reads of one buffer do not
// depend on the copies in flight into the other.
template <int PREC>
__device__ __forceinline__ void mfma_tile(const_ptr<MfmaParams> pp, const TensorPtrs &ptr, int a,
                                          int k, int et, unsigned char *bufA, unsigned char *bufB,
                                          unsigned char *sand)
{
    const auto &p = *pp;
    const int e0 = et * p.TE;
    const int te = min(p.TE, p.NE - e0);
    const int NN = p.NN, No = p.Norb;
    const int P = te * NN;
    const int Pst = p.TE * NN;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, h = lane >> 5;

    // MFMA column of this lane in tile t: pos0 + 32 t.  Columns at or past P
    // read in-plane words (a plane holds kPwg + spread NN words) and their
    // results are never used: an MFMA column depends on its B column only.
    const int pos0 = wave * kNT * 32 + (lane & 31);
    bool pval[kNT];
#pragma unroll
    for (int t = 0; t < kNT; ++t)
        pval[t] = pos0 + 32 * t < P;
    // Sandwich geometry (see the sandwich below): K = 3 Norb rounded up to the
    // MFMA K step, Ncol = 2 TE Norb columns (energy, orbital, re/im) in tiles
    // of 16, Norb rows in nmt tiles of 16.  LDS: G1 and B2 (Kp x Ncolp fp32
    // each), then Ap (Kp x Mp).
    const int Kp = (kN3D * No + 3) & ~3;
    const int Ncol = 2 * p.TE * No;
    const int Ncolp = (Ncol + 15) & ~15;
    const int nmt = (No + 15) >> 4;
    const int Mp = 16 * nmt;
    const int nst = (Ncolp >> 4) * nmt;  // 16 x 16 output tiles
    // one array indexed from its start (a short address chain keeps the
    // compiler's knowledge that this region is not the window buffers)
    float *sf = reinterpret_cast<float *>(sand);
    const int oB2 = Kp * Ncolp, oAp = 2 * Kp * Ncolp;  // G1 at 0
    // rows of G1 and B2 past 3 Norb and all of Ap start at zero (Ap's rows and
    // columns past the data stay zero); the window barriers order this before
    // the first sandwich
    for (int idx = tid; idx < (Kp - kN3D * No) * Ncolp; idx += kBlock) {
        sf[kN3D * No * Ncolp + idx] = 0.0f;
        sf[oB2 + kN3D * No * Ncolp + idx] = 0.0f;
    }
    for (int idx = tid; idx < Kp * Mp; idx += kBlock)
        sf[oAp + idx] = 0.0f;
    const float rNN = 1.0f / (float)NN, rNo = 1.0f / (float)No, r2No = 0.5f / (float)No;
    // Sigma tiles owned by this wave: s-th tile is wave + 8 s; their fp32 sums
    // over neighbours
    f32x4 S2[kSandT];
#pragma unroll
    for (int st = 0; st < kSandT; ++st)
        S2[st] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    const int64_t strideE = (int64_t)p.NA * NN;                 // elements per energy row
    const int64_t g_elems = (int64_t)p.Nkz * p.NE * strideE;
    const uint32_t *zero = reinterpret_cast<const uint32_t *>(ptr.aux);
    const unsigned char *afrag = reinterpret_cast<const unsigned char *>(ptr.aux) + kZeroPage;
    const int nch = p.taps.nchunk;
    const int nwin = p.NB * p.Nqz * nch;

    // window w = (b, q, c), c fastest; windows of invalid neighbours are skipped
    auto neighbour = [&](int b) { return ro(ptr.neigh)[(size_t)a * p.NB + b]; };
    auto next_valid = [&](int w) {
        while (w < nwin) {
            const int f = neighbour(w / (p.Nqz * nch));
            if ((unsigned)f < (unsigned)p.NA)
                break;
            w = (w / (p.Nqz * nch) + 1) * (p.Nqz * nch);
        }
        return w;
    };
    // start the copies of window w into buffer buf
    auto issue = [&](int w, unsigned char *buf) {
        const int b = w / (p.Nqz * nch), q = (w / nch) % p.Nqz, c = w % nch;
        const int f = neighbour(b);
        int kk = k - q;
        if (kk < 0)
            kk += p.Nkz;
        const int smax = p.taps.s[p.taps.cb[c]], smin = p.taps.s[p.taps.cb[c + 1] - 1];
        const int nrow = te + smax - smin;
        uint32_t *P0 = reinterpret_cast<uint32_t *>(buf);
        const int64_t row0 = (int64_t)kk * p.NE * strideE + (int64_t)f * NN;  // element index
        if constexpr (PREC == SSE_BF16X3) {
            // planar split G: hi words [g_elems], then lo words [g_elems]
            const uint32_t *Ghi = reinterpret_cast<const uint32_t *>(ptr.G) + row0;
            uint32_t *P1 = reinterpret_cast<uint32_t *>(buf + kPlaneBytes);
            if ((NN & 3) == 0) {
                copy_window<4, kBlock>(P0, Ghi, strideE, e0 - smax, p.NE, nrow, NN, zero);
                copy_window<4, kBlock>(P1, Ghi + g_elems, strideE, e0 - smax, p.NE, nrow, NN, zero);
            } else {
                copy_window<1, kBlock>(P0, Ghi, strideE, e0 - smax, p.NE, nrow, NN, zero);
                copy_window<1, kBlock>(P1, Ghi + g_elems, strideE, e0 - smax, p.NE, nrow, NN, zero);
            }
        } else {
            // complex64 G, (re, im) interleaved across both planes' space
            const uint32_t *Gw = reinterpret_cast<const uint32_t *>(ptr.G) + 2 * row0;
            if ((NN & 1) == 0)
                copy_window<4, kBlock>(P0, Gw, 2 * strideE, e0 - smax, p.NE, nrow, 2 * NN, zero);
            else
                copy_window<1, kBlock>(P0, Gw, 2 * strideE, e0 - smax, p.NE, nrow, 2 * NN, zero);
        }
        const int g0 = p.groups.gb[c], g1 = p.groups.gb[c + 1];
        const unsigned char *asrc =
            afrag + ((((size_t)a * p.NB + b) * p.Nqz + q) * p.groups.n + g0) * kAfragGroupBytes;
        copy_to_lds<4, kBlock>(reinterpret_cast<uint32_t *>(buf + 2 * kPlaneBytes),
                       (g1 - g0) * (kAfragGroupBytes / 16),
                       [&](int u) { return reinterpret_cast<const void *>(asrc + (size_t)u * 16); });
    };

    double acc[kNT][10];
    float dh[kDhR];  // this thread's share of the current neighbour's dH rows
    // window w from buf (its copies were issued earlier) while window wn is
    // copied into other; returns wn
    auto run_window = [&](int w, unsigned char *buf, unsigned char *other) {
        const int b = w / (p.Nqz * nch), q = (w / nch) % p.Nqz, c = w % nch;
        const int wn = next_valid(w + 1);
        // window w has landed and every wave is done with the other buffer
        __syncthreads();
        if (q == 0 && c == 0) {
            // neighbour b's dH rows for its sandwich, loaded before any copy is
            // issued behind them (vector-memory results return in order)
            const double *Ag = ptr.dH + ((size_t)a * p.NB + b) * kN3D * NN;
#pragma unroll
            for (int r = 0; r < kDhR; ++r) {
                const int idx = tid + r * kBlock;
                dh[r] = idx < kN3D * NN ? (float)Ag[idx] : 0.0f;
            }
        }
        if (wn < nwin)
            issue(wn, other);
        if (q == 0 && c == 0) {
#pragma unroll
            for (int t = 0; t < kNT; ++t)
#pragma unroll
                for (int v = 0; v < 10; ++v)
                    acc[t][v] = 0.0;
        }

        const int t1c = p.taps.cb[c + 1];
        const int smax = p.taps.s[p.taps.cb[c]];
        const uint32_t *P0 = reinterpret_cast<const uint32_t *>(buf);
        const uint32_t *P1 = reinterpret_cast<const uint32_t *>(buf + kPlaneBytes);
        const uint4 *Ab = reinterpret_cast<const uint4 *>(buf + 2 * kPlaneBytes);
        f32x16 C[kNT];
        // one group of kGS taps; the first group of a window starts from a zero
        // accumulator
        auto step = [&](int g, int gi, auto first) {
            constexpr bool kFirst = decltype(first)::value;
            const uint4 A0 = Ab[gi * 128 + lane * 2];
            const uint4 A1 = Ab[gi * 128 + lane * 2 + 1];
            const int tg = p.groups.t0[g];
            // the group's eight shifts, read unconditionally (the table is padded)
            // so that they arrive together; padding taps (t >= t1c) read offset 0
            int off[kGS];
#pragma unroll
            for (int u = 0; u < kGS; ++u) {
                const int sv = p.taps.s[tg + u];
                off[u] = (smax - sv) * NN * (int)(tg + u < t1c);  // no branch to sink the load into
            }
            if constexpr (PREC == SSE_BF16X3) {
                // lanes of half h carry taps tg + 4 h + u, u = 0..3
                int idx[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    idx[u] = pos0 + (h ? off[4 + u] : off[u]);
                const bf16x8 ahi = __builtin_bit_cast(bf16x8, A0);
                const bf16x8 alo = __builtin_bit_cast(bf16x8, A1);
                // all four tiles' B operands first, then the three products in
                // rounds over the tiles: consecutive MFMAs are independent
                bf16x8 bhi[kNT], blo[kNT];
#pragma unroll
                for (int t = 0; t < kNT; ++t) {
                    bhi[t] = __builtin_bit_cast(
                        bf16x8, make_uint4(P0[idx[0] + 32 * t], P0[idx[1] + 32 * t],
                                           P0[idx[2] + 32 * t], P0[idx[3] + 32 * t]));
                    blo[t] = __builtin_bit_cast(
                        bf16x8, make_uint4(P1[idx[0] + 32 * t], P1[idx[1] + 32 * t],
                                           P1[idx[2] + 32 * t], P1[idx[3] + 32 * t]));
                }
#pragma unroll
                for (int t = 0; t < kNT; ++t) {
                    if constexpr (kFirst)
                        C[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi[t], f32x16{}, 0, 0,
                                                                       0);
                    else
                        C[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bhi[t], C[t], 0, 0, 0);
                }
#pragma unroll
                for (int t = 0; t < kNT; ++t)
                    C[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, blo[t], C[t], 0, 0, 0);
#pragma unroll
                for (int t = 0; t < kNT; ++t)
                    C[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bhi[t], C[t], 0, 0, 0);
            } else {
                // K = 2 per instruction: lanes of half h carry component h of tap
                // tg + u, word 2 (position + offset) + h of the interleaved window
                const float av[8] = {__uint_as_float(A0.x), __uint_as_float(A0.y),
                                     __uint_as_float(A0.z), __uint_as_float(A0.w),
                                     __uint_as_float(A1.x), __uint_as_float(A1.y),
                                     __uint_as_float(A1.z), __uint_as_float(A1.w)};
                const float *W = reinterpret_cast<const float *>(P0) + h;
#pragma unroll
                for (int u = 0; u < kGS; ++u) {
                    const int t = tg + u;
                    // one tap per instruction: the padding taps of a chunk's
                    // last group are skipped (the first tap of a group is real)
                    if (u > 0 && t >= t1c)
                        break;
                    const int idx = 2 * (pos0 + off[u]);
#pragma unroll
                    for (int tt = 0; tt < kNT; ++tt) {
                        const float bv = W[idx + 64 * tt];
                        if (kFirst && u == 0)
                            C[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bv, f32x16{}, 0, 0,
                                                                         0);
                        else
                            C[tt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bv, C[tt], 0, 0, 0);
                    }
                }
            }
        };
        const int g0 = p.groups.gb[c], g1 = p.groups.gb[c + 1];
        step(g0, 0, std::true_type{});
        for (int g = g0 + 1; g < g1; ++g)
            step(g, g - g0, std::false_type{});
        // fold this window's fp32 partial sums into the binary64 accumulators
#pragma unroll
        for (int t = 0; t < kNT; ++t)
#pragma unroll
            for (int v = 0; v < 10; ++v)
                acc[t][v] += (double)C[t][v];

        if (q == p.Nqz - 1 && c == nch - 1) {
            // ---- sandwich of neighbour b on the matrix cores, fp32:
            //   step 1, per j:  T_j[m, (e, n, x)] = sum_(i,l) Ap[(i,l), m] Gh_ij[e][l, n]_x
            //   step 2:         S[n', (e, m, x)] += sum_(j,l) Ap[(j,l), n'] T_j[e][m, l]_x
            // with Ap[(i, l), m] = dH_i[m, l] in both steps (x = re | im).
            // v_mfma_f32_16x16x4f32: lane L holds A[L % 16][L / 16] and
            // B[L / 16][L % 16] and receives C[4 (L / 16) + r][L % 16], r < 4.
            lds_barrier();  // the previous neighbour's sandwich reads are done
#pragma unroll
            for (int r = 0; r < kDhR; ++r) {
                const int idx = tid + r * kBlock;  // dH_i[m, l], idx = i NN + m No + l
                if (idx < kN3D * NN) {
                    const int i = small_div(idx, NN, rNN), rem = idx - i * NN;
                    const int m = small_div(rem, No, rNo), l = rem - m * No;
                    sf[oAp + (i * No + l) * Mp + m] = dh[r];
                }
            }
            // per-lane indices, made opaque here so that the compiler does not
            // hoist them out of the window loop and hold them in registers
            int ln = lane, pz = pos0;
            asm volatile("" : "+v"(ln), "+v"(pz));
            const int kr = ln >> 4, kc = ln & 15;
            for (int j = 0; j < kN3D; ++j) {
                // Gh_{.j} -> G1[(i, l), (e, n, x)]; C rows held by this lane:
                // row = 8 (v / 4) + 4 h + v % 4 = 2 ij + x
#pragma unroll
                for (int t = 0; t < kNT; ++t) {
                    const int pos = pz + 32 * t;
                    const int e = small_div(pos, NN, rNN), rem = pos - e * NN;
                    const int l = small_div(rem, No, rNo), n = rem - l * No;
                    const int g1 = l * Ncolp + (e * No + n) * 2;
#pragma unroll
                    for (int v = 0; v < 10; v += 2) {
                        const int row = 8 * (v >> 2) + 4 * h + (v & 3);
                        const int ij = row >> 1;
                        if (ij < kNF && ij % kN3D == j && pval[t])
                            *reinterpret_cast<float2 *>(sf + g1 + (ij / kN3D) * No * Ncolp) =
                                make_float2((float)acc[t][v], (float)acc[t][v + 1]);
                    }
                }
                lds_barrier();
                // this wave's output tiles gt = wave + 8 st, the K steps outermost
                // so that the tiles' MFMAs are independent
                f32x4 T[kSandT];
#pragma unroll
                for (int st = 0; st < kSandT; ++st)
                    T[st] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                for (int ks = 0; ks < Kp; ks += 4) {
                    const int ia = oAp + (ks + kr) * Mp + kc, ib = (ks + kr) * Ncolp + kc;
#pragma unroll
                    for (int st = 0; st < kSandT; ++st) {
                        const int gt = wave + 8 * st;
                        if (gt < nst) {
                            const int ct = nmt == 1 ? gt : gt >> 1, mt = gt - ct * nmt;
                            T[st] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                sf[ia + mt * 16], sf[ib + ct * 16], T[st], 0, 0, 0);
                        }
                    }
                }
                // T_j[m][col = (e, n, x)] -> B2[(j, n), (e, m, x)]
#pragma unroll
                for (int st = 0; st < kSandT; ++st) {
                    const int gt = wave + 8 * st;
                    if (gt < nst) {
                        const int ct = nmt == 1 ? gt : gt >> 1, mt = gt - ct * nmt;
                        const int col = ct * 16 + kc;
                        const int e = small_div(col, 2 * No, r2No), rem = col - e * 2 * No;
                        const int n = rem >> 1, x = rem & 1;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int m = mt * 16 + 4 * kr + r;
                            if (m < No && col < Ncol)
                                sf[oB2 + (j * No + n) * Ncolp + (e * No + m) * 2 + x] = T[st][r];
                        }
                    }
                }
                lds_barrier();  // G1 reads (and, after j = 2, the B2 writes) are done
            }
            for (int ks = 0; ks < Kp; ks += 4) {
                const int ia = oAp + (ks + kr) * Mp + kc, ib = oB2 + (ks + kr) * Ncolp + kc;
#pragma unroll
                for (int st = 0; st < kSandT; ++st) {
                    const int gt = wave + 8 * st;
                    if (gt < nst) {
                        const int ct = nmt == 1 ? gt : gt >> 1, mt = gt - ct * nmt;
                        S2[st] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            sf[ia + mt * 16], sf[ib + ct * 16], S2[st], 0, 0, 0);
                    }
                }
            }
        }
        return wn;
    };
    int w = next_valid(0);
    if (w < nwin)
        issue(w, bufA);
    // every issue is followed by a window that begins with a barrier, so no
    // copy is in flight when the loop ends
    while (w < nwin) {
        w = run_window(w, bufA, bufB);
        if (w >= nwin)
            break;
        w = run_window(w, bufB, bufA);
    }

    // ---- Sigma[k, e0 + e, a] = alpha * sum: the tiles S[n', (e, m, x)] go
    // through LDS (G1 is free: every wave has passed the last sandwich's
    // step 1) and are stored by position, coalesced
    float *Sst = sf;
    {
        const int kr = lane >> 4, kc = lane & 15;
#pragma unroll
        for (int st = 0; st < kSandT; ++st) {
            const int gt = wave + 8 * st;
            if (gt < nst) {
                const int ct = nmt == 1 ? gt : gt >> 1, mt = gt - ct * nmt;
                const int col = ct * 16 + kc;
                const int e = small_div(col, 2 * No, r2No), rem = col - e * 2 * No;
                const int m = rem >> 1, x = rem & 1;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = mt * 16 + 4 * kr + r;
                    if (n < No && e < te)
                        Sst[(e * NN + m * No + n) * 2 + x] = S2[st][r];
                }
            }
        }
    }
    lds_barrier();
    float2 *Sk = (float2 *)ptr.Sigma + ((size_t)k * p.NE + e0) * strideE + (size_t)a * NN;
    for (int pos = tid; pos < P; pos += kBlock) {
        const float sre = Sst[2 * pos], sim = Sst[2 * pos + 1];
        const int e = small_div(pos, NN, rNN), c = pos - e * NN;
        Sk[(size_t)e * strideE + c] =
            make_float2((float)(p.alpha_re * sre - p.alpha_im * sim),
                        (float)(p.alpha_re * sim + p.alpha_im * sre));
    }
}

// bf16x3: every complex64 value of G as a hi word (re_hi | im_hi << 16) in
// out[0, n) and a lo word (re_lo | im_lo << 16) in out[n, 2 n).
__global__ void k_split_g(const float2 *__restrict__ G, uint32_t *__restrict__ out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 v = G[i];
        uint32_t rh, rl, ih, il;
        split_bf16(v.x, rh, rl);
        split_bf16(v.y, ih, il);
        out[i] = rh | ih << 16;
        out[n + i] = rl | il << 16;
    }
}

// The instances of a batch: blockIdx.y selects the instance.
struct SplitBatch {
    const float2 *G[kMaxBatch];
    uint32_t *out[kMaxBatch];
    int64_t n[kMaxBatch];
};

__global__ void k_split_g_batch(const SplitBatch sb)
{
    const int t = blockIdx.y;
    const float2 *__restrict__ G = sb.G[t];
    uint32_t *__restrict__ out = sb.out[t];
    const int64_t n = sb.n[t];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 v = G[i];
        uint32_t rh, rl, ih, il;
        split_bf16(v.x, rh, rl);
        split_bf16(v.y, ih, il);
        out[i] = rh | ih << 16;
        out[n + i] = rl | il << 16;
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock, 1) void k_sse_mfma(const MfmaParams p)
{
    __shared__ __align__(16) unsigned char bufA[kBufBytes];
    __shared__ __align__(16) unsigned char bufB[kBufBytes];
    __shared__ __align__(16) unsigned char sand[kSandBytes];
    // G: planar bf16 split (bf16x3) or complex64 (fp32); aux: zero page, A fragments
    const TensorPtrs ptr{p.neigh, p.dH, p.G, nullptr, p.Sigma, p.afrag};
    int64_t L = xcd_remap(blockIdx.x, p.n_wg);
    const int k = (int)(L % p.Nkz);
    L /= p.Nkz;
    const int et = (int)(L % p.n_etiles);
    const int a = (int)(L / p.n_etiles);
    mfma_tile<PREC>(ro(&p), ptr, a, k, et, bufA, bufB, sand);
}

// Persistent form over a batch's work queues (see pull_resolve).
template <int PREC>
__global__ __launch_bounds__(kBlock, 1) void k_sse_mfma_persistent(const BatchLaunch bl)
{
    __shared__ __align__(16) unsigned char bufA[kBufBytes];
    __shared__ __align__(16) unsigned char bufB[kBufBytes];
    __shared__ __align__(16) unsigned char sand[kSandBytes];
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
        mfma_tile<PREC>(ro(reinterpret_cast<const MfmaParams *>(bl.params)) + inst, bl.ptr[inst],
                        a, k, et, bufA, bufB, sand);
        if (threadIdx.x == 0)
            pull_resolve(bl, home, ticket, s_st, s_tile);
        __syncthreads();
    }
}

}  // namespace

hipError_t mfma_split_launch(const float2 *G, void *out, int64_t n, hipStream_t s)
{
    int64_t g = (n + 255) / 256;
    if (g > 65536)
        g = 65536;
    if (g < 1)
        g = 1;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_split_g, dim3((unsigned)g), dim3(256), 0, s, G, (uint32_t *)out, n);
    return hipGetLastError();
}

hipError_t mfma_split_batch_launch(const float2 *const *G, void *const *out, const int64_t *n,
                                   int count, hipStream_t s)
{
    if (count < 1 || count > kMaxBatch)
        return hipErrorInvalidValue;
    SplitBatch sb{};
    int64_t nmax = 1;
    for (int t = 0; t < count; ++t) {
        sb.G[t] = G[t];
        sb.out[t] = (uint32_t *)out[t];
        sb.n[t] = n[t];
        nmax = n[t] > nmax ? n[t] : nmax;
    }
    // about 65536 workgroups over the batch, at least one per instance
    int64_t g = (nmax + 255) / 256;
    const int64_t cap = std::max<int64_t>(1, 65536 / count);
    if (g > cap)
        g = cap;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_split_g_batch, dim3((unsigned)g, (unsigned)count), dim3(256), 0, s, sb);
    return hipGetLastError();
}

hipError_t mfma_prep_batch_launch(int prec, const BatchLaunch &bl, int count, hipStream_t s)
{
    if (count < 1 || count > kMaxBatch)
        return hipErrorInvalidValue;
    (void)hipGetLastError();
    if (prec == SSE_BF16X3)
        hipLaunchKernelGGL(k_prep_afrag_batch<SSE_BF16X3>, dim3(1024, (unsigned)count), dim3(256),
                           0, s, bl);
    else
        hipLaunchKernelGGL(k_prep_afrag_batch<SSE_FP32>, dim3(1024, (unsigned)count), dim3(256),
                           0, s, bl);
    return hipGetLastError();
}

hipError_t mfma_prep_launch(int prec, const MfmaPrepParams &p, hipStream_t s)
{
    const int64_t n = (int64_t)p.NA * p.NB * p.Nqz * p.groups.n * 64;
    const int64_t nb = (n + 255) / 256;
    if (nb > 0x7fffffffLL)
        return hipErrorInvalidConfiguration;
    if (prec == SSE_BF16X3) {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_prep_afrag<SSE_BF16X3>, dim3((unsigned)nb), dim3(256), 0, s, p);
    } else {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_prep_afrag<SSE_FP32>, dim3((unsigned)nb), dim3(256), 0, s, p);
    }
    return hipGetLastError();
}

// The MFMA kernels use static LDS only (two window buffers); lds_bytes is the
// dynamic amount, zero for these kernels.
hipError_t mfma_persistent_launch(int prec, const BatchLaunch &bl, int grid, size_t lds_bytes,
                                  hipStream_t s)
{
    if (prec == SSE_BF16X3) {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_sse_mfma_persistent<SSE_BF16X3>, dim3(grid), dim3(kBlock), lds_bytes,
                           s, bl);
    } else {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_sse_mfma_persistent<SSE_FP32>, dim3(grid), dim3(kBlock), lds_bytes, s,
                           bl);
    }
    return hipGetLastError();
}

hipError_t mfma_launch(int prec, const MfmaParams &p, size_t lds_bytes, hipStream_t s)
{
    if (p.n_wg <= 0)
        return hipSuccess;
    if (p.n_wg > 0x7fffffffLL)
        return hipErrorInvalidConfiguration;
    if (prec == SSE_BF16X3) {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_sse_mfma<SSE_BF16X3>, dim3((unsigned)p.n_wg), dim3(kBlock), lds_bytes,
                           s, p);
    } else {
        (void)hipGetLastError();
        hipLaunchKernelGGL(k_sse_mfma<SSE_FP32>, dim3((unsigned)p.n_wg), dim3(kBlock), lds_bytes, s,
                           p);
    }
    return hipGetLastError();
}

}  // namespace sse
