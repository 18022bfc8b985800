// sse_mfma.h -- declarations of the MFMA (complex64 storage) path of libsse:
// its tile constants, launch parameters and host helpers.  Shared by the
// runtime, the geometry code and sse_mfma.hip; the binary64 kernel does not
// include it.
#pragma once

#include "sse_internal.h"

namespace sse {

// MFMA kernel: 8 waves x 4 tiles of 32 columns (one workgroup per CU, two
// waves per SIMD); taps in groups of 8.  A window (one (b, q, tap chunk)) sits
// in one of two LDS buffers: two planes of 32-bit words (bf16 hi and lo words,
// or complex64 re/im interleaved across both), then the chunk's A fragments (at
// most kMaxG groups of 64 lanes x 32 bytes).  The sandwich (on the matrix
// cores) has its own LDS region.  The MFMA workspace starts with a zero page (the copy source of
// rows outside the energy grid), then the A fragments.
namespace mfmak {
constexpr int kBlock = 512;
constexpr int kNT = 4;
constexpr int kPwg = (kBlock / 64) * kNT * 32;
constexpr int kGS = 8;
constexpr int kPlaneWords = 5120;
constexpr size_t kPlaneBytes = (size_t)kPlaneWords * 4;
constexpr int kMaxG = 5;
constexpr size_t kAfragGroupBytes = 64 * 32;
constexpr size_t kBufBytes = 2 * kPlaneBytes + kMaxG * kAfragGroupBytes;
constexpr size_t kZeroPage = 256;
// Sandwich region (MFMA sandwich): two Kp x Ncolp fp32 matrices and Kp x Mp of
// dH (Kp = 3 Norb rounded up to 4, Ncolp = 2 TE Norb rounded up to 16, Mp = 16
// per 16 orbitals); the geometry keeps TE within it and within kSandT output
// tiles of 16 x 16 per wave.  The two window buffers, this region and the
// persistent kernel's tile slot fill the CU's 160 KiB.
constexpr size_t kSandBytes = 160 * 1024 - 2 * kBufBytes - 256;
constexpr int kSandT = 4;
// LDS bytes of the sandwich region for Norb and TE
constexpr size_t sand_bytes(int Norb, int TE)
{
    const size_t Kp = (size_t)((3 * Norb + 3) & ~3);
    const size_t Ncolp = (size_t)((2 * TE * Norb + 15) & ~15);
    const size_t Mp = (size_t)(16 * ((Norb + 15) >> 4));
    return (2 * Kp * Ncolp + Kp * Mp) * 4;
}
// 16 x 16 output tiles of the sandwich for Norb and TE
constexpr int sand_tiles(int Norb, int TE)
{
    return ((2 * TE * Norb + 15) >> 4) * ((Norb + 15) >> 4);
}
}  // namespace mfmak

// Groups of eight consecutive taps of one chunk (the K extent of one MFMA
// step); taps past the chunk's end are padding with zero weight.
struct GroupTable {
    int32_t n;                    // groups per qz row
    int32_t gb[kMaxTaps + 1];     // groups of chunk c are [gb[c], gb[c+1])
    int32_t t0[kMaxTaps];         // first tap of group g
};

// Launch parameters of the MFMA (complex64-storage) kernel, one component.
struct MfmaParams {
    const int32_t *neigh;
    const double *dH;
    const void *G;      // complex64 (fp32), or the planar bf16 split: hi words, then lo words
    const void *afrag;  // workspace: zero page, then the per (a, b, q, group, lane) A fragments
    float2 *Sigma;
    int32_t NA, NB, Norb, NN, Nkz, Nqz, NE, Nw;
    int32_t TE, n_etiles;
    int64_t n_wg;
    int32_t lds_win;   // 8-byte elements of the window region
    double alpha_re, alpha_im;
    TapTable taps;
    GroupTable groups;
};

struct MfmaPrepParams {
    const float2 *D;
    void *afrag;
    void *zero;         // zero page written by the prep kernel
    int32_t NA, NB, Nqz, Nw;
    TapTable taps;
    GroupTable groups;
};

// MFMA path (sse_mfma.hip).  prec is SSE_FP32 or SSE_BF16X3.
TileGeom mfma_geometry(int Norb, int NE, const TapTable &taps_unchunked, int te_request,
                       int chunk_cap, TapTable *taps_out, GroupTable *groups_out);
size_t mfma_afrag_bytes(int prec, int NA, int NB, int Nqz, const GroupTable &g);
// Workspace of one MFMA instance: zero page, A fragments, then (bf16x3) the
// planar split copy of G at mfma_split_offset.
size_t mfma_split_offset(int prec, int NA, int NB, int Nqz, const GroupTable &g);
size_t mfma_aux_bytes(int prec, int NA, int NB, int Nqz, int Nkz, int NE, int Norb,
                      const GroupTable &g);
hipError_t mfma_prep_launch(int prec, const MfmaPrepParams &p, hipStream_t s);
// the A fragments of the count instances of a batch in one launch (tables from
// bl.params, D~ and fragment buffers from bl.ptr)
hipError_t mfma_prep_batch_launch(int prec, const BatchLaunch &bl, int count, hipStream_t s);
// bf16x3: n complex64 values of G -> n hi words, then n lo words
hipError_t mfma_split_launch(const float2 *G, void *out, int64_t n, hipStream_t s);
// the same for the count (<= kMaxBatch) instances of a batch in one launch
hipError_t mfma_split_batch_launch(const float2 *const *G, void *const *out, const int64_t *n,
                                   int count, hipStream_t s);
hipError_t mfma_launch(int prec, const MfmaParams &p, size_t lds_bytes, hipStream_t s);
hipError_t mfma_persistent_launch(int prec, const BatchLaunch &bl, int grid, size_t lds_bytes,
                                  hipStream_t s);

}  // namespace sse
