// sse_internal.h -- types shared by the host runtime and the kernels of libsse.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sse.h"

namespace sse {

constexpr int kMaxTaps = 128;

// Data the kernels only read (parameter tables, D~, dH, the neighbour table)
// is addressed through the constant address space.  Nothing in a launch writes
// it, so wave-uniform reads may use scalar loads also after the kernel has
// stored results (a persistent kernel stores a tile, then reads the next
// tile's parameters).  The host compilation pass only type-checks kernel
// bodies, and there the alias is a plain pointer.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename X>
using const_ptr = const __attribute__((address_space(4))) X *;
#else
template <typename X>
using const_ptr = const X *;
#endif
template <typename X>
__device__ __forceinline__ const_ptr<X> ro(const X *p)
{
    return (const_ptr<X>)p;
}

// Binary64 tiled kernel: 256 threads, 4 positions each; two workgroups share
// one CU's 160 KiB of LDS.
namespace fp64k {
constexpr int kBlock = 256;
constexpr int kR = 4;
constexpr int kPmax = kBlock * kR;
constexpr size_t kLdsBudget = 78 * 1024;
}  // namespace fp64k

constexpr int kMaxNorb = 30;
constexpr int kMaxNB = 50;
constexpr int kN3D = 3;
constexpr int kNF = kN3D * kN3D;  // (i, j) filters

// Frequency taps, ordered by decreasing energy shift and cut into chunks whose
// G window (tile energies + shift spread of the chunk) fits the LDS budget.
// Tap t uses D~ frequency index w[t] and energy shift s[t]; chunk c covers
// taps [cb[c], cb[c+1]).
struct TapTable {
    int32_t n;
    int32_t nchunk;
    int32_t w[kMaxTaps + 8];  // padded by one group of 8 (zeros) so that a
    int32_t s[kMaxTaps + 8];  // group's entries can be read unconditionally
    int32_t cb[kMaxTaps + 1];
};

// Device pointers of one instance (one component); aux is the MFMA path's
// A-fragment buffer.
struct TensorPtrs {
    const int32_t *neigh;
    const double *dH;
    const void *G;
    const void *D;
    void *Sigma;
    const void *aux;
};

constexpr int kMaxBatch = 64;
constexpr int kQueues = 8;  // one work queue per XCD

// Kernel argument of a persistent batched launch.  Tiles are grouped in atom
// chunks (all (k, energy-tile) tiles of one atom of one instance); chunk j of
// queue x is chunk_inst/chunk_atom[j] for j in [qbeg[x], qbeg[x+1]) and its
// tiles have queue-local indices [chunk_start[j], chunk_start[j + 1]).
struct BatchLaunch {
    const void *params;            // per-instance Fp64Params / MfmaParams (sizes, taps)
    const int32_t *chunk_inst;
    const int32_t *chunk_atom;
    const int64_t *chunk_start;
    unsigned long long *counters;  // kQueues pull counters (workspace, cleared per launch)
    int32_t qbeg[kQueues + 1];
    int64_t qcount[kQueues];
    int32_t nkz[kMaxBatch];
    TensorPtrs ptr[kMaxBatch];
};

// Tile pulls of the persistent kernels, done by thread 0 of a workgroup: its
// home queue first, then the others.  A ticket (a queue-local tile index) is
// taken with one atomic when the previous tile starts, so the atomic's latency
// hides under that tile, and turned into a tile when it ends.  st[0] = queues
// given up so far (the current queue is (home + st[0]) % kQueues), st[1] = the
// chunk of this workgroup's previous ticket in the current queue, -1 if none.
// A workgroup's tickets from one queue increase, so the chunk search starts at
// st[1]: a ticket in the same chunk costs one load, one in the next chunk two,
// and only a ticket further on (or the first in a queue) a binary search.

// Ticket of the current queue; counts past the queue's end are harmless.  (The
// library is built with the compiler's atomic optimizer off: it would rewrite
// this single-lane atomic into a wave-reduced one and await its result at once.)
__device__ __forceinline__ long long pull_take(const BatchLaunch &bl, int home, const int *st)
{
    return (long long)atomicAdd(&bl.counters[(home + st[0]) & (kQueues - 1)], 1ULL);
}

// s_tile = (instance, atom, k, energy tile) of ticket t, or instance -1 once
// every queue is exhausted; a ticket past its queue's end moves on to the next
// queue (there the ticket is taken and awaited here).
__device__ __forceinline__ void pull_resolve(const BatchLaunch &bl, int home, long long t, int *st,
                                             int *s_tile)
{
    for (int d = st[0]; d < kQueues;) {
        const int qx = (home + d) & (kQueues - 1);
        if (t < bl.qcount[qx]) {
            int lo = st[1] >= 0 ? st[1] : bl.qbeg[qx];
            int hi = bl.qbeg[qx + 1] - 1;
            // chunk_start[lo] <= t; the chunk of t is the last such index:
            // step over at most two chunks, then search the rest
            int steps = 0;
            while (steps < 2 && lo < hi && bl.chunk_start[lo + 1] <= t) {
                ++lo;
                ++steps;
            }
            if (steps == 2) {
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (bl.chunk_start[mid] <= t)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
            }
            st[0] = d;
            st[1] = lo;
            const int inst = bl.chunk_inst[lo];
            const long long rem = t - bl.chunk_start[lo];
            const int nkz = bl.nkz[inst];
            s_tile[0] = inst;
            s_tile[1] = bl.chunk_atom[lo];
            s_tile[2] = (int)(rem % nkz);
            s_tile[3] = (int)(rem / nkz);
            return;
        }
        ++d;
        st[0] = d;
        st[1] = -1;
        if (d < kQueues)
            t = bl.qcount[(home + d) & (kQueues - 1)] > 0 ? pull_take(bl, home, st) : 0;
    }
    s_tile[0] = -1;
    s_tile[1] = s_tile[2] = s_tile[3] = 0;
}

// Thread 0's first pull: the home queue's first ticket, resolved.
__device__ __forceinline__ void pull_first(const BatchLaunch &bl, int home, int *st, int *s_tile)
{
    st[0] = 0;
    st[1] = -1;
    const long long t = bl.qcount[home] > 0 ? pull_take(bl, home, st) : 0;
    pull_resolve(bl, home, t, st, s_tile);
}

// Launch parameters of the FP64 tiled kernel (one component).  G, D and Sigma
// are complex128, or complex64 for SSE_FP64C64.
struct Fp64Params {
    const int32_t *neigh;
    const double *dH;
    const void *G;
    const void *D;
    void *Sigma;
    int32_t NA, NB, Norb, NN, Nkz, Nqz, NE, Nw;
    int32_t TE;        // energies per tile
    int32_t n_etiles;  // ceil(NE / TE)
    int64_t n_wg;      // n_etiles * Nkz * NA
    int32_t lds_win;   // complex elements of the window / sandwich scratch region
    double alpha_re, alpha_im;
    TapTable taps;
    // (w, s) of tap t at [2 t], [2 t + 1], padded: a tap pair's record is four
    // consecutive words, fetched one pair ahead
    int32_t tws[2 * kMaxTaps + 4];
};

// Fills Fp64Params::tws from Fp64Params::taps (host).
void fill_tap_pairs(Fp64Params &p);


// Phonon self-energy kernel (sse_pi.hip): 512 threads (8 waves, two per SIMD)
// per workgroup, one workgroup per CU; a chunk holds at most kMaxChunkTaps taps
// (two row tiles of the matrix cores) and a workgroup at most kMaxNbw
// neighbours (18 nbw <= 80 columns).
namespace pik {
constexpr int kBlock = 512;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxChunkTaps = 32;
constexpr int kMaxNbw = 4;
constexpr size_t kLdsBudgetOne = 156 * 1024;
constexpr int kMaxNorb = 16;                 // a G block row fits one load per thread
}  // namespace pik

// Tap chunks of the phonon kernel: taps sorted by increasing shift (tap t uses
// frequency tw[t], shift ts[t]); chunk c covers taps [cb[c], cb[c+1]) and needs a
// ring of at most R rows.  nbw neighbours per workgroup, mtiles row tiles.
struct PiGeom {
    int32_t nchunk;
    int32_t R;
    int32_t nbw;
    int32_t mtiles;
    int32_t cb[kMaxTaps + 1];
    int32_t tw[kMaxTaps];
    int32_t ts[kMaxTaps];
    size_t lds_bytes;
    bool ok;
};

struct PiParams {
    const double2 *X;  // the component whose energy is shifted (Pi<: G<)
    const double2 *Y;  // the opposite component (Pi<: G>)
    const double *dH;
    const int32_t *neigh;
    double2 *Pi;       // [Nqz, Nw, NA, NB + 1, 3, 3]
    int32_t NA, NB, Norb, NN, Nkz, Nqz, NE, Nw;
    int32_t nchunk, R, nbw, nbgroups, mtiles;
    int32_t cb[kMaxTaps + 1];
    int32_t tw[kMaxTaps];
    int32_t ts[kMaxTaps];
    int64_t n_wg;      // NA * Nqz * nbgroups * nchunk
    double beta_re, beta_im;
};

PiGeom pi_geometry(int Norb, int NB, const int32_t *w_shift, int Nw);

// The paper's own final form of Eq. (3) (sse_ablation.hip): transients
// M = dH G [chunk atoms][NB][3][Nkz][NE][Norb][Norb] and N = dH D
// [chunk atoms][NB][3][Nqz][Nw][Norb][Norb] in the workspace, then the
// Norb x Norb Nw x Norb GEMMs on the matrix cores.
namespace pik {
constexpr int kAblNT = 2;       // column tiles of 16: 2 Norb <= 32
constexpr int kAblBlock = 512;  // 8 waves, two per SIMD
constexpr int kAblRows = 128;   // rows (e, m) per workgroup: 8 waves x 16
}  // namespace pik
struct AblParams {
    const int32_t *neigh;
    const double *dH;
    const double2 *G;
    const double2 *D;
    double2 *Sigma;
    double2 *M;
    double2 *N;
    int32_t NA, NB, Norb, NN, Nkz, Nqz, NE, Nw;
    int32_t TE, n_etiles, smax, win_rows;
    double alpha_re, alpha_im;
    int32_t shift[kMaxTaps];
};
hipError_t ablation_launch(const AblParams &p, size_t lds_bytes, int chunk_atoms, hipStream_t s);
hipError_t pi_launch(const PiParams &p, size_t lds_bytes, hipStream_t s);

// Sampled binary64 check of a complex64 result (sse_check.hip).
struct CheckParams {
    const int32_t *neigh;
    const double *dH;
    const float2 *G;
    const float2 *D;
    const float2 *Sigma;
    const int32_t *blocks;  // [nblocks][3] = (k, e, a)
    int32_t nblocks;
    double *partial;        // [nblocks][2] workspace
    uint32_t *status;
    int32_t NA, NB, Norb, NN, Nkz, Nqz, NE, Nw;
    double alpha_re, alpha_im;
    int32_t shift[kMaxTaps];  // energy shift of frequency w
};

// Tile geometry for one problem: energies per tile, window size, LDS bytes.
struct TileGeom {
    int TE;
    int n_etiles;
    int lds_win;     // window elements (complex128 for fp64, 8-byte for the MFMA path)
    size_t lds_bytes;
};

// Host helpers (sse_fp64.hip).
TileGeom fp64_geometry(int Norb, int NE, const TapTable &taps_unchunked, int te_request,
                       int chunk_cap, TapTable *taps_out);
// ah: D~ anti-Hermitian per 3 x 3 block (only i <= j read; half the tap FMAs).
hipError_t fp64_launch(const Fp64Params &p, bool c64, bool ah, size_t lds_bytes, hipStream_t s);
hipError_t fp64_persistent_launch(const BatchLaunch &bl, bool c64, bool ah, int grid,
                                  size_t lds_bytes, hipStream_t s);


// Auxiliary kernels (sse_aux.hip).
hipError_t launch_clear_status(uint32_t *status, hipStream_t s);
hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s);
hipError_t launch_validate_neigh(const int32_t *neigh, int64_t n, int32_t NA, uint32_t *status,
                                 hipStream_t s);
// The same check for the count (<= kMaxBatch) tables of a batch in one launch:
// table t has n[t] entries that must lie in [0, NA[t]).
hipError_t launch_validate_neigh_batch(const int32_t *const *neigh, const int64_t *n,
                                       const int32_t *NA, int count, uint32_t *status,
                                       hipStream_t s);

constexpr uint32_t kStatusBadNeigh = 1u;
constexpr uint32_t kStatusBadBlock = 2u;
constexpr uint32_t kStatusAsymNeigh = 4u;  // an atom missing from its neighbour's row

// D -> Dt and the retarded components (sse_dtilde.hip).
hipError_t dtilde_launch(const void *D, void *Dt, const int32_t *neigh, int32_t *rmap,
                         uint32_t *status, int64_t nqw, int32_t NA, int32_t NB, bool c64,
                         hipStream_t s);
hipError_t retarded_launch(const void *X, void *XR, int64_t n, bool c64, hipStream_t s);

hipError_t check_launch(const CheckParams &p, double *out, hipStream_t s);

}  // namespace sse
