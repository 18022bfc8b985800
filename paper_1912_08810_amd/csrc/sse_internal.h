// sse_internal.h -- types shared by the host runtime and the kernels of libsse.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sse.h"

namespace sse {

constexpr int kMaxTaps = 128;
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
    int32_t w[kMaxTaps];
    int32_t s[kMaxTaps];
    int32_t cb[kMaxTaps + 1];
};

// Launch parameters of the FP64 tiled kernel (one component).
struct Fp64Params {
    const int32_t *neigh;
    const double *dH;
    const double2 *G;
    const double2 *D;
    double2 *Sigma;
    int32_t NA, NB, Norb, NN, Nkz, Nqz, NE, Nw;
    int32_t TE;        // energies per tile
    int32_t n_etiles;  // ceil(NE / TE)
    int64_t n_wg;      // n_etiles * Nkz * NA
    int32_t lds_win;   // complex elements of the window / sandwich scratch region
    double alpha_re, alpha_im;
    TapTable taps;
};

// Tile geometry for one problem: energies per tile, window size, LDS bytes.
struct TileGeom {
    int TE;
    int n_etiles;
    int lds_win;     // complex128 elements of the window/scratch region
    size_t lds_bytes;
};

// Host helpers (sse_fp64.hip).
TileGeom fp64_geometry(int Norb, int NE, const TapTable &taps_unchunked, int te_request,
                       TapTable *taps_out);
hipError_t fp64_launch(const Fp64Params &p, size_t lds_bytes, hipStream_t s);

// Auxiliary kernels (sse_aux.hip).
hipError_t launch_clear_status(uint32_t *status, hipStream_t s);
hipError_t launch_validate_neigh(const int32_t *neigh, int64_t n, int32_t NA, uint32_t *status,
                                 hipStream_t s);

constexpr uint32_t kStatusBadNeigh = 1u;

}  // namespace sse
