// sse_geometry.hip -- host-side tile geometry of the kernels: energies per
// tile, tap chunks whose G window fits the LDS budget, MFMA tap groups, LDS
// bytes and workspace sizes.  Host code only (also built by the host-side
// runtime test with a stand-in HIP header).
#include <algorithm>
#include <vector>

#include "sse_internal.h"
#include "sse_mfma.h"

namespace sse {

TileGeom fp64_geometry(int Norb, int NE, const TapTable &taps, int te_request, int chunk_cap,
                       TapTable *out)
{
    const int NN = Norb * Norb;
    int TE = fp64k::kPmax / NN;
    if (te_request > 0)
        TE = std::min(TE, te_request);
    TE = std::max(1, std::min(TE, NE));
    const size_t a_bytes = (size_t)kN3D * NN * sizeof(double);
    const long budget = (long)((fp64k::kLdsBudget - a_bytes) / sizeof(double2));

    *out = taps;
    out->nchunk = 0;
    int t = 0;
    long win_max = 0;
    while (t < taps.n) {
        int u = t + 1;
        while (u < taps.n && (chunk_cap <= 0 || u - t < chunk_cap) &&
               fp64k::kPmax + (long)(taps.s[t] - taps.s[u]) * NN <= budget)
            ++u;
        out->cb[out->nchunk++] = t;
        win_max = std::max(win_max, fp64k::kPmax + (long)(taps.s[t] - taps.s[u - 1]) * NN);
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

void fill_tap_pairs(Fp64Params &p)
{
    for (int t = 0; t < 2 * kMaxTaps + 4; ++t)
        p.tws[t] = 0;
    for (int t = 0; t < p.taps.n; ++t) {
        p.tws[2 * t] = p.taps.w[t];
        p.tws[2 * t + 1] = p.taps.s[t];
    }
}

TileGeom mfma_geometry(int Norb, int NE, const TapTable &taps, int te_request, int chunk_cap,
                       TapTable *out, GroupTable *groups)
{
    const int NN = Norb * Norb;
    int TE = mfmak::kPwg / NN;
    if (te_request > 0)
        TE = std::min(TE, te_request);
    TE = std::max(1, std::min(TE, NE));
    // the sandwich's LDS region and output tiles per wave bound TE too (small
    // Norb only: Norb >= 4 keeps TE = kPwg / Norb^2)
    while (TE > 1 && (mfmak::sand_bytes(Norb, TE) > mfmak::kSandBytes ||
                      mfmak::sand_tiles(Norb, TE) > 8 * mfmak::kSandT))
        --TE;
    // A plane holds the window rows plus the reach of the columns past the
    // tile's last position: kPwg + (shift spread of the chunk) NN words; a
    // chunk's A fragments fill at most kMaxG groups.
    *out = taps;
    out->nchunk = 0;
    groups->n = 0;
    int t = 0;
    long win_max = 0;
    while (t < taps.n) {
        int u = t + 1;
        while (u < taps.n && u - t < mfmak::kMaxG * mfmak::kGS &&
               (chunk_cap <= 0 || u - t < chunk_cap) &&
               mfmak::kPwg + (long)(taps.s[t] - taps.s[u]) * NN <= mfmak::kPlaneWords)
            ++u;
        groups->gb[out->nchunk] = groups->n;
        for (int g = t; g < u; g += mfmak::kGS)
            groups->t0[groups->n++] = g;
        out->cb[out->nchunk++] = t;
        win_max = std::max(win_max, (long)(TE + taps.s[t] - taps.s[u - 1]) * NN);
        t = u;
    }
    out->cb[out->nchunk] = taps.n;
    groups->gb[out->nchunk] = groups->n;
    TileGeom g;
    g.TE = TE;
    g.n_etiles = (NE + TE - 1) / TE;
    g.lds_win = (int)win_max;
    g.lds_bytes = 0;  // static LDS: two window buffers and the sandwich region
    return g;
}

size_t mfma_afrag_bytes(int, int NA, int NB, int Nqz, const GroupTable &g)
{
    return (size_t)NA * NB * Nqz * g.n * 64 * 32;
}

size_t mfma_split_offset(int prec, int NA, int NB, int Nqz, const GroupTable &g)
{
    return (mfmak::kZeroPage + mfma_afrag_bytes(prec, NA, NB, Nqz, g) + 255) & ~(size_t)255;
}

size_t mfma_aux_bytes(int prec, int NA, int NB, int Nqz, int Nkz, int NE, int Norb,
                      const GroupTable &g)
{
    size_t b = mfma_split_offset(prec, NA, NB, Nqz, g);
    if (prec == SSE_BF16X3)
        b += (size_t)Nkz * NE * NA * Norb * Norb * 8;
    return b;
}

// Geometry of the phonon kernel (sse_pi.hip): the most neighbours per
// workgroup (up to 4) whose buffers leave room for a ring of the taps' rows,
// then the taps, sorted by increasing shift, cut into chunks of at most 32
// whose ring fits.  LDS per workgroup: ring R + 2 rows (a step's R rows, a
// spare for the next step's top row, a zero row) of NNp (the pairs padded to an
// even count) complex128 values; Zb NNp rows of 16 ntn binary64 columns;
// per neighbour U (3 blocks) and Y (1 block) complex128 and dH (3 blocks) binary64.
PiGeom pi_geometry(int Norb, int NB, const int32_t *w_shift, int Nw)
{
    PiGeom gm{};
    const size_t NN = (size_t)Norb * Norb, NNp = NN + (NN & 1);
    std::vector<int> order(Nw);
    for (int w = 0; w < Nw; ++w)
        order[w] = w;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return w_shift[x] < w_shift[y]; });
    for (int t = 0; t < Nw; ++t) {
        gm.tw[t] = order[t];
        gm.ts[t] = w_shift[order[t]];
    }
    auto ntn_of = [](int nbw) { return (nbw * 9 * 2 + 15) / 16; };
    auto fixed_of = [&](int nbw) {
        return 2 * NNp * 16 + NNp * 16 * ntn_of(nbw) * 8 + (size_t)nbw * NN * (3 * 16 + 16 + 3 * 8);
    };
    const size_t per_row = NNp * 16;
    const size_t budget = pik::kLdsBudgetOne;
    const int want_rows = std::min(gm.ts[Nw - 1] - gm.ts[0] + 1, 8);
    int rmax = 0;
    for (gm.nbw = std::min(NB, pik::kMaxNbw); gm.nbw >= 1; --gm.nbw) {
        const size_t fixed = fixed_of(gm.nbw);
        rmax = fixed < budget ? (int)((budget - fixed) / per_row) : 0;
        if (rmax >= want_rows || gm.nbw == 1)
            break;
    }
    gm.R = 0;
    gm.nchunk = 0;
    int maxtaps = 0;
    int t = 0;
    while (t < Nw && rmax >= 1) {
        int e = t + 1;
        while (e < Nw && e - t < pik::kMaxChunkTaps && gm.ts[e] - gm.ts[t] + 1 <= rmax)
            ++e;
        gm.cb[gm.nchunk] = t;
        gm.R = std::max(gm.R, gm.ts[e - 1] - gm.ts[t] + 1);
        maxtaps = std::max(maxtaps, e - t);
        ++gm.nchunk;
        t = e;
    }
    gm.cb[gm.nchunk] = Nw;
    gm.mtiles = maxtaps <= 16 ? 1 : 2;
    // the final reduction reuses LDS for half the waves' accumulator tiles
    gm.lds_bytes = std::max((size_t)gm.R * per_row + fixed_of(gm.nbw),
                            (size_t)(pik::kWaves / 2) * 16 * gm.mtiles * 16 * ntn_of(gm.nbw) * 8);
    gm.ok = rmax >= 1 && gm.lds_bytes <= budget;
    return gm;
}

}  // namespace sse
