// Host-side check of the phonon kernel's geometry (pi_geometry) against the
// kernel's LDS layout and task mapping, over orbital counts, neighbour counts,
// frequency counts and shift tables: every accepted geometry must fit the LDS
// it reserves, every tap chunk must fit the ring, and every wave's second-round
// tasks must fit two per lane.  Exits non-zero at the first violation.
#include <cstdio>
#include <vector>

#include "sse_internal.h"

using namespace sse;

static int fail(const char *what, int Norb, int NB, int Nw, int pattern)
{
    std::printf("FAIL %s: Norb=%d NB=%d Nw=%d pattern=%d\n", what, Norb, NB, Nw, pattern);
    return 1;
}

int main()
{
    const int nws[] = {1, 2, 3, 7, 16, 17, 30, 32, 33, 64, 100, 128};
    long checked = 0, refused = 0;
    for (int Norb = 1; Norb <= pik::kMaxNorb; ++Norb)
        for (int NB = 1; NB <= 9; ++NB)
            for (int Nw : nws)
                for (int pattern = 0; pattern < 4; ++pattern) {
                    std::vector<int32_t> s(Nw);
                    for (int w = 0; w < Nw; ++w) {
                        if (pattern == 0)
                            s[w] = w + 1;                      // contiguous, positive
                        else if (pattern == 1)
                            s[w] = w - Nw / 2;                 // contiguous, both signs
                        else if (pattern == 2)
                            s[w] = 3 * w - 40;                 // spread 3 (Nw - 1)
                        else
                            s[w] = ((w * 37) % Nw) - Nw / 3;   // unsorted permutation
                    }
                    const PiGeom g = pi_geometry(Norb, NB, s.data(), Nw);
                    if (!g.ok) {
                        ++refused;
                        continue;
                    }
                    ++checked;
                    const size_t NN = (size_t)Norb * Norb, NNp = NN + (NN & 1);
                    const size_t ntn = (size_t)(g.nbw * kNF * 2 + 15) / 16;
                    // the kernel's layout: ring (R + 2 rows), Zb, U, Y, dH
                    const size_t layout = (size_t)(g.R + 2) * NNp * 16 + NNp * 16 * ntn * 8 +
                                          (size_t)g.nbw * NN * (3 * 16 + 16 + 3 * 8);
                    const size_t reduction =
                        (size_t)(pik::kWaves / 2) * 16 * g.mtiles * 16 * ntn * 8;
                    if (layout > g.lds_bytes || reduction > g.lds_bytes ||
                        g.lds_bytes > pik::kLdsBudgetOne)
                        return fail("lds", Norb, NB, Nw, pattern);
                    if (g.nbw < 1 || g.nbw > NB || g.nbw > pik::kMaxNbw)
                        return fail("nbw", Norb, NB, Nw, pattern);
                    if (g.nchunk < 1 || g.cb[0] != 0 || g.cb[g.nchunk] != Nw)
                        return fail("chunks", Norb, NB, Nw, pattern);
                    for (int c = 0; c < g.nchunk; ++c) {
                        const int t0 = g.cb[c], t1 = g.cb[c + 1];
                        if (t1 <= t0 || t1 - t0 > 16 * g.mtiles)
                            return fail("chunk size", Norb, NB, Nw, pattern);
                        if (g.ts[t1 - 1] - g.ts[t0] + 1 > g.R)
                            return fail("ring", Norb, NB, Nw, pattern);
                        for (int t = t0 + 1; t < t1; ++t)
                            if (g.ts[t] < g.ts[t - 1])
                                return fail("order", Norb, NB, Nw, pattern);
                    }
                    // every frequency appears once, with its own shift
                    std::vector<int> seen(Nw, 0);
                    for (int t = 0; t < Nw; ++t) {
                        if (g.tw[t] < 0 || g.tw[t] >= Nw || seen[g.tw[t]]++ ||
                            g.ts[t] != s[g.tw[t]])
                            return fail("taps", Norb, NB, Nw, pattern);
                    }
                    // first sandwich round: at most two tasks per thread, dealt over the waves
                    const size_t per_wave = (g.nbw * NN + pik::kWaves - 1) / pik::kWaves;
                    if (per_wave > 128)
                        return fail("first-round tasks", Norb, NB, Nw, pattern);
                    // second sandwich round: the rows a wave's MFMA steps read, times nbw
                    for (int w = 0; w < pik::kWaves; ++w) {
                        size_t rows = 0;
                        for (size_t c = 0; c < NN; ++c)
                            if ((c >> 1) % pik::kWaves == (size_t)w)
                                ++rows;
                        if (rows * g.nbw > 128)
                            return fail("second-round tasks", Norb, NB, Nw, pattern);
                    }
                }
    std::printf("OK %ld geometries checked, %ld refused\n", checked, refused);
    return checked > 0 ? 0 : 1;
}
