/*
 * Drives the two C oracles (Sigma of Eq. (3), Pi of Eqs. (4)-(5)) through
 * every path they have, for a build under AddressSanitizer and UBSan with
 * OpenMP: the full evaluation, a block list in scrambled order, the gslot
 * (stacked blocks) path, an absent needed block, and out-of-range neighbour
 * and block indices.  A block-list or gslot result must equal the full
 * evaluation's bit for bit (each block's arithmetic does not depend on how
 * the blocks are listed).  Exits non-zero at the first mismatch.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int sse_oracle(int NA, int NB, int Norb, int N3D, int Nkz, int Nqz, int NE, int Nw,
               const int32_t *shift, const int32_t *neigh, const double *dH, const double *G,
               const int64_t *gslot, const double *Dt, double alpha_re, double alpha_im,
               int64_t nblk, const int32_t *blk, double *out, int nthreads);
int pi_oracle(int NA, int NB, int Norb, int N3D, int Nkz, int Nqz, int NE, int Nw,
              const int32_t *shift, const int32_t *neigh, const double *dH, const double *X,
              const double *Y, const int64_t *gslot, double beta_re, double beta_im, int64_t nblk,
              const int32_t *blk, double *out, int nthreads);

enum { NA = 4, NB = 3, NO = 3, N3 = 3, NK = 3, NQ = 3, NE = 5, NW = 3 };

static uint64_t state = 0x9e3779b97f4a7c15ull;

static double uniform(void)
{
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

static double *random_array(size_t n)
{
    double *p = malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i)
        p[i] = uniform();
    return p;
}

static int fail(const char *what)
{
    printf("FAIL %s\n", what);
    return 1;
}

int main(void)
{
    const int32_t shift[NW] = {1, -2, 0};
    int32_t neigh[NA * NB];
    for (int a = 0; a < NA; ++a)
        for (int b = 0; b < NB; ++b)
            neigh[a * NB + b] = (a + b + 1) % NA; /* includes a self-neighbour (a = 3, b = 0) */
    const size_t nn2 = (size_t)NO * NO * 2;
    const size_t ngblk = (size_t)NK * NE * NA;
    double *dH = random_array((size_t)NA * NB * N3 * nn2);
    double *G = random_array(ngblk * nn2);
    double *G2 = random_array(ngblk * nn2);
    double *Dt = random_array((size_t)NQ * NW * NA * NB * N3 * N3 * 2);

    /* stacked copy of G: block t of [Nkz, NE, NA] in slot ngblk - 1 - t */
    int64_t *gslot = malloc(ngblk * sizeof(int64_t));
    double *Gs = malloc(ngblk * nn2 * sizeof(double));
    double *G2s = malloc(ngblk * nn2 * sizeof(double));
    for (size_t t = 0; t < ngblk; ++t) {
        gslot[t] = (int64_t)(ngblk - 1 - t);
        memcpy(Gs + (ngblk - 1 - t) * nn2, G + t * nn2, nn2 * sizeof(double));
        memcpy(G2s + (ngblk - 1 - t) * nn2, G2 + t * nn2, nn2 * sizeof(double));
    }

    /* Sigma: full, block list, gslot, absent block, bad indices */
    const size_t nsig = ngblk;
    double *full = malloc(nsig * nn2 * sizeof(double));
    if (sse_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, NULL, Dt, 0.0, 1.0, 0,
                   NULL, full, 2) != 0)
        return fail("sigma full");
    int32_t blk[3 * 7];
    const int pick[7] = {59, 0, 17, 31, 44, 3, 52};
    for (int t = 0; t < 7; ++t) {
        blk[3 * t] = pick[t] / (NE * NA);
        blk[3 * t + 1] = (pick[t] / NA) % NE;
        blk[3 * t + 2] = pick[t] % NA;
    }
    double *part = malloc(7 * nn2 * sizeof(double));
    if (sse_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, NULL, Dt, 0.0, 1.0, 7, blk,
                   part, 3) != 0)
        return fail("sigma block list");
    for (int t = 0; t < 7; ++t)
        if (memcmp(part + t * nn2, full + (size_t)pick[t] * nn2, nn2 * sizeof(double)))
            return fail("sigma block list differs from the full evaluation");
    double *viaslot = malloc(nsig * nn2 * sizeof(double));
    if (sse_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, Gs, gslot, Dt, 0.0, 1.0, 0,
                   NULL, viaslot, 2) != 0)
        return fail("sigma gslot");
    if (memcmp(viaslot, full, nsig * nn2 * sizeof(double)))
        return fail("sigma gslot differs from the full evaluation");
    gslot[17] = -1;
    if (sse_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, Gs, gslot, Dt, 0.0, 1.0, 0,
                   NULL, viaslot, 2) != 2)
        return fail("sigma absent block not reported");
    gslot[17] = (int64_t)(ngblk - 1 - 17);
    neigh[5] = NA;
    if (sse_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, NULL, Dt, 0.0, 1.0, 0,
                   NULL, full, 2) != 1)
        return fail("sigma neighbour out of range not reported");
    neigh[5] = (1 + 2 + 1) % NA;
    blk[3 * 2 + 1] = NE;
    if (sse_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, NULL, Dt, 0.0, 1.0, 7, blk,
                   part, 2) != 1)
        return fail("sigma block out of range not reported");

    /* Pi: full, block list, gslot, absent block, bad indices */
    const size_t npi = (size_t)NQ * NW * NA, per = (size_t)(NB + 1) * N3 * N3 * 2;
    double *pfull = malloc(npi * per * sizeof(double));
    if (pi_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, G2, NULL, 0.0, 1.0, 0, NULL,
                  pfull, 2) != 0)
        return fail("pi full");
    int32_t pblk[3 * 5];
    const int ppick[5] = {35, 2, 20, 9, 27};
    for (int t = 0; t < 5; ++t) {
        pblk[3 * t] = ppick[t] / (NW * NA);
        pblk[3 * t + 1] = (ppick[t] / NA) % NW;
        pblk[3 * t + 2] = ppick[t] % NA;
    }
    double *ppart = malloc(5 * per * sizeof(double));
    if (pi_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, G2, NULL, 0.0, 1.0, 5, pblk,
                  ppart, 3) != 0)
        return fail("pi block list");
    for (int t = 0; t < 5; ++t)
        if (memcmp(ppart + t * per, pfull + (size_t)ppick[t] * per, per * sizeof(double)))
            return fail("pi block list differs from the full evaluation");
    double *pslot = malloc(npi * per * sizeof(double));
    if (pi_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, Gs, G2s, gslot, 0.0, 1.0, 0,
                  NULL, pslot, 2) != 0)
        return fail("pi gslot");
    if (memcmp(pslot, pfull, npi * per * sizeof(double)))
        return fail("pi gslot differs from the full evaluation");
    gslot[40] = -1;
    if (pi_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, Gs, G2s, gslot, 0.0, 1.0, 0,
                  NULL, pslot, 2) != 2)
        return fail("pi absent block not reported");
    neigh[0] = -1;
    if (pi_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, G2, NULL, 0.0, 1.0, 0, NULL,
                  pfull, 2) != 1)
        return fail("pi neighbour out of range not reported");
    neigh[0] = 1;
    pblk[3 * 4 + 1] = -1;
    if (pi_oracle(NA, NB, NO, N3, NK, NQ, NE, NW, shift, neigh, dH, G, G2, NULL, 0.0, 1.0, 5, pblk,
                  ppart, 2) != 1)
        return fail("pi block out of range not reported");

    free(dH);
    free(G);
    free(G2);
    free(Dt);
    free(gslot);
    free(Gs);
    free(G2s);
    free(full);
    free(part);
    free(viaslot);
    free(pfull);
    free(ppart);
    free(pslot);
    printf("OK both oracles, every path\n");
    return 0;
}
