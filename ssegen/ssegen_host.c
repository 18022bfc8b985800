/*
 * ssegen_host.c -- host side of the seeded input generator (see ssegen_core.h).
 *
 * Layouts are those of the self-energy kernel's arguments, row-major, complex
 * values interleaved (re, im):
 *   neigh [NA, NB]                   int32, NB distinct atoms != a per row
 *   dH    [NA, NB, N3D, Norb, Norb]  real N(0,1)
 *   G     [Nkz, NE, NA, Norb, Norb]  complex, each Norb x Norb block anti-Hermitian
 *   D     [Nqz, Nw, NA, NB, N3D, N3D] complex, each 3 x 3 block anti-Hermitian
 * G may be produced for a list of blocks only (flat block index
 * (k * NE + e) * NA + a), which is how large problems are sampled on the host.
 */
#include "ssegen_core.h"

#include <math.h>
#include <stddef.h>
#include <stdint.h>

int ssegen_host_neigh(uint64_t seed, int NA, int NB, int32_t *out)
{
    if (NA < 2 || NB < 1 || NB > NA - 1)
        return 1;
    for (int a = 0; a < NA; ++a) {
        int32_t *row = out + (size_t)a * NB;
        int have = 0;
        for (uint32_t t = 0; have < NB; ++t) {
            ssegen_u4 x = ssegen_philox((uint32_t)a, 0u, SSEGEN_S_NEIGH, t, (uint32_t)seed,
                                        (uint32_t)(seed >> 32));
            for (int s = 0; s < 4 && have < NB; ++s) {
                int32_t c = (int32_t)(((uint64_t)x.w[s] * (uint64_t)(NA - 1)) >> 32);
                if (c >= a)
                    c += 1; /* skip self */
                int dup = 0;
                for (int u = 0; u < have; ++u)
                    dup |= (row[u] == c);
                if (!dup)
                    row[have++] = c;
            }
        }
    }
    return 0;
}

void ssegen_host_dH(uint64_t seed, int64_t n, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = ssegen_normal(seed, (uint64_t)i, SSEGEN_S_DH, 0);
}

/* Anti-Hermitian G blocks for the listed flat block indices. */
void ssegen_host_G_blocks(uint64_t seed, int comp, int Norb, int scaled, int64_t nblk,
                          const int64_t *blk, double *out)
{
    const int nn = Norb * Norb;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nblk; ++t) {
        uint64_t B = (uint64_t)blk[t];
        double s = scaled ? ssegen_block_scale(seed, B, SSEGEN_S_GSCALE + comp) : 1.0;
        double *o = out + (size_t)t * nn * 2;
        for (int m = 0; m < Norb; ++m)
            for (int n = 0; n < Norb; ++n) {
                double re, im;
                ssegen_antiherm(seed, B * nn, Norb, m, n, SSEGEN_S_G + comp, &re, &im);
                o[2 * (m * Norb + n)] = re * s;
                o[2 * (m * Norb + n) + 1] = im * s;
            }
    }
}

/* All anti-Hermitian 3x3 (N3D x N3D) D~ blocks, nblk = Nqz * Nw * NA * NB. */
void ssegen_host_D(uint64_t seed, int comp, int N3D, int64_t nblk, double *out)
{
    const int nn = N3D * N3D;
#pragma omp parallel for schedule(static)
    for (int64_t B = 0; B < nblk; ++B) {
        double *o = out + (size_t)B * nn * 2;
        for (int i = 0; i < N3D; ++i)
            for (int j = 0; j < N3D; ++j) {
                double re, im;
                ssegen_antiherm(seed, (uint64_t)B * nn, N3D, i, j, SSEGEN_S_D + comp, &re, &im);
                o[2 * (i * N3D + j)] = re;
                o[2 * (i * N3D + j) + 1] = im;
            }
    }
}

/* Perturbation standing in for one Green's-function update:
 *   X <- X + 0.01 * (|X|_F / |N|_F) * N
 * with N a fresh anti-Hermitian complex-normal block keyed by (seed,
 * iteration, stream).  blk holds the flat block index of each listed block
 * (it keys N), data the blocks themselves (n_side x n_side complex). */
void ssegen_host_perturb(uint64_t seed, int iteration, uint32_t stream, int n_side, int64_t nblk,
                         const int64_t *blk, double *data)
{
    const int nn = n_side * n_side;
    const uint32_t st = stream | ((uint32_t)(iteration + 1) << 8);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nblk; ++t) {
        double *x = data + (size_t)t * nn * 2;
        uint64_t base = (uint64_t)blk[t] * nn;
        double nx = 0.0, nr = 0.0;
        for (int e = 0; e < nn; ++e) {
            double re, im;
            ssegen_antiherm(seed, base, n_side, e / n_side, e % n_side, st, &re, &im);
            nx = nx + (x[2 * e] * x[2 * e] + x[2 * e + 1] * x[2 * e + 1]);
            nr = nr + (re * re + im * im);
        }
        double f = nr > 0.0 ? 0.01 * (sqrt(nx) / sqrt(nr)) : 0.0;
        for (int e = 0; e < nn; ++e) {
            double re, im;
            ssegen_antiherm(seed, base, n_side, e / n_side, e % n_side, st, &re, &im);
            x[2 * e] = x[2 * e] + f * re;
            x[2 * e + 1] = x[2 * e + 1] + f * im;
        }
    }
}

/* Raw Philox block, exported for the known-answer test. */
void ssegen_host_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    ssegen_u4 x = ssegen_philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    for (int i = 0; i < 4; ++i)
        out[i] = x.w[i];
}

double ssegen_host_normal(uint64_t seed, uint64_t idx, uint32_t stream)
{
    return ssegen_normal(seed, idx, stream, 0);
}
