/*
 * pi_oracle.c -- ORACLE.  Test infrastructure only: the plain, slow, obviously
 * correct CPU evaluation of the phonon scattering self-energy against which the
 * GPU kernel is checked.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load it; nothing in the product calls it, and it shares
 * no code with the GPU path.
 *
 * What it computes: Eqs. (4) and (5) of Ziogas et al., SC'19 (Sec. 2), the
 * lesser/greater phonon scattering self-energy in the layout of the phonon
 * Green's function (Sec. 2: [Nqz, Nw, NA, NB + 1, N3D, N3D] -- the NB
 * neighbour blocks and the diagonal block of each atom).  For frequency w,
 * momentum q, atom a and neighbour slot b (f = neigh[a, b]),
 *
 *   P[q, w, a, b, i, j] = sum_k sum_e tr( dH_ba,i . X[(k + q) mod Nkz, e + s_w, a]
 *                                         . dH_ab,j . Y[k, e, f] )
 *
 *   Pi[q, w, a, b,  i, j] =  beta * P[q, w, a, b, i, j]          (Eq. (5), beta = i)
 *   Pi[q, w, a, NB, i, j] = -beta * sum_b P[q, w, a, b, i, j]    (Eq. (4), the diagonal)
 *
 * where X and Y are the electron Green's functions of the two opposite
 * components: Pi< takes X = G<, Y = G>; Pi> takes X = G>, Y = G<.  Readings
 * where the paper is silent or garbled:
 *   - dH_ba is the transpose of the stored dH_ab (real H), dH_ab,j = dH[a, b, j];
 *   - beta = i, the prefactor of Eq. (5); Eq. (4) carries -i and sums the same
 *     trace over the neighbours l of a; the energy measure is folded in;
 *   - E + hbar*omega is e + s_w for the integer shift table s of the Sigma
 *     kernel; terms whose energy index leaves [0, NE) contribute zero;
 *   - kz + qz is periodic: index (k + q) mod Nkz;
 *   - the diagonal block is stored in neighbour slot NB.
 * Arithmetic: binary64; the sum runs over k, then e; for each term the product
 * is formed as ((dH_ab,i^T . X) . dH_ab,j) and its trace with Y as
 * sum_m sum_l T[m][l] Y[l][m]; the diagonal sums P over b in order.
 *
 * Layouts: row-major, complex interleaved (re, im): neigh int32 [NA, NB];
 * dH [NA, NB, N3D, Norb, Norb]; X, Y [Nkz, NE, NA, Norb, Norb] -- or, when
 * gslot is given, stacks of blocks with gslot[(k * NE + e) * NA + atom] naming a
 * block's slot in both stacks (-1 = absent, an error if it is needed);
 * out [nblk, NB + 1, N3D, N3D].
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

typedef struct {
    int NA, NB, Norb, N3D, Nkz, Nqz, NE, Nw;
} pi_dims;

static const double *block_at(const pi_dims *d, const double *T, const int64_t *gslot, int k,
                              int e, int atom, int *missing)
{
    const int64_t flat = ((int64_t)k * d->NE + e) * d->NA + atom;
    const size_t nn2 = (size_t)d->Norb * d->Norb * 2;
    if (!gslot)
        return T + (size_t)flat * nn2;
    if (gslot[flat] < 0) {
        *missing = 1;
        return NULL;
    }
    return T + (size_t)gslot[flat] * nn2;
}

/* One output block Pi[q, w, a] (NB + 1 blocks of N3D x N3D); returns 1 if a
 * needed G block is absent. */
static int pi_block(const pi_dims *d, const int32_t *shift, const int32_t *neigh, const double *dH,
                    const double *X, const double *Y, const int64_t *gslot, double beta_re,
                    double beta_im, int q, int w, int a, double *out)
{
    const int No = d->Norb, nn = No * No, N3 = d->N3D, NB = d->NB;
    double *P = calloc((size_t)NB * N3 * N3 * 2, sizeof(double));
    double *t1 = malloc((size_t)nn * 2 * sizeof(double)); /* dH_i^T . X    */
    double *t2 = malloc((size_t)nn * 2 * sizeof(double)); /* t1 . dH_j     */
    int missing = 0;

    for (int b = 0; b < NB; ++b) {
        const int f = neigh[(size_t)a * NB + b];
        double *Pb = P + (size_t)b * N3 * N3 * 2;
        for (int k = 0; k < d->Nkz; ++k) {
            const int kk = (k + q) % d->Nkz;
            for (int e = 0; e < d->NE; ++e) {
                const int ee = e + shift[w];
                if (ee < 0 || ee >= d->NE)
                    continue;
                const double *x = block_at(d, X, gslot, kk, ee, a, &missing);
                const double *y = block_at(d, Y, gslot, k, e, f, &missing);
                if (!x || !y)
                    continue;
                for (int i = 0; i < N3; ++i) {
                    const double *Ai = dH + (((size_t)a * NB + b) * N3 + i) * nn;
                    /* t1 = A_i^T . X, i.e. t1[m][n] = sum_l A_i[l][m] X[l][n] */
                    for (int m = 0; m < No; ++m)
                        for (int n = 0; n < No; ++n) {
                            double sr = 0.0, si = 0.0;
                            for (int l = 0; l < No; ++l) {
                                sr += Ai[l * No + m] * x[2 * (l * No + n)];
                                si += Ai[l * No + m] * x[2 * (l * No + n) + 1];
                            }
                            t1[2 * (m * No + n)] = sr;
                            t1[2 * (m * No + n) + 1] = si;
                        }
                    for (int j = 0; j < N3; ++j) {
                        const double *Aj = dH + (((size_t)a * NB + b) * N3 + j) * nn;
                        /* t2 = t1 . A_j */
                        for (int m = 0; m < No; ++m)
                            for (int n = 0; n < No; ++n) {
                                double sr = 0.0, si = 0.0;
                                for (int l = 0; l < No; ++l) {
                                    sr += t1[2 * (m * No + l)] * Aj[l * No + n];
                                    si += t1[2 * (m * No + l) + 1] * Aj[l * No + n];
                                }
                                t2[2 * (m * No + n)] = sr;
                                t2[2 * (m * No + n) + 1] = si;
                            }
                        /* tr(t2 . Y) = sum_m sum_l t2[m][l] Y[l][m] */
                        double tr = 0.0, ti = 0.0;
                        for (int m = 0; m < No; ++m)
                            for (int l = 0; l < No; ++l) {
                                const double ar = t2[2 * (m * No + l)], ai = t2[2 * (m * No + l) + 1];
                                const double br = y[2 * (l * No + m)], bi = y[2 * (l * No + m) + 1];
                                tr += ar * br - ai * bi;
                                ti += ar * bi + ai * br;
                            }
                        Pb[2 * (i * N3 + j)] += tr;
                        Pb[2 * (i * N3 + j) + 1] += ti;
                    }
                }
            }
        }
    }
    for (int b = 0; b < NB; ++b)
        for (int x = 0; x < N3 * N3; ++x) {
            const double r = P[2 * ((size_t)b * N3 * N3 + x)], im = P[2 * ((size_t)b * N3 * N3 + x) + 1];
            out[2 * ((size_t)b * N3 * N3 + x)] = beta_re * r - beta_im * im;
            out[2 * ((size_t)b * N3 * N3 + x) + 1] = beta_re * im + beta_im * r;
        }
    for (int x = 0; x < N3 * N3; ++x) {
        double r = 0.0, im = 0.0;
        for (int b = 0; b < NB; ++b) {
            r += P[2 * ((size_t)b * N3 * N3 + x)];
            im += P[2 * ((size_t)b * N3 * N3 + x) + 1];
        }
        out[2 * ((size_t)NB * N3 * N3 + x)] = -(beta_re * r - beta_im * im);
        out[2 * ((size_t)NB * N3 * N3 + x) + 1] = -(beta_re * im + beta_im * r);
    }
    free(P);
    free(t1);
    free(t2);
    return missing;
}

/*
 * Pi for a list of nblk output blocks blk[3t..3t+2] = (q, w, a); blk == NULL
 * means every block of [Nqz, Nw, NA] in row-major order.  Returns 0 on success,
 * 1 if an input index is out of range, 2 if a needed G block is absent.
 * Output blocks are independent and spread over nthreads OpenMP threads
 * (0 = the runtime's default); the arithmetic of each is the same.
 */
int pi_oracle(int NA, int NB, int Norb, int N3D, int Nkz, int Nqz, int NE, int Nw,
              const int32_t *shift, const int32_t *neigh, const double *dH, const double *X,
              const double *Y, const int64_t *gslot, double beta_re, double beta_im, int64_t nblk,
              const int32_t *blk, double *out, int nthreads)
{
    const pi_dims d = {NA, NB, Norb, N3D, Nkz, Nqz, NE, Nw};
    for (int64_t t = 0; t < (int64_t)NA * NB; ++t)
        if (neigh[t] < 0 || neigh[t] >= NA)
            return 1;
    if (blk == NULL)
        nblk = (int64_t)Nqz * Nw * NA;
    for (int64_t t = 0; blk && t < nblk; ++t)
        if (blk[3 * t] < 0 || blk[3 * t] >= Nqz || blk[3 * t + 1] < 0 || blk[3 * t + 1] >= Nw ||
            blk[3 * t + 2] < 0 || blk[3 * t + 2] >= NA)
            return 1;
    int missing = 0;
    const size_t per = (size_t)(NB + 1) * N3D * N3D * 2;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) reduction(| : missing) num_threads(nthreads)
    for (int64_t t = 0; t < nblk; ++t) {
        int q, w, a;
        if (blk) {
            q = blk[3 * t];
            w = blk[3 * t + 1];
            a = blk[3 * t + 2];
        } else {
            q = (int)(t / ((int64_t)Nw * NA));
            w = (int)((t / NA) % Nw);
            a = (int)(t % NA);
        }
        missing |= pi_block(&d, shift, neigh, dH, X, Y, gslot, beta_re, beta_im, q, w, a,
                            out + (size_t)t * per);
    }
    return missing ? 2 : 0;
}
