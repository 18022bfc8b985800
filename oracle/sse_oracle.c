/*
 * sse_oracle.c -- ORACLE.  Test infrastructure only: the plain, slow,
 * obviously correct CPU evaluation of the electron scattering self-energy
 * against which the GPU kernels are checked.  Only the tests, the smoke check
 * and the CPU-baseline leg of the benchmark load it; nothing in the product
 * calls it, and it shares no code with the GPU path.
 *
 * What it computes: Eq. (3) of Ziogas et al., SC'19 (Sec. 2), the diagonal
 * block of the lesser/greater electron scattering self-energy,
 *
 *   Sigma[k, e, a] = alpha * sum_b sum_q sum_w sum_i sum_j
 *        Dt[q, w, a, b, i, j] * ( dH[a, b, i] . G[(k - q) mod Nkz, e - s_w, f(a,b)] . dH[a, b, j]^T )
 *
 * with f(a, b) = neigh[a, b] (the neighbour indirection of Sec. 4.1), Dt the
 * phonon Green's function already combined as D_ba - D_bb - D_aa + D_ab
 * (Eq. (3); Sec. 4.2 lists it as a kernel input), the tensor shapes of the
 * typed program signature in Sec. 3, and these readings where the paper is
 * silent or garbled:
 *   - the back-bond derivative dH_ba is the transpose of dH_ab (real H);
 *   - alpha = i, the prefactor of Eq. (3), with the energy measure folded in;
 *   - the energy argument E - hbar*omega is e - s_w for an integer shift table
 *     s (s_w = w + 1 on a uniform grid); terms whose energy index leaves
 *     [0, NE) contribute zero;
 *   - kz - qz is periodic: index (k - q) mod Nkz;
 *   - the neighbour slot b is the summation index written l in Eq. (3);
 *   - the result overwrites Sigma.
 * Arithmetic: binary64, summation in the order b, q, w, i, j; for each term
 * the triple product is formed as (dH_i . G) . dH_j^T.
 *
 * Layouts: row-major, complex interleaved (re, im):
 *   neigh int32 [NA, NB]; dH [NA, NB, N3D, Norb, Norb]; Dt [Nqz, Nw, NA, NB, N3D, N3D];
 *   G [Nkz, NE, NA, Norb, Norb] -- or, when gslot is given, a list of blocks
 *   with gslot[(k * NE + e) * NA + a] naming the block's slot (-1 = absent, an error
 *   if it is needed);  out [nblk, Norb, Norb].
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

typedef struct {
    int NA, NB, Norb, N3D, Nkz, Nqz, NE, Nw;
} oracle_dims;

/* One output block Sigma[k, e, a]; returns 0, or 1 if a needed G block is absent. */
static int sigma_block(const oracle_dims *d, const int32_t *shift, const int32_t *neigh,
                       const double *dH, const double *G, const int64_t *gslot, const double *Dt,
                       double alpha_re, double alpha_im, int k, int e, int a, double *out)
{
    const int No = d->Norb, nn = No * No, N3 = d->N3D;
    double *acc = calloc((size_t)nn * 2, sizeof(double));
    double *t1 = malloc((size_t)nn * 2 * sizeof(double)); /* dH_i . G      */
    double *t2 = malloc((size_t)nn * 2 * sizeof(double)); /* t1 . dH_j^T   */
    int missing = 0;

    for (int b = 0; b < d->NB; ++b) {
        const int f = neigh[(size_t)a * d->NB + b];
        for (int q = 0; q < d->Nqz; ++q) {
            const int kk = ((k - q) % d->Nkz + d->Nkz) % d->Nkz;
            for (int w = 0; w < d->Nw; ++w) {
                const int ee = e - shift[w];
                if (ee < 0 || ee >= d->NE)
                    continue;
                const int64_t bidx = ((int64_t)kk * d->NE + ee) * d->NA + f;
                const double *g;
                if (gslot) {
                    const int64_t s = gslot[bidx];
                    if (s < 0) {
                        missing = 1;
                        continue;
                    }
                    g = G + (size_t)s * nn * 2;
                } else {
                    g = G + (size_t)bidx * nn * 2;
                }
                for (int i = 0; i < N3; ++i) {
                    const double *Ai = dH + (((size_t)a * d->NB + b) * N3 + i) * nn;
                    /* t1 = A_i . G */
                    for (int m = 0; m < No; ++m)
                        for (int n = 0; n < No; ++n) {
                            double sr = 0.0, si = 0.0;
                            for (int l = 0; l < No; ++l) {
                                sr += Ai[m * No + l] * g[2 * (l * No + n)];
                                si += Ai[m * No + l] * g[2 * (l * No + n) + 1];
                            }
                            t1[2 * (m * No + n)] = sr;
                            t1[2 * (m * No + n) + 1] = si;
                        }
                    for (int j = 0; j < N3; ++j) {
                        const double *Aj = dH + (((size_t)a * d->NB + b) * N3 + j) * nn;
                        /* t2 = t1 . A_j^T, i.e. t2[m][n] = sum_l t1[m][l] * A_j[n][l] */
                        for (int m = 0; m < No; ++m)
                            for (int n = 0; n < No; ++n) {
                                double sr = 0.0, si = 0.0;
                                for (int l = 0; l < No; ++l) {
                                    sr += t1[2 * (m * No + l)] * Aj[n * No + l];
                                    si += t1[2 * (m * No + l) + 1] * Aj[n * No + l];
                                }
                                t2[2 * (m * No + n)] = sr;
                                t2[2 * (m * No + n) + 1] = si;
                            }
                        /* acc += Dt[q, w, a, b, i, j] * t2 */
                        const size_t di =
                            (((((size_t)q * d->Nw + w) * d->NA + a) * d->NB + b) * N3 + i) * N3 + j;
                        const double dr = Dt[2 * di], dim = Dt[2 * di + 1];
                        for (int x = 0; x < nn; ++x) {
                            const double tr = t2[2 * x], ti = t2[2 * x + 1];
                            acc[2 * x] += dr * tr - dim * ti;
                            acc[2 * x + 1] += dr * ti + dim * tr;
                        }
                    }
                }
            }
        }
    }
    for (int x = 0; x < nn; ++x) {
        const double r = acc[2 * x], im = acc[2 * x + 1];
        out[2 * x] = alpha_re * r - alpha_im * im;
        out[2 * x + 1] = alpha_re * im + alpha_im * r;
    }
    free(acc);
    free(t1);
    free(t2);
    return missing;
}

/*
 * Sigma for a list of nblk output blocks blk[3t..3t+2] = (k, e, a); blk == NULL
 * means every block of [Nkz, NE, NA] in row-major order.  Returns 0 on success,
 * 1 if an input index is out of range, 2 if a needed G block is absent.
 * Output blocks are independent, so they are spread over nthreads OpenMP
 * threads (0 = the runtime's default); the arithmetic of each is the same.
 */
int sse_oracle(int NA, int NB, int Norb, int N3D, int Nkz, int Nqz, int NE, int Nw,
               const int32_t *shift, const int32_t *neigh, const double *dH, const double *G,
               const int64_t *gslot, const double *Dt, double alpha_re, double alpha_im,
               int64_t nblk, const int32_t *blk, double *out, int nthreads)
{
    const oracle_dims d = {NA, NB, Norb, N3D, Nkz, Nqz, NE, Nw};
    for (int64_t t = 0; t < (int64_t)NA * NB; ++t)
        if (neigh[t] < 0 || neigh[t] >= NA)
            return 1;
    if (blk == NULL)
        nblk = (int64_t)Nkz * NE * NA;
    for (int64_t t = 0; blk && t < nblk; ++t)
        if (blk[3 * t] < 0 || blk[3 * t] >= Nkz || blk[3 * t + 1] < 0 || blk[3 * t + 1] >= NE ||
            blk[3 * t + 2] < 0 || blk[3 * t + 2] >= NA)
            return 1;
    int missing = 0;
    const size_t nn2 = (size_t)Norb * Norb * 2;
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) reduction(| : missing) num_threads(nthreads)
    for (int64_t t = 0; t < nblk; ++t) {
        int k, e, a;
        if (blk) {
            k = blk[3 * t];
            e = blk[3 * t + 1];
            a = blk[3 * t + 2];
        } else {
            k = (int)(t / ((int64_t)NE * NA));
            e = (int)((t / NA) % NE);
            a = (int)(t % NA);
        }
        missing |= sigma_block(&d, shift, neigh, dH, G, gslot, Dt, alpha_re, alpha_im, k, e, a,
                               out + (size_t)t * nn2);
    }
    return missing ? 2 : 0;
}
