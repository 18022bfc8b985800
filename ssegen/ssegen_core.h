/*
 * ssegen_core.h -- seeded, counter-based input generator for the SSE kernel's
 * tensors (neighbour table, dH, G, D~) and for the per-iteration perturbation
 * that stands in for the Green's-function phase of a self-consistent run.
 *
 * This module holds none of the self-energy arithmetic.  It is included by
 * the host generator (ssegen_host.c, built with gcc) and by the device
 * generator (ssegen_device.hip, built with hipcc); SSEGEN_FN supplies the
 * function qualifiers for each side.  Every step uses only integer operations
 * and exactly rounded IEEE-754 binary64 +, -, *, / (no fused multiply-add,
 * no library transcendental), so the host and the device produce the same
 * bits for every element.
 *
 * Random bits: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), key = the 64-bit seed, counter =
 * (element index lo, element index hi, stream word, draw number).
 *
 * Normal variates: the classical Irwin-Hall approximation, the sum of twelve
 * U[0,1) values minus six (mean 0, variance 1).  With U = x * 2^-32 every
 * partial sum is a multiple of 2^-32 below 12, so the sum is exact in
 * binary64 and independent of summation order.
 */
#ifndef SSEGEN_CORE_H
#define SSEGEN_CORE_H

#include <stdint.h>

#ifndef SSEGEN_FN
#define SSEGEN_FN static inline
#endif

/* Stream words (third counter word).  Perturbation streams put the SCBA
 * iteration number in the upper 24 bits. */
enum {
    SSEGEN_S_NEIGH = 1,
    SSEGEN_S_DH = 2,
    SSEGEN_S_G = 16,      /* + component (0: lesser, 1: greater) */
    SSEGEN_S_GSCALE = 24, /* + component: per-block magnitude */
    SSEGEN_S_D = 32,      /* + component */
    SSEGEN_S_PERT_G = 64, /* + component, | (iteration + 1) << 8 */
    SSEGEN_S_PERT_D = 72  /* + component, | (iteration + 1) << 8 */
};

typedef struct {
    uint32_t w[4];
} ssegen_u4;

/* One Philox4x32 round followed by the counter update of the published
 * algorithm; multipliers and Weyl key increments as published. */
SSEGEN_FN ssegen_u4 ssegen_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                  uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    ssegen_u4 out;
    out.w[0] = c0;
    out.w[1] = c1;
    out.w[2] = c2;
    out.w[3] = c3;
    return out;
}

/* Approximate N(0,1) value for (element, stream): draws first_draw,
 * first_draw+1, first_draw+2 supply the twelve 32-bit words. */
SSEGEN_FN double ssegen_normal(uint64_t seed, uint64_t idx, uint32_t stream, uint32_t first_draw)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t i0 = (uint32_t)idx, i1 = (uint32_t)(idx >> 32);
    double s = 0.0;
    for (uint32_t d = 0; d < 3; ++d) {
        ssegen_u4 x = ssegen_philox(i0, i1, stream, first_draw + d, k0, k1);
        for (int t = 0; t < 4; ++t)
            s = s + (double)x.w[t] * 0x1p-32;
    }
    return s - 6.0;
}

/* Raw complex normal X[idx]: real part from draws 0..2, imaginary from 3..5. */
SSEGEN_FN void ssegen_cnormal(uint64_t seed, uint64_t idx, uint32_t stream, double *re, double *im)
{
    *re = ssegen_normal(seed, idx, stream, 0);
    *im = ssegen_normal(seed, idx, stream, 3);
}

/* Element (m, n) of the anti-Hermitian part (X - X^H)/2 of the raw complex
 * normal block whose element (0, 0) has flat index base and whose side is n_side. */
SSEGEN_FN void ssegen_antiherm(uint64_t seed, uint64_t base, int n_side, int m, int n,
                               uint32_t stream, double *re, double *im)
{
    double ar, ai, br, bi;
    ssegen_cnormal(seed, base + (uint64_t)m * n_side + n, stream, &ar, &ai);
    ssegen_cnormal(seed, base + (uint64_t)n * n_side + m, stream, &br, &bi);
    /* X[m,n] - conj(X[n,m]) = (ar - br) + i (ai + bi) */
    *re = (ar - br) * 0.5;
    *im = (ai + bi) * 0.5;
}

/* Per-block magnitude for the precision stress test: (1 + u) * 2^n with n
 * uniform in {-20, ..., 6}, a discretised log-uniform spread over about
 * 1e-6 .. 1e2 (exact in binary64). */
SSEGEN_FN double ssegen_block_scale(uint64_t seed, uint64_t block, uint32_t stream)
{
    ssegen_u4 x = ssegen_philox((uint32_t)block, (uint32_t)(block >> 32), stream, 0,
                                (uint32_t)seed, (uint32_t)(seed >> 32));
    double m = 1.0 + (double)x.w[0] * 0x1p-32;
    int e = -20 + (int)(((uint64_t)x.w[1] * 27u) >> 32);
    double p = 1.0;
    if (e >= 0) {
        for (int t = 0; t < e; ++t) p = p * 2.0;
    } else {
        for (int t = 0; t < -e; ++t) p = p * 0.5;
    }
    return m * p;
}

#endif /* SSEGEN_CORE_H */
