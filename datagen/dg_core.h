/*
 * Per-element arithmetic of the synthetic-input generator.
 *
 * Compiled twice: by gcc for the host generator (datagen.c) and by hipcc for
 * the device generator (datagen_gpu.hip).  The includer defines DG_FN (the
 * function qualifiers) before including this file.  To give bit-identical
 * values on both sides, everything below uses only integer operations and the
 * IEEE-754 binary64 operations +, -, *, / (correctly rounded on both the x86
 * SSE2 unit and the CDNA vector ALU), never a library transcendental, and the
 * includer disables multiply-add contraction (-ffp-contract=off).
 *
 *  - Philox4x32-10: Salmon et al., SC'11 (counter-based; key = seed).
 *  - Gaussian pair: Box-Muller, g0 = r cos(2 pi u2), g1 = r sin(2 pi u2),
 *    r = sqrt(-2 ln u1), with ln, sqrt, sin and cos written out below
 *    (accurate to a few ulp; determinism, not last-bit accuracy, is the goal).
 */
#ifndef DG_CORE_H
#define DG_CORE_H

#include <stdint.h>

#define DG_M0 0xD2511F53u
#define DG_M1 0xCD9E8D57u
#define DG_W0 0x9E3779B9u
#define DG_W1 0xBB67AE85u

DG_FN void dg_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                     uint32_t* out) {
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)DG_M0 * c0;
        uint64_t p1 = (uint64_t)DG_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += DG_W0;
        k1 += DG_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in (0, 1]. */
DG_FN double dg_u53(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 1.0) * 0x1.0p-53;
}

DG_FN uint64_t dg_bits(double x) { union { double d; uint64_t u; } v; v.d = x; return v.u; }
DG_FN double dg_from_bits(uint64_t u) { union { double d; uint64_t u; } v; v.u = u; return v.d; }

/* Natural log of a normal positive double: x = 2^e f, f in [sqrt(1/2), sqrt(2)),
 * ln f = 2 atanh(s), s = (f - 1)/(f + 1), |s| < 0.1716, odd series to s^23. */
DG_FN double dg_log(double x) {
    uint64_t b = dg_bits(x);
    int e = (int)((b >> 52) & 0x7FF) - 1023;
    double f = dg_from_bits((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
    if (f > 1.4142135623730951) { f = f * 0.5; e = e + 1; }
    double s = (f - 1.0) / (f + 1.0);
    double s2 = s * s;
    double p = 1.0 / 23.0;
    p = p * s2 + 1.0 / 21.0;
    p = p * s2 + 1.0 / 19.0;
    p = p * s2 + 1.0 / 17.0;
    p = p * s2 + 1.0 / 15.0;
    p = p * s2 + 1.0 / 13.0;
    p = p * s2 + 1.0 / 11.0;
    p = p * s2 + 1.0 / 9.0;
    p = p * s2 + 1.0 / 7.0;
    p = p * s2 + 1.0 / 5.0;
    p = p * s2 + 1.0 / 3.0;
    p = p * s2 + 1.0;
    double lnf = 2.0 * s * p;
    /* ln 2 split so that e * LN2_HI is exact for |e| < 2^11 */
    const double LN2_HI = 6.93147180369123816490e-01;
    const double LN2_LO = 1.90821492927058770002e-10;
    return ((double)e * LN2_HI + lnf) + (double)e * LN2_LO;
}

/* sqrt of a positive normal double: exponent halving + 6 Newton steps. */
DG_FN double dg_sqrt(double x) {
    uint64_t b = dg_bits(x);
    int e = (int)((b >> 52) & 0x7FF) - 1023;
    int h = (e >= 0) ? e / 2 : -((-e + 1) / 2); /* floor(e / 2) */
    double m = dg_from_bits((b & 0x000FFFFFFFFFFFFFull) | ((uint64_t)(e - 2 * h + 1023) << 52)); /* [1, 4) */
    double y = 0.5 + 0.5 * m; /* >= sqrt(m) */
    for (int i = 0; i < 6; ++i) y = 0.5 * (y + m / y);
    return y * dg_from_bits((uint64_t)(h + 1023) << 52);
}

/* sin and cos of (pi/2) t for t in [0, 1/2]: Taylor series to degree 21/20. */
DG_FN void dg_sincos_quarter(double t, double* s, double* c) {
    const double HALF_PI = 1.5707963267948966;
    double x = t * HALF_PI;
    double x2 = x * x;
    /* sin x / x = sum (-x^2)^k / (2k+1)!,  cos x = sum (-x^2)^k / (2k)!  (Horner) */
    double ps = 1.0 / 51090942171709440000.0;    /* 1/21! */
    ps = 1.0 / 121645100408832000.0 - ps * x2;   /* 1/19! */
    ps = 1.0 / 355687428096000.0 - ps * x2;      /* 1/17! */
    ps = 1.0 / 1307674368000.0 - ps * x2;        /* 1/15! */
    ps = 1.0 / 6227020800.0 - ps * x2;           /* 1/13! */
    ps = 1.0 / 39916800.0 - ps * x2;             /* 1/11! */
    ps = 1.0 / 362880.0 - ps * x2;               /* 1/9!  */
    ps = 1.0 / 5040.0 - ps * x2;                 /* 1/7!  */
    ps = 1.0 / 120.0 - ps * x2;                  /* 1/5!  */
    ps = 1.0 / 6.0 - ps * x2;                    /* 1/3!  */
    ps = 1.0 - ps * x2;
    double pc = 1.0 / 2432902008176640000.0;     /* 1/20! */
    pc = 1.0 / 6402373705728000.0 - pc * x2;     /* 1/18! */
    pc = 1.0 / 20922789888000.0 - pc * x2;       /* 1/16! */
    pc = 1.0 / 87178291200.0 - pc * x2;          /* 1/14! */
    pc = 1.0 / 479001600.0 - pc * x2;            /* 1/12! */
    pc = 1.0 / 3628800.0 - pc * x2;              /* 1/10! */
    pc = 1.0 / 40320.0 - pc * x2;                /* 1/8!  */
    pc = 1.0 / 720.0 - pc * x2;                  /* 1/6!  */
    pc = 1.0 / 24.0 - pc * x2;                   /* 1/4!  */
    pc = 1.0 / 2.0 - pc * x2;                    /* 1/2!  */
    pc = 1.0 - pc * x2;
    *s = x * ps;
    *c = pc;
}

/* sin and cos of 2 pi u for u in (0, 1]. */
DG_FN void dg_sincos_2pi(double u, double* s, double* c) {
    double v = u * 4.0;                /* exact */
    int q = (int)v;                    /* quadrant 0..4 */
    double t = v - (double)q;          /* exact, [0, 1) */
    double sa, ca;
    if (t <= 0.5) {
        dg_sincos_quarter(t, &sa, &ca);
    } else {
        dg_sincos_quarter(1.0 - t, &ca, &sa); /* sin(pi/2 t) = cos(pi/2 (1 - t)) */
    }
    switch (q & 3) {
        case 0: *s = sa; *c = ca; break;
        case 1: *s = ca; *c = -sa; break;
        case 2: *s = -sa; *c = -ca; break;
        default: *s = -ca; *c = sa; break;
    }
}

/* Two N(0,1) draws addressed by (seed, stream, row, block). */
DG_FN void dg_gauss_pair(uint64_t seed, uint32_t stream, uint64_t row, uint32_t block, double* g0, double* g1) {
    uint32_t w[4];
    dg_philox(block, (uint32_t)row, (uint32_t)(row >> 32), stream, (uint32_t)seed, (uint32_t)(seed >> 32), w);
    double u1 = dg_u53(w[0], w[1]);
    double u2 = dg_u53(w[2], w[3]);
    double r2 = -2.0 * dg_log(u1);
    double r = (r2 > 0.0) ? dg_sqrt(r2) : 0.0;
    double s, c;
    dg_sincos_2pi(u2, &s, &c);
    *g0 = r * c;
    *g1 = r * s;
}

/* The mixture's centre value (U[0, 255]) for centre c, dimension j. */
DG_FN double dg_centre_value(uint64_t seed, uint32_t stream_c, uint64_t c, int32_t j) {
    uint32_t w[4];
    dg_philox((uint32_t)(j / 2), (uint32_t)c, (uint32_t)(c >> 32), stream_c, (uint32_t)seed, (uint32_t)(seed >> 32), w);
    double u = (j & 1) ? dg_u53(w[2], w[3]) : dg_u53(w[0], w[1]);
    return 255.0 * ((u - 0x1.0p-53) / (1.0 - 0x1.0p-53));
}

/* Uniform integer in [0, bound) from a 64-bit draw (multiply-shift). */
DG_FN uint64_t dg_mulshift(uint64_t r, uint64_t bound) {
    uint64_t a_hi = r >> 32, a_lo = r & 0xFFFFFFFFull;
    uint64_t b_hi = bound >> 32, b_lo = bound & 0xFFFFFFFFull;
    uint64_t lolo = a_lo * b_lo;
    uint64_t hilo = a_hi * b_lo;
    uint64_t lohi = a_lo * b_hi;
    uint64_t hihi = a_hi * b_hi;
    uint64_t mid = (lolo >> 32) + (hilo & 0xFFFFFFFFull) + (lohi & 0xFFFFFFFFull);
    return hihi + (hilo >> 32) + (lohi >> 32) + (mid >> 32);
}

/* Cluster of mixture row `row` (block 0xFFFFFFFF of the row's counter). */
DG_FN uint64_t dg_mixture_cluster(uint64_t seed, uint32_t stream, uint64_t row, uint64_t n_centres) {
    uint32_t w[4];
    dg_philox(0xFFFFFFFFu, (uint32_t)row, (uint32_t)(row >> 32), stream, (uint32_t)seed, (uint32_t)(seed >> 32), w);
    uint64_t r = ((uint64_t)w[0] << 32) | w[1];
    return dg_mulshift(r, n_centres);
}

/* Round half to even, then clip to [0, 255] (values here are < 2^52). */
DG_FN double dg_round_clip(double v) {
    double a = v < 0.0 ? -v : v;
    double r = (a + 0x1.0p52) - 0x1.0p52; /* RNE to an integer */
    r = v < 0.0 ? -r : r;
    if (r < 0.0) r = 0.0;
    if (r > 255.0) r = 255.0;
    return r;
}

#endif
