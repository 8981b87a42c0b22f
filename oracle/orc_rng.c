/* Oracle (test infrastructure): Wiener increments of Eq.(2), (4) and (5).
 *
 * The paper only requires Gaussian increments, with the same dW_i driving
 * Eq.(2) and Eq.(4) (Sec. II). Reading R-09 fixes a counter-based generator
 * so that every particle-step draws the same numbers on the CPU and the GPU:
 *   Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), key = seed,
 *   counter = (id, step, stream, block), blocks 0..2 -> 12 words,
 *   H_m = word m, L_m = word 6+m (m = 0..5),
 *   u_m = (2*((H_m << 20) | (L_m >> 12)) + 1) * 2^-53   (exact, in (0,1)).
 * Reading R-10 turns u_0..u_5 into xi_0..xi_5 by Box-Muller,
 *   xi_{2j} = sqrt(-2 ln u_{2j}) cos(2 pi u_{2j+1}),
 *   xi_{2j+1} = sqrt(-2 ln u_{2j}) sin(2 pi u_{2j+1}),
 * with ln and sincos(2 pi .) written out below from their series, in a fixed
 * operation order, so that two independent implementations agree bit for bit.
 */
#include "orc_internal.h"
#include <math.h>

/* Philox4x32 round constants from the published definition */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0; k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_uniforms(uint64_t seed, uint32_t id, uint32_t step, uint32_t stream, double u[6])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[12];
    for (uint32_t blk = 0; blk < 3; ++blk) {
        uint32_t ctr[4] = {id, step, stream, blk};   /* purpose 0 (time step) */
        orc_philox4x32_10(ctr, key, w + 4 * blk);
    }
    for (int m = 0; m < 6; ++m) {
        uint64_t K = ((uint64_t)w[m] << 20) | (uint64_t)(w[6 + m] >> 12);
        u[m] = ldexp((double)(2 * K + 1), -53);
    }
}

void orc_uniform6(uint64_t seed, uint32_t id, uint32_t step, uint32_t stream, double u[6])
{
    orc_uniforms(seed, id, step, stream, u);
}

/* ln(u) for u > 0 normal: u = m 2^e with m in [sqrt(1/2), sqrt(2));
 * ln m = 2 atanh(s), s = (m-1)/(m+1), atanh(s) = s (1 + z/3 + z^2/5 + ...),
 * z = s^2 <= 0.0295, summed to z^10/21 (remainder < 2^-56 relative);
 * ln u = e ln2_hi + (e ln2_lo + ln m) with ln2 split so e*ln2_hi is exact. */
double orc_ln(double u)
{
    const double LN2_HI = 0x1.62e42fee00000p-1;
    const double LN2_LO = 0x1.a39ef35793c76p-33;
    const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;
    int e;
    double m = frexp(u, &e);
    if (m < SQRT_HALF) { m = 2.0 * m; e -= 1; }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = fma(p, z, 1.0 / 21.0);
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    double t = 2.0 * s;
    double lnm = fma(t, z * p, t);
    double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, lnm));
}

/* sin and cos of 2 pi u: t = 4u, q = nearest integer (ties to even),
 * f = t - q in [-1/2, 1/2] (exact), x = f pi/2 in [-pi/4, pi/4];
 * Taylor series of sin to x^19 and cos to x^18, (-1)^k x^(2k+1)/(2k+1)! and
 * (-1)^k x^(2k)/(2k)!, in Horner form, then quadrant rotation. */
void orc_sincos2pi(double u, double* s_out, double* c_out)
{
    const double PI_2 = 0x1.921fb54442d18p+0;
    double t = 4.0 * u;
    double q = rint(t);
    double f = t - q;
    double x = f * PI_2;
    double z = x * x;
    double ps = -1.0 / 121645100408832000.0;       /* -1/19! */
    ps = fma(ps, z, 1.0 / 355687428096000.0);      /* 1/17! */
    ps = fma(ps, z, -1.0 / 1307674368000.0);       /* -1/15! */
    ps = fma(ps, z, 1.0 / 6227020800.0);           /* 1/13! */
    ps = fma(ps, z, -1.0 / 39916800.0);            /* -1/11! */
    ps = fma(ps, z, 1.0 / 362880.0);               /* 1/9! */
    ps = fma(ps, z, -1.0 / 5040.0);                /* -1/7! */
    ps = fma(ps, z, 1.0 / 120.0);                  /* 1/5! */
    ps = fma(ps, z, -1.0 / 6.0);                   /* -1/3! */
    double sx = fma(x, z * ps, x);
    double pc = -1.0 / 6402373705728000.0;         /* -1/18! */
    pc = fma(pc, z, 1.0 / 20922789888000.0);       /* 1/16! */
    pc = fma(pc, z, -1.0 / 87178291200.0);         /* -1/14! */
    pc = fma(pc, z, 1.0 / 479001600.0);            /* 1/12! */
    pc = fma(pc, z, -1.0 / 3628800.0);             /* -1/10! */
    pc = fma(pc, z, 1.0 / 40320.0);                /* 1/8! */
    pc = fma(pc, z, -1.0 / 720.0);                 /* -1/6! */
    pc = fma(pc, z, 1.0 / 24.0);                   /* 1/4! */
    pc = fma(pc, z, -0.5);                         /* -1/2! */
    double cx = fma(z, pc, 1.0);
    int quad = ((int)q) & 3;
    double s, c;
    switch (quad) {
    case 0: s = sx; c = cx; break;
    case 1: s = cx; c = -sx; break;
    case 2: s = -sx; c = -cx; break;
    default: s = -cx; c = sx; break;
    }
    *s_out = s; *c_out = c;
}

void orc_gauss6(uint64_t seed, uint32_t id, uint32_t step, uint32_t stream, double xi[6])
{
    double u[6];
    orc_uniforms(seed, id, step, stream, u);
    for (int j = 0; j < 3; ++j) {
        double r = sqrt(-2.0 * orc_ln(u[2 * j]));
        double s, c;
        orc_sincos2pi(u[2 * j + 1], &s, &c);
        xi[2 * j] = r * c;
        xi[2 * j + 1] = r * s;
    }
}

/* Initial-state draws (R-29, R-30): the same generator with purpose 1 in the
 * counter, counter = (id, 0, stream, (1 << 8) | block), blocks 0..4 ->
 * 20 words; uniform m = 0..9 from words 2m (high) and 2m+1 (low),
 * u_m = (2*((w_{2m} << 20) | (w_{2m+1} >> 12)) + 1) * 2^-53. */
void orc_init_uniforms(uint64_t seed, uint32_t id, uint32_t stream, double u[10])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[20];
    for (uint32_t b = 0; b < 5; ++b) {
        uint32_t ctr[4] = {id, 0u, stream, (1u << 8) | b};
        orc_philox4x32_10(ctr, key, w + 4 * b);
    }
    for (int m = 0; m < 10; ++m) {
        uint64_t K = ((uint64_t)w[2 * m] << 20) | (uint64_t)(w[2 * m + 1] >> 12);
        u[m] = (double)(2 * K + 1) * 0x1p-53;
    }
}
