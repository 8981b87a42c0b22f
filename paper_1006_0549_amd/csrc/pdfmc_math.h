// Wiener increments for the particle SDEs, Eq.(2), (4) and (5).
//
// Reading R-09: counter-based Philox4x32-10 (Salmon et al., SC'11, the
// published round function and constants), key = (seed low, seed high),
// counter = (particle id, step, stream, block). Blocks 0..2 give 12 words;
// H_m = word m, L_m = word 6+m, m = 0..5.
//   FP64 uniform: u_m = (2 ((H_m << 20) | (L_m >> 12)) + 1) 2^-53
//   FP32 uniform: u_m = (2 (H_m >> 9) + 1) 2^-24   (blocks 0..1 only)
// Both are exact conversions into (0, 1); the FP32 value approximates the
// FP64 one, so the two precisions follow nearly the same sample path.
//
// Reading R-10: Box-Muller, xi_{2j} = sqrt(-2 ln u_{2j}) cos(2 pi u_{2j+1}),
// xi_{2j+1} = sqrt(-2 ln u_{2j}) sin(2 pi u_{2j+1}). In FP64, ln and
// sincos(2 pi .) are evaluated from their series in a fixed operation order
// (written below from the mathematics) so the result is bit-identical to any
// other implementation of the same order with correctly rounded +,-,*,/,
// fma and sqrt. In FP32 the hardware transcendentals are used: v_log_f32
// (log2) and v_sin_f32 / v_cos_f32, which take their argument in turns.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdfmc {

__device__ inline void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        // each 32 x 32 -> 64-bit product in one multiply (high and low word together)
        const uint64_t p0 = (uint64_t)m0 * c0, p1 = (uint64_t)m1 * c2;
        const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
        const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        uint32_t n0 = h1 ^ c1 ^ k0;
        uint32_t n2 = h0 ^ c3 ^ k1;
        c0 = n0; c1 = l1; c2 = n2; c3 = l0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// ln(u), u > 0 normal: u = m 2^e, m in [sqrt(1/2), sqrt(2)); s = (m-1)/(m+1),
// ln m = 2s (1 + z/3 + z^2/5 + ... + z^10/23), z = s^2;
// ln u = fma(e, ln2_hi, fma(e, ln2_lo, ln m)), ln2_hi having 32 significant bits.
__device__ inline double ln_series(double u)
{
    const double LN2_HI = 0x1.62e42fee00000p-1;
    const double LN2_LO = 0x1.a39ef35793c76p-33;
    const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;
    int e;
    double m = __builtin_frexp(u, &e);
    if (m < SQRT_HALF) { m = 2.0 * m; e -= 1; }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = __builtin_fma(p, z, 1.0 / 21.0);
    p = __builtin_fma(p, z, 1.0 / 19.0);
    p = __builtin_fma(p, z, 1.0 / 17.0);
    p = __builtin_fma(p, z, 1.0 / 15.0);
    p = __builtin_fma(p, z, 1.0 / 13.0);
    p = __builtin_fma(p, z, 1.0 / 11.0);
    p = __builtin_fma(p, z, 1.0 / 9.0);
    p = __builtin_fma(p, z, 1.0 / 7.0);
    p = __builtin_fma(p, z, 1.0 / 5.0);
    p = __builtin_fma(p, z, 1.0 / 3.0);
    double t = 2.0 * s;
    double lnm = __builtin_fma(t, z * p, t);
    double de = (double)e;
    return __builtin_fma(de, LN2_HI, __builtin_fma(de, LN2_LO, lnm));
}

// sin and cos of 2 pi u: t = 4u, q = rint(t), f = t - q (exact), x = f pi/2;
// sin x = x + x z (-1/3! + z/5! - ... - z^8/19!), cos x = 1 + z (-1/2! + ... - z^8/18!),
// z = x^2, Horner from the highest term; then rotate by the quadrant q mod 4.
__device__ inline void sincos2pi_series(double u, double& s_out, double& c_out)
{
    const double PI_2 = 0x1.921fb54442d18p+0;
    double t = 4.0 * u;
    double q = __builtin_rint(t);
    double f = t - q;
    double x = f * PI_2;
    double z = x * x;
    double ps = -1.0 / 121645100408832000.0;
    ps = __builtin_fma(ps, z, 1.0 / 355687428096000.0);
    ps = __builtin_fma(ps, z, -1.0 / 1307674368000.0);
    ps = __builtin_fma(ps, z, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, z, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, z, 1.0 / 362880.0);
    ps = __builtin_fma(ps, z, -1.0 / 5040.0);
    ps = __builtin_fma(ps, z, 1.0 / 120.0);
    ps = __builtin_fma(ps, z, -1.0 / 6.0);
    double sx = __builtin_fma(x, z * ps, x);
    double pc = -1.0 / 6402373705728000.0;
    pc = __builtin_fma(pc, z, 1.0 / 20922789888000.0);
    pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);
    pc = __builtin_fma(pc, z, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, z, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, z, 1.0 / 40320.0);
    pc = __builtin_fma(pc, z, -1.0 / 720.0);
    pc = __builtin_fma(pc, z, 1.0 / 24.0);
    pc = __builtin_fma(pc, z, -0.5);
    double cx = __builtin_fma(z, pc, 1.0);
    int quad = ((int)q) & 3;
    if (quad == 0) { s_out = sx; c_out = cx; }
    else if (quad == 1) { s_out = cx; c_out = -sx; }
    else if (quad == 2) { s_out = -sx; c_out = -cx; }
    else { s_out = -cx; c_out = sx; }
}

__device__ inline void gauss6_f64(uint32_t k0, uint32_t k1, uint32_t id, uint32_t step, uint32_t stream, double xi[6])
{
    uint32_t w[12];
#pragma unroll
    for (uint32_t b = 0; b < 3; ++b) {
        uint32_t c0 = id, c1 = step, c2 = stream, c3 = b;
        philox4x32_10(c0, c1, c2, c3, k0, k1);
        w[4 * b] = c0; w[4 * b + 1] = c1; w[4 * b + 2] = c2; w[4 * b + 3] = c3;
    }
    double u[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        uint64_t K = ((uint64_t)w[m] << 20) | (uint64_t)(w[6 + m] >> 12);
        u[m] = (double)(2 * K + 1) * 0x1p-53;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double r = __builtin_sqrt(-2.0 * ln_series(u[2 * j]));
        double s, c;
        sincos2pi_series(u[2 * j + 1], s, c);
        xi[2 * j] = r * c;
        xi[2 * j + 1] = r * s;
    }
}

__device__ inline void gauss6_f32(uint32_t k0, uint32_t k1, uint32_t id, uint32_t step, uint32_t stream, float xi[6])
{
    uint32_t w[8];
#pragma unroll
    for (uint32_t b = 0; b < 2; ++b) {
        uint32_t c0 = id, c1 = step, c2 = stream, c3 = b;
        philox4x32_10(c0, c1, c2, c3, k0, k1);
        w[4 * b] = c0; w[4 * b + 1] = c1; w[4 * b + 2] = c2; w[4 * b + 3] = c3;
    }
    const float LN2x2 = 1.38629436111989061883f;   // 2 ln 2
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float u0 = (float)(2u * (w[2 * j] >> 9) + 1u) * 0x1p-24f;
        float u1 = (float)(2u * (w[2 * j + 1] >> 9) + 1u) * 0x1p-24f;
        float r = __builtin_sqrtf(-LN2x2 * __builtin_amdgcn_logf(u0));
        float s = __builtin_amdgcn_sinf(u1);
        float c = __builtin_amdgcn_cosf(u1);
        xi[2 * j] = r * c;
        xi[2 * j + 1] = r * s;
    }
}

// Initial-state draws (R-29, R-30): the same generator with purpose 1 in the
// counter, counter = (id, 0, stream, (1 << 8) | block), blocks 0..4 ->
// 20 words; uniform m = 0..9 from words 2m (high) and 2m+1 (low),
// u_m = (2 ((w_2m << 20) | (w_2m+1 >> 12)) + 1) 2^-53.
__device__ inline void init_uniforms(uint32_t k0, uint32_t k1, uint32_t id, uint32_t stream, double u[10])
{
    uint32_t w[20];
#pragma unroll
    for (uint32_t b = 0; b < 5; ++b) {
        uint32_t c0 = id, c1 = 0u, c2 = stream, c3 = (1u << 8) | b;
        philox4x32_10(c0, c1, c2, c3, k0, k1);
        w[4 * b] = c0; w[4 * b + 1] = c1; w[4 * b + 2] = c2; w[4 * b + 3] = c3;
    }
#pragma unroll
    for (int m = 0; m < 10; ++m) {
        const uint64_t K = ((uint64_t)w[2 * m] << 20) | (uint64_t)(w[2 * m + 1] >> 12);
        u[m] = (double)(2 * K + 1) * 0x1p-53;
    }
}

}  // namespace pdfmc
