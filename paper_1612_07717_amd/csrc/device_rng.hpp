// device_rng.hpp -- counter-based normals for the particle paths (gfx950).
//
// The paper only requires xi_n ~ N(0, 1) i.i.d. (Sec. 3.1). Each sample draws its
// normals from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): a 10-round bijection of a 128-bit counter under a 64-bit
// key, so any draw is computed from its coordinates with no stored state. Counter =
// (block, sample_lo, sample_hi, level | stream << 8), key = seed. One block gives two
// uniforms and, by Box-Muller (Box & Muller 1958), the two normals of fine steps 2m
// and 2m+1 (or of steps 2m, 2m+1 on level 0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ldm {

// Philox4x32 round constants: the two S-box multipliers and the key's Weyl increments.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// Reserved blocks of a sample for its initial state.
constexpr uint32_t kBlockInitW = 0xFFFFFFFFu;
constexpr uint32_t kBlockInitX = 0xFFFFFFFEu;

struct Words {
    uint32_t r0, r1, r2, r3;
};

// The part of the counter fixed for a sample, and the key.
struct Stream {
    uint32_t c1, c2, c3;
    uint32_t k0, k1;
};

__device__ __forceinline__ Stream make_stream(uint64_t seed, uint32_t stream_id, int level,
                                              uint64_t sample) {
    Stream s;
    s.c1 = (uint32_t)sample;
    s.c2 = (uint32_t)(sample >> 32);
    s.c3 = ((uint32_t)level & 0xFFu) | (stream_id << 8);
    s.k0 = (uint32_t)seed;
    s.k1 = (uint32_t)(seed >> 32);
    return s;
}

__device__ __forceinline__ Words philox(const Stream& s, uint32_t block) {
    uint32_t x0 = block, x1 = s.c1, x2 = s.c2, x3 = s.c3;
    uint32_t k0 = s.k0, k1 = s.k1;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // S-box: two 32x32 -> 64-bit products (one v_mad_u64_u32 each); high halves
        // mixed with the other words and the round key, low halves passed on.
        const uint64_t p0 = (uint64_t)kPhiloxM0 * x0, p1 = (uint64_t)kPhiloxM1 * x2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t y0 = hi1 ^ x1 ^ k0;
        const uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return Words{x0, x1, x2, x3};
}

// Open-interval uniforms: FP64 from the top 52 bits of a 64-bit word pair,
// (2m + 1) 2^-53 in (0, 1); FP32 from the top 23 bits of the high word,
// (2m + 1) 2^-24. Both are exact, and the FP32 value is the FP64 one to 2^-24.
__device__ __forceinline__ double uniform64(uint32_t hi, uint32_t lo) {
    const uint64_t m = ((((uint64_t)hi) << 32) | lo) >> 12;
    return (double)((m << 1) | 1u) * 0x1p-53;
}

__device__ __forceinline__ float uniform32(uint32_t hi) {
    return (float)(((hi >> 9) << 1) | 1u) * 0x1p-24f;
}

template <typename R>
struct Normals;

// ln u for u = (2j + 1) 2^-53 in (0, 1), to about half an ulp. With u = m 2^e and m in
// [sqrt(1/2), sqrt(2)): ln u = e ln 2 + 2 atanh(s), s = (m - 1) / (m + 1), |s| <= 0.1716,
// and 2 atanh(s) = 2s + 2s t (1/3 + t/5 + ... + t^9/21), t = s^2 (the next term is below
// 1e-18 relative). s = q + sl: q the rounded quotient, sl from its exact residual (m + 1
// is carried as den + dlo, both exact). ln 2 = ln2_hi + ln2_lo, ln2_hi with 29
// significant bits so that e ln2_hi is exact; e ln2_hi + 2q is summed with its rounding
// error kept (|e ln2_hi| >= |2q| unless e = 0), and every small term joins that error.
__device__ __forceinline__ double log_unit(double u) {
    const int e = __builtin_amdgcn_frexp_exp(u);          // u = m 2^e, m in [1/2, 1)
    double m = __builtin_amdgcn_frexp_mant(u);
    const bool lo = m < 0.70710678118654752;
    m = lo ? 2.0 * m : m;
    const double ed = (double)(lo ? e - 1 : e);
    const double num = m - 1.0;                           // exact
    const double den = m + 1.0;
    const double dlo = m - (den - 1.0);                   // m + 1 = den + dlo, both exact
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    const double q = num * r;
    const double sl = (fma(-q, den, num) - q * dlo) * r;
    const double t = q * q;
    double p = 1.0 / 21.0;
    p = fma(p, t, 1.0 / 19.0);
    p = fma(p, t, 1.0 / 17.0);
    p = fma(p, t, 1.0 / 15.0);
    p = fma(p, t, 1.0 / 13.0);
    p = fma(p, t, 1.0 / 11.0);
    p = fma(p, t, 1.0 / 9.0);
    p = fma(p, t, 1.0 / 7.0);
    p = fma(p, t, 1.0 / 5.0);
    p = fma(p, t, 1.0 / 3.0);
    const double a = ed * 0x1.62e42ffp-1;                 // exact
    const double b = 2.0 * q;
    const double hi = a + b;
    const double err = b - (hi - a);                      // a + b = hi + err exactly
    const double small = fma(2.0 * q * t, p, fma(ed, -0x1.718432a1b0e26p-35, fma(2.0, sl, err)));
    return hi + small;
}

// sin and cos of theta in [0, 2 pi] (theta as FP64 holds it), to about half an ulp.
// theta = k pi/2 + x with k = rint(theta 2/pi) and pi/2 = P1 + P2 + ..., P1 its FP64
// rounding: x1 = theta - k P1 is exact (one fused multiply-add; its result is a multiple
// of 2^-53 below 1), and x = x1 - d, d = k P2, so sin x = sin x1 - d cos x1 and
// cos x = cos x1 + d sin x1 to within d^2 < 1e-31. sin x1 and cos x1 are their Taylor
// series to degree 17 and 18 (|x1| <= pi/4: truncation below 1e-18 relative), led by
// x1 and 1 - x1^2/2 with the rounding errors of x1^2 and 1 - x1^2/2 carried into the
// tail. k mod 4 picks the quadrant.
__device__ __forceinline__ void sincos_fp64(double theta, double& sn, double& cs) {
    const double k = rint(theta * 0.63661977236758134);
    const double x = fma(-k, 1.5707963267948966, theta);  // exact
    const double d = k * 6.123233995736766e-17;
    const double y = x * x;
    const double yl = fma(x, x, -y);                      // x^2 = y + yl exactly
    double ps = 1.0 / 355687428096000.0;                  // 1/17!
    ps = fma(ps, y, -1.0 / 1307674368000.0);
    ps = fma(ps, y, 1.0 / 6227020800.0);
    ps = fma(ps, y, -1.0 / 39916800.0);
    ps = fma(ps, y, 1.0 / 362880.0);
    ps = fma(ps, y, -1.0 / 5040.0);
    ps = fma(ps, y, 1.0 / 120.0);
    ps = fma(ps, y, -1.0 / 6.0);
    double pc = -1.0 / 6402373705728000.0;                // -1/18!
    pc = fma(pc, y, 1.0 / 20922789888000.0);
    pc = fma(pc, y, -1.0 / 87178291200.0);
    pc = fma(pc, y, 1.0 / 479001600.0);
    pc = fma(pc, y, -1.0 / 3628800.0);
    pc = fma(pc, y, 1.0 / 40320.0);
    pc = fma(pc, y, -1.0 / 720.0);
    pc = fma(pc, y, 1.0 / 24.0);
    const double hy = 0.5 * y;
    const double w = 1.0 - hy;
    const double wl = (1.0 - w) - hy;                     // 1 - hy = w + wl exactly
    const double c0 = w + fma(y * y, pc, fma(d, x, fma(-0.5, yl, wl)));
    const double s0 = x + fma(x * y, ps, -d * w);
    const int q = (int)k & 3;
    const double sa = (q & 1) ? c0 : s0;                  // |sin|, |cos| of the quadrant
    const double ca = (q & 1) ? s0 : c0;
    sn = (q & 2) ? -sa : sa;
    cs = ((q + 1) & 2) ? -ca : ca;
}

template <>
struct Normals<double> {
    // rho = sqrt(-2 ln u); (rho cos 2 pi v, rho sin 2 pi v)
    static __device__ __forceinline__ void pair(const Words& w, double& z0, double& z1) {
        const double u = uniform64(w.r1, w.r0);
        const double v = uniform64(w.r3, w.r2);
        const double l = -2.0 * log_unit(u);
        double rho = __builtin_amdgcn_rsq(l);               // sqrt(l) = l rsq(l), refined
        double h = 0.5 * rho;
        rho *= l;
        const double e = fma(-rho, h, 0.5);
        rho = fma(rho, e, rho);
        h = fma(h, e, h);
        rho = fma(fma(-rho, rho, l), h, rho);
        rho = fma(fma(-rho, rho, l), h, rho);
        double s, c;
        sincos_fp64(6.283185307179586 * v, s, c);
        z0 = rho * c;
        z1 = rho * s;
    }
};

template <>
struct Normals<float> {
    // Hardware transcendentals: v_log_f32 is log2, v_sin_f32 / v_cos_f32 take their
    // argument in revolutions, so sin(2 pi v) = v_sin_f32(v) for v in (0, 1).
    static __device__ __forceinline__ void pair(const Words& w, float& z0, float& z1) {
        const float u = uniform32(w.r1);
        const float v = uniform32(w.r3);
        const float rho = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));
        z0 = rho * __builtin_amdgcn_cosf(v);
        z1 = rho * __builtin_amdgcn_sinf(v);
    }
};

}  // namespace ldm
