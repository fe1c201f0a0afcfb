// device_model.hpp -- one coupled MLMC sample per lane, state in registers (gfx950).
//
// Model (Sec. 2): dU = -lambda(X) U dt - dV/dX(X, U) dt + sigma(X) dW, dX = U dt
// (Eq. 4) with lambda = 1/tau, sigma^2 = 2 sigma_U^2 / tau and the well-mixed drift
// -dV/dX = (1/2)(1 + U^2/sigma_U^2) d(sigma_U^2)/dX (Eq. 3). For the neutral layer
// (Eq. 5, cut off by Eq. 7) this drift is -a(X) - b(X) U^2 with
//     a = (3/4) (kappa_sigma u_*)^2 sqrt(1 - X/H) / H,   b = (3/4) / (H - X)
// inside [eps_reg, H - eps_reg] and 0 in the cut-off layers, where sigma_U is frozen.
//
// Integrators: symplectic Euler (Eq. 8), geometric Langevin OBA (Eq. 9), BAOAB
// (Eq. 10). The O-step noise amplitude sigma sqrt((1 - e^{-2 lambda h}) / (2 lambda))
// equals sigma_U sqrt(1 - w^2) with w = e^{-lambda h}; both w and 1 - w^2 come from one
// e1 = expm1(-lambda h): w = 1 + e1, 1 - w^2 = -e1 (2 + e1), free of cancellation.
//
// Reflection (Eq. 6, Sec. 4): after every position update the position is folded back
// into [0, H] (X -> -X or 2H - X), the velocity flips and the path's reflection sign S
// flips. The noise entering a path is multiplied by the S in force at that moment:
// the fine path's extended noise is S_f xi (Eq. 30), the coarse path's physical noise
// is S_c times the combined extended noise (Eqs. 31, 32). S is kept as a sign-bit
// mask, so applying it is one XOR.
//
// Coupling (Sec. 3.3): the coarse step 2h uses (xi~_2m + xi~_2m+1)/sqrt(2) for SE
// (Eq. 18) and (w xi~_2m + xi~_2m+1)/sqrt(w^2 + 1) for GL and BAOAB (Eq. 19), w being
// e^{-lambda h} of the first fine O-step of the pair.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_rng.hpp"
#include "ld_internal.hpp"

namespace ldm {

constexpr uint32_t kSignBit = 0x80000000u;

template <typename R>
struct Math;

template <>
struct Math<float> {
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float flip(float v, uint32_t mask) {
        return __uint_as_float(__float_as_uint(v) ^ mask);
    }
    static __device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float floor_(float x) { return __builtin_floorf(x); }
    static __device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    // v_med3_f32: the median of (x, lo, hi) is x clamped to [lo, hi] for lo <= hi
    static __device__ __forceinline__ float clamp_(float x, float lo, float hi) {
        return __builtin_amdgcn_fmed3f(x, lo, hi);
    }
    // sqrt(d) and 1/d from one reciprocal square root
    static __device__ __forceinline__ void sqrt_and_rcp(float d, float& sq, float& inv) {
        const float r = __builtin_amdgcn_rsqf(d);
        sq = d * r;
        inv = r * r;
    }
    // x < 0 or x > H (H > 0): non-negative floats order as their bit patterns, and a
    // set sign bit (or a NaN) compares above H's pattern
    static __device__ __forceinline__ bool outside(float x, float H) {
        return __float_as_uint(x) > __float_as_uint(H);
    }

    // expm1 by argument reduction x = k ln2 + r, |r| <= ln2/2 (Cody & Waite's two-part
    // ln2), the Taylor series of expm1(r) to degree 7 (truncation < 2e-8 relative), and
    // expm1(x) = 2^k expm1(r) + (2^k - 1), which has no cancellation for k != 0.
    static __device__ __forceinline__ float expm1_(float x) {
        const float k = __builtin_rintf(x * 1.4426950408889634f);
        float r = __builtin_fmaf(-k, 0.693145751953125f, x);
        r = __builtin_fmaf(-k, 1.428606820309417e-06f, r);
        float p = 1.0f / 5040.0f;
        p = __builtin_fmaf(p, r, 1.0f / 720.0f);
        p = __builtin_fmaf(p, r, 1.0f / 120.0f);
        p = __builtin_fmaf(p, r, 1.0f / 24.0f);
        p = __builtin_fmaf(p, r, 1.0f / 6.0f);
        p = __builtin_fmaf(p, r, 0.5f);
        p = __builtin_fmaf(p, r, 1.0f);
        p = p * r;
        const int ki = (int)k;
        const float two_k = __builtin_amdgcn_ldexpf(1.0f, ki);
        return __builtin_fmaf(two_k, p, two_k - 1.0f);
    }
    // expm1(z) for |z| <= kSmallZ: the Taylor series to degree 5 (truncation below
    // 1.5e-9 relative), evaluated in Estrin form so that only three dependent
    // operations follow z: z + z^2 (1/2 + z/6) + z^4 (1/24 + z/120).
    static constexpr float kSmallZ = 0.0625f;
    static __device__ __forceinline__ float expm1_small(float z) {
        const float z2 = z * z;
        const float a = __builtin_fmaf(z, 1.0f / 6.0f, 0.5f);
        const float b = __builtin_fmaf(z, 1.0f / 120.0f, 1.0f / 24.0f);
        const float z4 = z2 * z2;
        return __builtin_fmaf(z4, b, __builtin_fmaf(z2, a, z));
    }
    // expm1(z) for |z| <= kTinyZ: the series to degree 3 (truncation below 2.6e-9
    // relative, under half an FP32 ulp), z + z^2 (1/2 + z/6): two operations follow z.
    static constexpr float kTinyZ = 0.00390625f;
    static __device__ __forceinline__ float expm1_tiny(float z) {
        return __builtin_fmaf(z * z, __builtin_fmaf(z, 1.0f / 6.0f, 0.5f), z);
    }
};

template <>
struct Math<double> {
    // Square root, reciprocal and reciprocal square root for the path arithmetic, whose
    // arguments are finite, non-negative and far from the range ends (heights, step
    // sizes, rates): the hardware estimate refined by Newton steps, without the range
    // scaling of the library routines. sqrt: s = x r, h = r/2 from r = rsq(x), one
    // coupled Newton step on (s, h), then two corrections s += (x - s^2) h; the argument is
    // raised to the least normal number first so that sqrt(0) = 0. rcp: two Newton steps
    // r += r (1 - x r). Both are within an ulp or so of the correctly rounded result.
    static __device__ __forceinline__ double sqrt_(double x) {
        const double xs = fmax(x, 2.2250738585072014e-308);
        const double r = __builtin_amdgcn_rsq(xs);
        double s = x * r, h = 0.5 * r;
        const double e = fma(-s, h, 0.5);
        s = fma(s, e, s);
        h = fma(h, e, h);
        s = fma(fma(-s, s, x), h, s);
        return fma(fma(-s, s, x), h, s);
    }
    static __device__ __forceinline__ double rcp(double x) {
        double r = __builtin_amdgcn_rcp(x);
        r = fma(r, fma(-x, r, 1.0), r);
        return fma(r, fma(-x, r, 1.0), r);
    }
    static __device__ __forceinline__ double rsqrt(double x) {
        const double r = __builtin_amdgcn_rsq(x);                 // x > 0
        const double hr = 0.5 * r;
        const double y = fma(-hr, x * r, 1.5) * r;                 // r (3 - x r^2) / 2
        return fma(-0.5 * y, x * y, 1.5) * y;
    }
    static __device__ __forceinline__ double flip(double v, uint32_t mask) {
        return __hiloint2double(__double2hiint(v) ^ (int)mask, __double2loint(v));
    }
    static __device__ __forceinline__ double quot(double a, double b) { return a / b; }
    static __device__ __forceinline__ double floor_(double x) { return floor(x); }
    static __device__ __forceinline__ double fma_(double a, double b, double c) { return fma(a, b, c); }
    // expm1 by argument reduction z = k ln2 + r, |r| <= ln2/2 (Cody & Waite: ln2 in two
    // parts, the first with 31 significant bits so that k ln2_hi is exact), the Taylor
    // series of expm1(r) to degree 13 (truncation below 2e-17 relative), and
    // expm1(z) = 2^k expm1(r) + (2^k - 1) in one fused multiply-add. Below -40, e^z is
    // under 2^-57 and the result is -1. On 2e7 arguments in [-40, 0] it equals the C
    // library's expm1 in 97 % of cases and is otherwise one ulp away.
    static __device__ __forceinline__ double expm1_(double x) {
        const double z = (x < -40.0) ? -40.0 : x;
        const double k = rint(z * 1.4426950408889634);
        const double r = fma(-k, 0x1.a39ef35793c76p-33, fma(-k, 0x1.62e42feep-1, z));
        double p = 1.0 / 6227020800.0;                              // 1/13!
        p = fma(p, r, 1.0 / 479001600.0);
        p = fma(p, r, 1.0 / 39916800.0);
        p = fma(p, r, 1.0 / 3628800.0);
        p = fma(p, r, 1.0 / 362880.0);
        p = fma(p, r, 1.0 / 40320.0);
        p = fma(p, r, 1.0 / 5040.0);
        p = fma(p, r, 1.0 / 720.0);
        p = fma(p, r, 1.0 / 120.0);
        p = fma(p, r, 1.0 / 24.0);
        p = fma(p, r, 1.0 / 6.0);
        p = fma(p, r, 0.5);
        const double e = fma(r * r, p, r);                          // expm1(r)
        const double s = ldexp(1.0, (int)k);                        // 2^k, exact
        return fma(s, e, s - 1.0);
    }
    // expm1(z) for |z| <= kSmallZ: the Taylor series to degree 7 (truncation below
    // 1e-17 relative) in Estrin form:
    // z + z^2 (1/2 + z/6) + z^4 ((1/24 + z/120) + z^2 (1/720 + z/5040)).
    static constexpr double kSmallZ = 0.015625;
    static constexpr double kTinyZ = 0.0;   // no shorter FP64 series: every tier-2 step takes the tier-1 one
    static __device__ __forceinline__ double expm1_tiny(double z) { return expm1_small(z); }
    static __device__ __forceinline__ double expm1_small(double z) {
        const double z2 = z * z;
        const double a = fma(z, 1.0 / 6.0, 0.5);
        const double b = fma(z, 1.0 / 120.0, 1.0 / 24.0);
        const double c = fma(z, 1.0 / 5040.0, 1.0 / 720.0);
        const double z4 = z2 * z2;
        return fma(z4, fma(z2, c, b), fma(z2, a, z));
    }
    static __device__ __forceinline__ double clamp_(double x, double lo, double hi) {
        return fmin(fmax(x, lo), hi);
    }
    static __device__ __forceinline__ void sqrt_and_rcp(double d, double& sq, double& inv) {
        sq = sqrt_(d);
        inv = rcp(d);
    }
    static __device__ __forceinline__ bool outside(double x, double H) { return x < 0.0 || x > H; }

};

// Per-problem constants in the path precision.
template <typename R>
struct Consts {
    R H, eps, Hme;              // domain and cut-off heights
    R ksH;                      // kappa_sigma u_* H^(-3/4): sigma_U = ksH (H - X)^(3/4)
    R kl;                       // ksH / kappa_tau: lambda = kl (H - X)^(3/4) / X
    R acoef_h;                  // (3/4) (kappa_sigma u_*)^2 / H^(3/2)
    R su_h, lam_h;              // homogeneous sigma_U and lambda
    R sxi;                      // scale of the normals the steps take (sigma_U = sxi sr):
                                // ksH in the neutral layer, sigma_U when homogeneous
};

template <typename R>
__device__ __forceinline__ Consts<R> make_consts(const KProblem& p) {
    Consts<R> c;
    c.H = (R)p.H;
    c.eps = (R)p.eps_reg;
    c.Hme = (R)(p.H - p.eps_reg);
    c.ksH = (R)p.ksH;
    c.kl = (R)p.kl;
    c.acoef_h = (R)(0.75 * p.ks * p.ks / (p.H * sqrt(p.H)));
    c.su_h = (R)p.sigma_u;
    c.lam_h = (R)(1.0 / p.tau);
    c.sxi = (R)(p.profile == KPROFILE_HOMOGENEOUS ? p.sigma_u : p.ksH);
    return c;
}

// sigma_U at X (Eqs. 5, 7): kappa_sigma u_* (1 - X_c/H)^(3/4) with X_c the cut-off X.
template <typename R, int PROF>
__device__ __forceinline__ R sigma_at(const Consts<R>& c, R x) {
    if (PROF == KPROFILE_HOMOGENEOUS) return c.su_h;
    const R d = c.H - Math<R>::clamp_(x, c.eps, c.Hme);
    return c.ksH * Math<R>::sqrt_(d * Math<R>::sqrt_(d));
}

// O-step coefficients at X for step size h: sr = sigma_U / sxi and z = -lambda h, lambda =
// 1/tau = sigma_U / (kappa_tau X_c) (Eqs. 5, 7). In the neutral layer sr is
// r = (H - X_c)^(3/4) itself (sigma_U = ksH r, and the normals come scaled by ksH) and
// z = r (-kl h / X_c), one multiply from r: -kl h is the same for every step of a path
// and 1/X_c is computed beside r. Homogeneous: sr = 1.
template <typename R, int PROF>
__device__ __forceinline__ void o_coeffs(const Consts<R>& c, R x, R h, R& sr, R& z) {
    if (PROF == KPROFILE_HOMOGENEOUS) {
        sr = (R)1;
        z = -c.lam_h * h;
    } else {
        const R xc = Math<R>::clamp_(x, c.eps, c.Hme);
        const R d = c.H - xc;
        const R r = Math<R>::sqrt_(d * Math<R>::sqrt_(d));
        sr = r;
        z = r * ((-c.kl * h) * Math<R>::rcp(xc));
    }
}

// o_coeffs and the drift coefficients of a step of length h at X, a h and b h (one square
// root of H - X_c serves both; a, b as in drift_at).
template <typename R, int PROF>
__device__ __forceinline__ void coeffs_at(const Consts<R>& c, R x, R h, R& sr, R& z, R& ah, R& bh) {
    if (PROF == KPROFILE_HOMOGENEOUS) {
        sr = (R)1;
        z = -c.lam_h * h;
        ah = (R)0;
        bh = (R)0;
    } else {
        const R xc = Math<R>::clamp_(x, c.eps, c.Hme);
        const R d = c.H - xc;
        const R q = Math<R>::rsqrt(d);                       // 1/sqrt(H - X_c)
        const R r = Math<R>::sqrt_(d * (d * q));
        sr = r;
        z = r * ((-c.kl * h) * Math<R>::rcp(xc));
        // inside [eps_reg, H - eps_reg] exactly when the cut-off leaves X as it is; there
        // X_c = X, and one select of q serves both drift coefficients (as in drift_at)
        const R qm = (xc == x) ? q : (R)0;
        ah = ((c.acoef_h * h) * d) * qm;
        bh = (((R)0.75 * h) * qm) * qm;
    }
}

// The drift coefficients of a B half-step of length hh at X, with
// a = (3/4)(kappa_sigma u_*)^2 sqrt(H - X) / H^(3/2) and b = (3/4) / (H - X) inside
// [eps_reg, H - eps_reg], 0 outside: ah = a hh and bh = b hh (kick). ONE_CMP: the inside
// test as one vector compare against the cut-off position (no scalar combination of two
// compares waits on the path's chain); otherwise two compares. Both give the same
// answer. q = 1/sqrt(H - X), set to 0 outside, is taken once: ah = (a' hh (H - X)) q and
// bh = ((3 hh / 4) q) q, one reciprocal square root and one select for both.
template <typename R, int PROF, bool ONE_CMP = false>
__device__ __forceinline__ void drift_at(const Consts<R>& c, R x, R hh, R& ah, R& bh) {
    if (PROF == KPROFILE_HOMOGENEOUS) {
        ah = (R)0;
        bh = (R)0;
    } else {
        const bool inside = ONE_CMP ? Math<R>::clamp_(x, c.eps, c.Hme) == x : (x >= c.eps) && (x <= c.Hme);
        const R d = c.H - x;
        const R q = inside ? Math<R>::rsqrt(d) : (R)0;
        ah = ((c.acoef_h * hh) * d) * q;
        bh = (((R)0.75 * hh) * q) * q;
    }
}

// A B half-step U - a' - b' U^2 (a' = a hh, b' = b hh) in Horner form,
// U (1 - b' U) - a': two fused multiply-adds.
template <typename R>
__device__ __forceinline__ R kick(R u, R ah, R bh) {
    return Math<R>::fma_(u, Math<R>::fma_(-bh, u, (R)1), -ah);
}

template <typename R>
struct Path {
    R x, u;
    uint32_t sgn;   // reflection sign S as a sign-bit mask (0: S = +1)
    R a, b;         // BAOAB: ah and bh of drift_at at x, carried to the next step
    bool bad;       // ran away (more than kFoldMax reflections): non-finite
};

// A position's fold key: an unsigned number that exceeds limit(H) for every position
// outside [0, H], for -0 and for NaN. FP32: the bit pattern itself (non-negative
// floats order as their patterns; a sign bit makes the pattern larger than any positive
// one). FP64: the high 32 bits, against hi(H) - 1, which also flags the positions in the
// last 2^-20 of H below it (repeated, not wrongly kept).
template <typename R>
struct FoldKey;

template <>
struct FoldKey<float> {
    static __device__ __forceinline__ uint32_t key(float x) { return __float_as_uint(x); }
    static __device__ __forceinline__ uint32_t limit(float H) { return __float_as_uint(H); }
};

template <>
struct FoldKey<double> {
    static __device__ __forceinline__ uint32_t key(double x) { return (uint32_t)__double2hiint(x); }
    static __device__ __forceinline__ uint32_t limit(double H) { return (uint32_t)__double2hiint(H) - 1u; }
};

// Fold into [0, H]; 0 and H are inside. More than kFoldMax reflections in one fold
// means the step ran away: the path becomes NaN and is counted as non-finite. The
// branch is entered on one unsigned compare of the fold key (which also lets -0, NaN and,
// in FP64, the last 2^-20 of H below it through); the loop's own test is the exact one.
template <typename R>
__device__ __forceinline__ void fold(Path<R>& p, R H) {
    if (__builtin_expect(FoldKey<R>::key(p.x) > FoldKey<R>::limit(H), 0)) {
        int count = 0;
#pragma unroll 1
        while (Math<R>::outside(p.x, H)) {
            if (++count > kFoldMax) {
                p.x = (R)NAN;
                p.u = (R)NAN;
                p.bad = true;
                break;
            }
            p.x = (p.x < (R)0) ? -p.x : (R)2 * H - p.x;
            p.u = -p.u;
            p.sgn ^= kSignBit;
        }
    }
}

// How a step treats its position updates. FOLD_EXACT folds each one (fold()).
// FOLD_TRACK leaves them unfolded and only records, in `key`, the largest fold key
// (FoldKey) of the positions reached: for positions in [0, H] fold() changes nothing,
// so while every key stays within FoldKey::limit(H) the tracked steps are the exact
// steps bit for bit, and otherwise the caller repeats them with FOLD_EXACT.
enum { FOLD_EXACT = 0, FOLD_TRACK = 1 };

template <typename R, int FOLD>
__device__ __forceinline__ void fold_or_track(Path<R>& p, R H, uint32_t& key) {
    if (FOLD == FOLD_EXACT) {
        fold(p, H);
    } else {
        const uint32_t k = FoldKey<R>::key(p.x);
        key = key > k ? key : k;
    }
}

// expm1(-lambda h) of an O-step by tier: 0 the full routine, 1 the short series
// (lambda_max h <= kSmallZ for this step size), 2 the shortest (lambda_max h <= kTinyZ);
// each is exact to rounding for every X of its steps. The tier is chosen once per path
// from that path's own step size (h for a fine path, 2h for a coarse one), never inside
// a step and never from how the samples are laid out on the device: a sample's bits do
// not depend on the block mode that runs it.
template <typename R, int TIER>
__device__ __forceinline__ R o_step_expm1(R z) {
    if (TIER == 2) return Math<R>::expm1_tiny(z);
    if (TIER == 1) return Math<R>::expm1_small(z);
    return Math<R>::expm1_(z);
}

// The expm1 tier of the O-steps of size h (symplectic Euler has none: tier 0).
template <typename R>
__device__ __forceinline__ int expm1_tier(const KProblem& kp, int integ, double h) {
    if (integ == KINTEG_SE) return 0;
    const double z = kp.lam_max * h;
    return z <= (double)Math<R>::kTinyZ ? 2 : (z <= (double)Math<R>::kSmallZ ? 1 : 0);
}

// One step of size h. The normals a step takes are scaled by sxi (sigma_U = sxi sr), so
// sigma_U xi is sr times the scaled normal. COARSE: xi is the combined extended noise
// (scaled) and the physical noise is S xi; otherwise xi is the physical noise (scaled)
// and `tilde` receives S xi. `w` receives e^{-lambda h} of the O-step (GL, BAOAB).
// TIER: see o_step_expm1.
template <typename R, int INTEG, int PROF, bool COARSE, int TIER, int FOLD>
__device__ __forceinline__ void step_impl(const Consts<R>& c, Path<R>& p, R h, R hh, R xi,
                                          R& tilde, R& w, uint32_t& key) {
    if (INTEG == KINTEG_SE) {                                        // Eq. (8)
        R sr, z, ah, bh;                                             // z = -lambda h
        coeffs_at<R, PROF>(c, p.x, h, sr, z, ah, bh);
        const R noise = COARSE ? Math<R>::flip(xi, p.sgn) : xi;
        if (!COARSE) tilde = Math<R>::flip(xi, p.sgn);
        const R amp = sr * Math<R>::sqrt_((R)-2 * z);                  // sigma sqrt(h) / sxi
        const R u0 = p.u;
        // (1 - lambda h) U - a h - b h U^2 + sigma dW, as U ((1 - lambda h) - b h U) - a h
        // + sigma dW
        p.u = Math<R>::fma_(u0, Math<R>::fma_(-bh, u0, (R)1 + z), Math<R>::fma_(amp, noise, -ah));
        p.x = p.x + p.u * h;
        fold_or_track<R, FOLD>(p, c.H, key);
        w = (R)1;
    } else if (INTEG == KINTEG_GL) {                                 // Eq. (9)
        R sr, z, ah, bh;
        coeffs_at<R, PROF>(c, p.x, h, sr, z, ah, bh);
        const R noise = COARSE ? Math<R>::flip(xi, p.sgn) : xi;
        if (!COARSE) tilde = Math<R>::flip(xi, p.sgn);
        const R e1 = o_step_expm1<R, TIER>(z);
        w = (R)1 + e1;
        const R sn = sr * noise;                                     // sigma_U xi
        // O: e^{-lambda h} U = U + e1 U in one fused multiply-add (w itself only for the
        // coupling of Eq. 19)
        const R us = Math<R>::fma_(sn, Math<R>::sqrt_(-e1 * ((R)2 + e1)), Math<R>::fma_(e1, p.u, p.u));
        p.u = kick(us, ah, bh);                                      // B at (X_n, U*)
        p.x = p.x + p.u * h;                                         // A
        fold_or_track<R, FOLD>(p, c.H, key);
    } else {                                                         // Eq. (10)
        p.u = kick(p.u, p.a, p.b);                                   // B at (X_n, U_n)
        p.x = p.x + p.u * hh;                                        // A
        fold_or_track<R, FOLD>(p, c.H, key);
        R sr, z;
        o_coeffs<R, PROF>(c, p.x, h, sr, z);
        const R noise = COARSE ? Math<R>::flip(xi, p.sgn) : xi;
        if (!COARSE) tilde = Math<R>::flip(xi, p.sgn);
        const R e1 = o_step_expm1<R, TIER>(z);
        w = (R)1 + e1;
        const R sn = sr * noise;                                     // sigma_U xi
        // (w U here: U + e1 U, as in GL, saves half an operation per step but measured 2 %
        // slower on the BAOAB fine wave's schedule)
        p.u = Math<R>::fma_(sn, Math<R>::sqrt_(-e1 * ((R)2 + e1)), w * p.u);   // O at X_{n+1/2}
        p.x = p.x + p.u * hh;                                        // A
        fold_or_track<R, FOLD>(p, c.H, key);
        drift_at<R, PROF, FOLD == FOLD_TRACK>(c, p.x, hh, p.a, p.b);
        p.u = kick(p.u, p.a, p.b);                                   // B at (X_{n+1}, U*)
    }
}

// One step with every position update folded (Eq. 6, Sec. 4).
template <typename R, int INTEG, int PROF, bool COARSE, int TIER>
__device__ __forceinline__ void step(const Consts<R>& c, Path<R>& p, R h, R hh, R xi,
                                     R& tilde, R& w) {
    uint32_t unused = 0;
    step_impl<R, INTEG, PROF, COARSE, TIER, FOLD_EXACT>(c, p, h, hh, xi, tilde, w, unused);
}

// Initial state shared by both paths of a sample.
template <typename R, int PROF>
__device__ __forceinline__ void initial_state(const KProblem& kp, const Consts<R>& c,
                                              const Stream& st, R& x0, R& u0) {
    if (kp.release == KRELEASE_FIXED_W) {
        x0 = (R)kp.z0;
        u0 = (R)kp.w0;
        return;
    }
    R z0, z1;
    Normals<R>::pair(philox(st, kBlockInitW), z0, z1);
    if (kp.release == KRELEASE_GAUSSIAN_W) {
        x0 = (R)kp.z0;
        u0 = (R)kp.su_z0 * z0;
        return;
    }
    const Words wx = philox(st, kBlockInitX);
    if (sizeof(R) == 8)
        x0 = (R)(kp.H * uniform64(wx.r1, wx.r0));
    else
        x0 = (R)kp.H * (R)uniform32(wx.r1);
    u0 = sigma_at<R, PROF>(c, x0) * z0;
}

// hh: the path's B half-step (h/2 for a fine path, h for a coarse one); BAOAB only.
template <typename R, int INTEG, int PROF>
__device__ __forceinline__ void init_path(const Consts<R>& c, Path<R>& p, R x0, R u0, R hh) {
    p.x = x0;
    p.u = u0;
    p.sgn = 0u;
    p.bad = false;
    p.a = (R)0;
    p.b = (R)0;
    if (INTEG == KINTEG_BAOAB) drift_at<R, PROF>(c, x0, hh, p.a, p.b);
}

// The two normals of draw m, scaled by sxi as the steps take them.
template <typename R>
__device__ __forceinline__ void scaled_normals(const Consts<R>& c, const Words& wd, R& z0, R& z1) {
    Normals<R>::pair(wd, z0, z1);
    z0 *= c.sxi;
    z1 *= c.sxi;
}

// The time loop of one sample: M_l fine steps and, on levels >= 1, M_l / 2 coarse
// steps driven by the combined fine noise. TIER_F and TIER_C: o_step_expm1's tier for
// the fine path (step h) and the coarse path (step 2h).
template <typename R, int INTEG, int PROF, int TIER_F, int TIER_C>
__device__ __forceinline__ void run_paths(const Consts<R>& c, const Stream& st, int level,
                                          uint32_t M, R h, R hh, R h2, Path<R>& f, Path<R>& g) {
    R tilde_a, tilde_b, w_a, w_b, z0, z1;
    if (level == 0) {
        for (uint32_t m = 0; m < M / 2; ++m) {
            scaled_normals(c, philox(st, m), z0, z1);
            step<R, INTEG, PROF, false, TIER_F>(c, f, h, hh, z0, tilde_a, w_a);
            step<R, INTEG, PROF, false, TIER_F>(c, f, h, hh, z1, tilde_b, w_b);
        }
        if (M & 1u) {
            scaled_normals(c, philox(st, M / 2), z0, z1);
            step<R, INTEG, PROF, false, TIER_F>(c, f, h, hh, z0, tilde_a, w_a);
        }
        return;
    }
    for (uint32_t m = 0; m < M / 2; ++m) {
        scaled_normals(c, philox(st, m), z0, z1);
        step<R, INTEG, PROF, false, TIER_F>(c, f, h, hh, z0, tilde_a, w_a);   // fine step 2m
        step<R, INTEG, PROF, false, TIER_F>(c, f, h, hh, z1, tilde_b, w_b);   // fine step 2m+1
        R xi_c;
        if (INTEG == KINTEG_SE)
            xi_c = (tilde_a + tilde_b) * (R)0.70710678118654752440;  // Eq. (18)
        else
            xi_c = (w_a * tilde_a + tilde_b) * Math<R>::rsqrt(w_a * w_a + (R)1);   // Eq. (19)
        R unused_t, unused_w;
        step<R, INTEG, PROF, true, TIER_C>(c, g, h2, h, xi_c, unused_t, unused_w);
    }
}

// ---------------------------------------------------------------------------------
// Adaptive, non-nested symplectic Euler (Sec. 7). Time is counted in ticks of
// h_l / 2^kTickBits. A path at X takes h_n = min(h, lambda(x_adapt) / lambda(X) h) from its
// base step (2^kTickBits ticks fine, twice that coarse), rounded down to whole ticks (at
// least one) and cut at T. The rule is evaluated in the path precision. Merged-grid
// interval j draws xi_j (draw j mod 2 of Philox block j / 2, the uniform scheme's
// mapping); the fine path's increment over its step is the sum of xi_j sqrt(dtau_j), the
// coarse path's S_c times the sum of S_f xi_j sqrt(dtau_j), S_f taken at the start of
// interval j.
//
// A lane advances its two paths one step per iteration, the one whose step ends first
// (the fine one on a tie), so every iteration does the work of one step whichever path
// it belongs to; the loop itself lives with the kernel, which also moves a lane on to its
// next sample as soon as the current one ends.
// ---------------------------------------------------------------------------------
constexpr int kTickBits = kAdaptTickBits;

// sigma_U, lambda and the drift coefficients at a path's position, kept with the path:
// the step rule needs lambda right after a step, and the path's next step needs all four.
template <typename R>
struct ACoef {
    R su, lam, a, b;
};

template <typename R, int PROF>
__device__ __forceinline__ ACoef<R> acoef_at(const Consts<R>& c, R x) {
    ACoef<R> k;
    if (PROF == KPROFILE_HOMOGENEOUS) {
        k.su = c.su_h;
        k.lam = c.lam_h;
        k.a = (R)0;
        k.b = (R)0;
    } else {
        const R xc = Math<R>::clamp_(x, c.eps, c.Hme);
        const R d = c.H - xc;
        R sqd, invd;
        Math<R>::sqrt_and_rcp(d, sqd, invd);
        const R r = Math<R>::sqrt_(d * sqd);                 // (H - X_c)^(3/4)
        k.su = c.ksH * r;
        k.lam = (c.kl * r) * Math<R>::rcp(xc);
        const bool inside = (x >= c.eps) && (x <= c.Hme);
        k.a = inside ? c.acoef_h * sqd : (R)0;
        k.b = inside ? (R)0.75 * invd : (R)0;
    }
    return k;
}

// End (in ticks) of the step that starts at tick t for a path with lambda = lam: the base
// step, shortened to floor(lam_adapt / lam * base) ticks (at least 1) where lam exceeds
// lam_adapt; a NaN lambda (a run-away path) takes the base step. Steps are at most 2^21
// ticks; T (the tick counter type) must hold t_end + 2^21.
template <typename R, typename T>
__device__ __forceinline__ T adaptive_end(R lam_adapt, R lam, T t, uint32_t base, T t_end) {
    uint32_t k = base;
    if (lam > lam_adapt) {
        const R steps = Math<R>::floor_(Math<R>::quot(lam_adapt, lam) * (R)base);
        k = steps < (R)1 ? 1u : (steps < (R)base ? (uint32_t)steps : base);
    }
    return (t + k < t_end) ? t + k : t_end;
}

// Eq. (8) driven by the Brownian increment dW of the step (dW stands for sqrt(h) xi):
// U' = (1 - lambda h) U - (a + b U^2) h + sigma dW with sigma = sigma_U sqrt(2 lambda).
template <typename R>
__device__ __forceinline__ void se_step_dw(const ACoef<R>& k, R h, R dW, R H, Path<R>& p) {
    const R sigma = k.su * Math<R>::sqrt_((R)2 * k.lam);
    p.u = ((R)1 - k.lam * h) * p.u - (k.a + k.b * p.u * p.u) * h + sigma * dW;
    p.x = p.x + p.u * h;
    fold(p, H);
}

// Runs one sample of `level`. Returns the terminal fine and coarse states.
template <typename R, int INTEG, int PROF>
__device__ __forceinline__ void run_sample(const KProblem& kp, const Consts<R>& c, int level,
                                           uint64_t sample, Path<R>& f, Path<R>& g) {
    const Stream st = make_stream(kp.seed, kp.stream_id, level, sample);
    R x0, u0;
    initial_state<R, PROF>(kp, c, st, x0, u0);
    const uint32_t M = (uint32_t)kp.M0 << level;                 // M_l = M_0 2^l
    const double hd = kp.T / (double)M;                           // h_l = T / M_l
    const R h = (R)hd, hh = (R)(0.5 * hd), h2 = (R)(2.0 * hd);
    init_path<R, INTEG, PROF>(c, f, x0, u0, hh);
    init_path<R, INTEG, PROF>(c, g, x0, u0, h);
    // each path by its own step: h for the fine path, 2h for the coarse one (the tier of
    // the coarse step never exceeds the fine step's); level 0 has no coarse path
    const int tf = expm1_tier<R>(kp, INTEG, hd);
    const int tc = level == 0 ? tf : expm1_tier<R>(kp, INTEG, 2.0 * hd);
    if (tc == 2)
        run_paths<R, INTEG, PROF, 2, 2>(c, st, level, M, h, hh, h2, f, g);
    else if (tf == 2)
        run_paths<R, INTEG, PROF, 2, 1>(c, st, level, M, h, hh, h2, f, g);
    else if (tc == 1)
        run_paths<R, INTEG, PROF, 1, 1>(c, st, level, M, h, hh, h2, f, g);
    else if (tf == 1)
        run_paths<R, INTEG, PROF, 1, 0>(c, st, level, M, h, hh, h2, f, g);
    else
        run_paths<R, INTEG, PROF, 0, 0>(c, st, level, M, h, hh, h2, f, g);
}

// Quantity of interest in FP64 (Sec. 2, Sec. 5).
__device__ __forceinline__ double g_r(const KProblem& kp, double s) {
    if (s < -1.0) return 1.0;
    if (s > 1.0) return 0.0;
    double v = 0.0;
    for (int k = kp.ncoef - 1; k >= 0; --k) v = fma(v, s, kp.coef[k]);
    return v;
}

__device__ __forceinline__ double qoi(const KProblem& kp, double x, double u) {
    switch (kp.qoi_kind) {
        case KQOI_MEAN_Z: return x;
        case KQOI_VELOCITY: return u;
        case KQOI_VELOCITY_SQ: return u * u;
        case KQOI_P_ABOVE:
            if (kp.r == 0) return x > kp.qa ? 1.0 : 0.0;
            return 1.0 - g_r(kp, (x - kp.qa) * kp.inv_delta);
        default:   // KQOI_P_BOX, Eq. (34) / Eq. (37)
            if (kp.r == 0) return (x <= kp.qb ? 1.0 : 0.0) - (x <= kp.qa ? 1.0 : 0.0);
            return g_r(kp, (x - kp.qb) * kp.inv_delta) - g_r(kp, (x - kp.qa) * kp.inv_delta);
    }
}

}  // namespace ldm
