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

template <>
struct Normals<double> {
    // rho = sqrt(-2 ln u); (rho cos 2 pi v, rho sin 2 pi v)
    static __device__ __forceinline__ void pair(const Words& w, double& z0, double& z1) {
        const double u = uniform64(w.r1, w.r0);
        const double v = uniform64(w.r3, w.r2);
        const double rho = sqrt(-2.0 * log(u));
        double s, c;
        sincos(6.283185307179586 * v, &s, &c);
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
