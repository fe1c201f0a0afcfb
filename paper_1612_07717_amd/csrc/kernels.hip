// kernels.hip -- level-sum kernels for gfx950.
//
// level_kernel: one coupled sample per lane at a time (each lane runs `spl` samples of
// its block's range), the fine and coarse paths entirely in registers; no input
// arrays. Each lane keeps Neumaier (compensated) FP64 sums of Y_l, Y_l^2, P_l, P_l^2
// (Eq. 16); a wave combines them with xor-shuffles, the four waves of a block through
// LDS, and the block writes one 80-byte partial. merge_kernel then combines each
// item's partials in a fixed order. No atomics: results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_model.hpp"
#include "ld_internal.hpp"

namespace ldm {

struct Acc {
    double s[4];
    double c[4];
    uint64_t n;
    uint64_t nbad;
};

__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
    const double t = s + x;
    const double big = (fabs(s) >= fabs(x)) ? s : x;
    const double small = (fabs(s) >= fabs(x)) ? x : s;
    c += (big - t) + small;
    s = t;
}

// Adds the compensated pair (s2, c2) to (s, c). Symmetric in its two operands, so
// both lanes of a shuffle pair hold identical results.
__device__ __forceinline__ void neumaier_merge(double& s, double& c, double s2, double c2) {
    const double t = s + s2;
    const double big = (fabs(s) >= fabs(s2)) ? s : s2;
    const double small = (fabs(s) >= fabs(s2)) ? s2 : s;
    c = (c + c2) + ((big - t) + small);
    s = t;
}

__device__ __forceinline__ void acc_zero(Acc& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a.s[k] = 0.0;
        a.c[k] = 0.0;
    }
    a.n = 0;
    a.nbad = 0;
}

// Wave (64 lanes) then block (kBlock / 64 waves, fixed order) reduction; the result is
// valid in thread 0.
__device__ __forceinline__ void block_reduce(Acc& a) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double so = __shfl_xor(a.s[k], off, 64);
            const double co = __shfl_xor(a.c[k], off, 64);
            neumaier_merge(a.s[k], a.c[k], so, co);
        }
        a.n += __shfl_xor(a.n, off, 64);
        a.nbad += __shfl_xor(a.nbad, off, 64);
    }
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh_s[kWaves][4], sh_c[kWaves][4];
    __shared__ uint64_t sh_n[kWaves], sh_bad[kWaves];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sh_s[wave][k] = a.s[k];
            sh_c[wave][k] = a.c[k];
        }
        sh_n[wave] = a.n;
        sh_bad[wave] = a.nbad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kWaves; ++w) {
#pragma unroll
            for (int k = 0; k < 4; ++k) neumaier_merge(a.s[k], a.c[k], sh_s[w][k], sh_c[w][k]);
            a.n += sh_n[w];
            a.nbad += sh_bad[w];
        }
    }
}

// Wave index as a scalar (uniform) value: branches on it are scalar branches.
__device__ __forceinline__ uint32_t wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Block reduction for loops that take work item by item (persistent and grid-stride
// kernels): like block_reduce, but every thread ends with the block total (the wave
// results are merged in the same fixed order by all threads), so no single-lane
// region sits at the end of a loop body. Ends with a barrier: LDS may be reused.
__device__ __forceinline__ void block_reduce_all(Acc& a) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double so = __shfl_xor(a.s[k], off, 64);
            const double co = __shfl_xor(a.c[k], off, 64);
            neumaier_merge(a.s[k], a.c[k], so, co);
        }
        a.n += __shfl_xor(a.n, off, 64);
        a.nbad += __shfl_xor(a.nbad, off, 64);
    }
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh_s[kWaves][4], sh_c[kWaves][4];
    __shared__ uint64_t sh_n[kWaves], sh_bad[kWaves];
    const uint32_t wave = wave_index();
    // every lane of a wave holds the wave total; all of them store the same values
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sh_s[wave][k] = a.s[k];
        sh_c[wave][k] = a.c[k];
    }
    sh_n[wave] = a.n;
    sh_bad[wave] = a.nbad;
    __syncthreads();
    Acc t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        t.s[k] = sh_s[0][k];
        t.c[k] = sh_c[0][k];
    }
    t.n = sh_n[0];
    t.nbad = sh_bad[0];
    for (int w = 1; w < kWaves; ++w) {
#pragma unroll
        for (int k = 0; k < 4; ++k) neumaier_merge(t.s[k], t.c[k], sh_s[w][k], sh_c[w][k]);
        t.n += sh_n[w];
        t.nbad += sh_bad[w];
    }
    a = t;
    __syncthreads();
}

__device__ __forceinline__ void store_sums(ld_level_sums* out, const Acc& a) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        out->s[k] = a.s[k];
        out->c[k] = a.c[k];
    }
    out->n = a.n;
    out->n_nonfinite = a.nbad;
}

template <typename R, int INTEG, int PROF>
__device__ __forceinline__ void sample_qoi(const KProblem& kp, const Consts<R>& c, int level,
                                           uint64_t sample, double& pf, double& pc, bool& bad) {
    Path<R> f, g;
    run_sample<R, INTEG, PROF>(kp, c, level, sample, f, g);
    pf = qoi(kp, (double)f.x, (double)f.u);
    pc = (level == 0) ? 0.0 : qoi(kp, (double)g.x, (double)g.u);
    bad = f.bad || (level != 0 && g.bad) || !isfinite(pf) || !isfinite(pc);
}

// Branch-free: a non-finite sample contributes exact zeros (adding 0 leaves a
// compensated pair unchanged) and is only counted.
__device__ __forceinline__ void accumulate(Acc& acc, double pf, double pc, bool bad) {
    const double y = bad ? 0.0 : pf - pc;
    const double p = bad ? 0.0 : pf;
    neumaier_add(acc.s[0], acc.c[0], y);
    neumaier_add(acc.s[1], acc.c[1], y * y);
    neumaier_add(acc.s[2], acc.c[2], p);
    neumaier_add(acc.s[3], acc.c[3], p * p);
    acc.n += bad ? 0u : 1u;
    acc.nbad += bad ? 1u : 0u;
}

// PIPE mode (coupled levels only): 64 samples per block. Waves 0 and 1 draw the
// (scaled) normals of alternate coarse steps of a chunk, wave 2 advances the fine paths
// over the chunk before and wave 3 the coarse paths over the chunk before that. The
// coarse wave forms S xi itself from the normals and the fine path's S over the chunk,
// which the fine wave publishes once per chunk with e^{-lambda h} of every first step of
// a pair. Normals are triple-buffered (drawn, fine, coarse), messages double-buffered;
// one barrier per chunk of pipe_chunk<R>() coarse steps; the arithmetic per path is that of
// STREAM mode.
// Coarse steps per chunk: 16 for FP32 paths, whose chunks are unrolled whole (a chunk's
// fixed cost, the saved state, the LDS addresses, the repeat test and the barrier,
// spread over 32 fine steps; FP32 level 12 of the single large workload 7 % faster than
// with 8), kPipeChunk = 8 for FP64 paths (twice the LDS per element, and the compiler's
// own unrolling: forcing it spills).
template <typename R>
constexpr int pipe_chunk() { return sizeof(R) == 4 ? 2 * kPipeChunk : kPipeChunk; }

// for (j = 0; j < pipe_chunk<R>(); ++j) body(j), unrolled whole for FP32 paths, left to the
// compiler for FP64 ones.
template <typename R, typename F>
__device__ __forceinline__ void chunk_loop(F&& body) {
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int j = 0; j < pipe_chunk<R>(); ++j) body(j);
    } else {
        for (int j = 0; j < pipe_chunk<R>(); ++j) body(j);
    }
}

template <typename R>
struct PipeLds {
    R nrm[3][pipe_chunk<R>()][2][64];   // scaled normals of a chunk (S xi after a repeated chunk)
    R msg[2][pipe_chunk<R>()][64];      // fine -> coarse: e^{-lambda h} of fine step 2m
    uint32_t sgn[2][64];           // fine -> coarse: the fine path's S over the chunk
    double end_pc[64];
    int end_bad[64];
};

// Fine wave of a wave-specialised block: K fine step pairs of one chunk (fine steps
// 2m, 2m + 1 for m = m0 .. m0 + K - 1 below P), reading the normals of buffer b3. The
// chunk runs first without folds, tracking how far its positions went (FOLD_TRACK): a
// path stays in [0, H] on almost every chunk, and then no position test or branch sits
// on the chain of its steps and S is the same for the whole chunk. A lane whose
// positions left [0, H] repeats the chunk from its saved state with folded steps,
// writes each step's S xi over its normal and publishes S = +1, so every lane ends with
// the folded steps' results bit for bit and the coarse wave reads the right S xi
// either way. FULL: all K step pairs lie below P (every chunk but a ragged last one),
// so the tracked pass has no per-pair test and is one straight run.
template <typename R, int INTEG, int PROF, int TIER, bool FULL>
__device__ __forceinline__ void pipe_fine_chunk(const Consts<R>& c, Path<R>& p, R h, R hh,
                                                PipeLds<R>& L, uint32_t b3, uint32_t b2,
                                                uint32_t m0, uint32_t P, int lane) {
    const Path<R> p0 = p;
    uint32_t key = 0;
    chunk_loop<R>([&](int j) {
        if (FULL || m0 + j < P) {
            R ta, tb, wa, wb;
            step_impl<R, INTEG, PROF, false, TIER, FOLD_TRACK>(c, p, h, hh, L.nrm[b3][j][0][lane], ta, wa, key);
            step_impl<R, INTEG, PROF, false, TIER, FOLD_TRACK>(c, p, h, hh, L.nrm[b3][j][1][lane], tb, wb, key);
            if (INTEG != KINTEG_SE) L.msg[b2][j][lane] = wa;
        }
    });
    const bool repeat = key > FoldKey<R>::limit(c.H);
    L.sgn[b2][lane] = repeat ? 0u : p0.sgn;
    if (__builtin_expect(repeat, 0)) {
        p = p0;
#pragma unroll 1
        for (int j = 0; j < pipe_chunk<R>(); ++j) {
            if (m0 + j < P) {
                R ta, tb, wa, wb;
                step<R, INTEG, PROF, false, TIER>(c, p, h, hh, L.nrm[b3][j][0][lane], ta, wa);
                step<R, INTEG, PROF, false, TIER>(c, p, h, hh, L.nrm[b3][j][1][lane], tb, wb);
                L.nrm[b3][j][0][lane] = ta;
                L.nrm[b3][j][1][lane] = tb;
                if (INTEG != KINTEG_SE) L.msg[b2][j][lane] = wa;
            }
        }
    }
}

// Coarse wave: the K coarse steps of one chunk, each driven by the combined noise of
// its fine pair (Eq. 18 for SE, Eq. 19 otherwise). Like the fine wave, the chunk runs
// without folds first and a lane whose positions left [0, H] repeats it with them.
template <typename R, int INTEG, int PROF, int FOLD, int TIER>
__device__ __forceinline__ void coarse_steps(const Consts<R>& c, Path<R>& p, R h2, R h,
                                             PipeLds<R>& L, uint32_t b3, uint32_t b2,
                                             uint32_t m0, uint32_t P, int lane, uint32_t& key) {
    const uint32_t sf = L.sgn[b2][lane];
    chunk_loop<R>([&](int j) {
        if (m0 + j < P) {
            const R ta = Math<R>::flip(L.nrm[b3][j][0][lane], sf);
            const R tb = Math<R>::flip(L.nrm[b3][j][1][lane], sf);
            R xi_c;
            if (INTEG == KINTEG_SE) {
                xi_c = (ta + tb) * (R)0.70710678118654752440;             // Eq. (18)
            } else {
                const R wa = L.msg[b2][j][lane];
                xi_c = (wa * ta + tb) * Math<R>::rsqrt(wa * wa + (R)1);  // Eq. (19)
            }
            R unused_t, unused_w;
            step_impl<R, INTEG, PROF, true, TIER, FOLD>(c, p, h2, h, xi_c, unused_t, unused_w, key);
        }
    });
}

template <typename R, int INTEG, int PROF, int TIER>
__device__ __forceinline__ void pipe_coarse_chunk(const Consts<R>& c, Path<R>& p, R h2, R h,
                                                  PipeLds<R>& L, uint32_t b3, uint32_t b2,
                                                  uint32_t m0, uint32_t P, int lane) {
    const Path<R> p0 = p;
    uint32_t key = 0;
    coarse_steps<R, INTEG, PROF, FOLD_TRACK, TIER>(c, p, h2, h, L, b3, b2, m0, P, lane, key);
    if (__builtin_expect(key > FoldKey<R>::limit(c.H), 0)) {
        p = p0;
        coarse_steps<R, INTEG, PROF, FOLD_EXACT, TIER>(c, p, h2, h, L, b3, b2, m0, P, lane, key);
    }
}

// The fine wave's chunk with o_step_expm1's tier TIER, or (TIER < 0) the tier `tier`
// chosen at run time, chunk by chunk.
template <typename R, int INTEG, int PROF, int TIER, bool FULL>
__device__ __forceinline__ void fine_chunk_tier(int tier, const Consts<R>& c, Path<R>& p, R h, R hh,
                                                PipeLds<R>& L, uint32_t b3, uint32_t b2,
                                                uint32_t m0, uint32_t P, int lane) {
    if constexpr (TIER >= 0) {
        pipe_fine_chunk<R, INTEG, PROF, TIER, FULL>(c, p, h, hh, L, b3, b2, m0, P, lane);
    } else if (tier == 2) {
        pipe_fine_chunk<R, INTEG, PROF, 2, FULL>(c, p, h, hh, L, b3, b2, m0, P, lane);
    } else if (tier == 1) {
        pipe_fine_chunk<R, INTEG, PROF, 1, FULL>(c, p, h, hh, L, b3, b2, m0, P, lane);
    } else {
        pipe_fine_chunk<R, INTEG, PROF, 0, FULL>(c, p, h, hh, L, b3, b2, m0, P, lane);
    }
}

template <typename R, int INTEG, int PROF, int TIER>
__device__ __forceinline__ void coarse_chunk_tier(int tier, const Consts<R>& c, Path<R>& p, R h2, R h,
                                                  PipeLds<R>& L, uint32_t b3, uint32_t b2,
                                                  uint32_t m0, uint32_t P, int lane) {
    if constexpr (TIER >= 0) {
        pipe_coarse_chunk<R, INTEG, PROF, TIER>(c, p, h2, h, L, b3, b2, m0, P, lane);
    } else if (tier == 2) {
        pipe_coarse_chunk<R, INTEG, PROF, 2>(c, p, h2, h, L, b3, b2, m0, P, lane);
    } else if (tier == 1) {
        pipe_coarse_chunk<R, INTEG, PROF, 1>(c, p, h2, h, L, b3, b2, m0, P, lane);
    } else {
        pipe_coarse_chunk<R, INTEG, PROF, 0>(c, p, h2, h, L, b3, b2, m0, P, lane);
    }
}

// TF, TC: o_step_expm1's tiers of the fine and the coarse path, fixed for the block (no
// chunk re-tests them), or -1: each chunk takes them from the path's step (see
// pipe_samples).
template <typename R, int INTEG, int PROF, int TF, int TC>
__device__ __forceinline__ void pipe_samples_t(const KProblem& kp, const Consts<R>& c,
                                               const KItem& item, uint32_t local_block, Acc& acc,
                                               double* dump, PipeLds<R>& L) {
    constexpr int K = pipe_chunk<R>();
    auto& nrm = L.nrm;
    auto& end_pc = L.end_pc;
    auto& end_bad = L.end_bad;
    const int wave = (int)wave_index(), lane = threadIdx.x & 63;   // roles: scalar branches
    const uint64_t local = (uint64_t)local_block * 64 + lane;
    const bool active = local < item.n_samples;
    const int level = item.level;
    const uint32_t M = (uint32_t)kp.M0 << level;
    const uint32_t P = M / 2;
    const uint32_t nch = (P + K - 1) / K;
    const double hd = kp.T / (double)M;
    const R h = (R)hd, hh = (R)(0.5 * hd), h2 = (R)(2.0 * hd);
    const int tier_f = TF >= 0 ? TF : expm1_tier<R>(kp, INTEG, hd);
    const int tier_c = TC >= 0 ? TC : expm1_tier<R>(kp, INTEG, 2.0 * hd);
    const Stream st = make_stream(kp.seed, kp.stream_id, level, item.sample_begin + local);
    Path<R> p;
    if (wave >= 2) {
        R x0, u0;
        initial_state<R, PROF>(kp, c, st, x0, u0);
        init_path<R, INTEG, PROF>(c, p, x0, u0, wave == 2 ? hh : h);   // fine or coarse B half-step
    }
    // phase s: the normal waves fill chunk s (buffer s mod 3), the fine wave runs chunk
    // s - 1 and the coarse wave chunk s - 2
    uint32_t r3 = 0;   // s mod 3
    for (uint32_t s = 0; s < nch + 2; ++s) {
        if (wave < 2) {
            if (s < nch) {
#pragma unroll
                for (int j = 0; j < K; j += 2) {
                    const uint32_t m = s * K + j + wave;
                    if (m < P) {
                        R z0, z1;
                        scaled_normals(c, philox(st, m), z0, z1);
                        nrm[r3][j + wave][0][lane] = z0;
                        nrm[r3][j + wave][1][lane] = z1;
                    }
                }
            }
        } else if (wave == 2) {
            if (s >= 1 && s <= nch) {
                const uint32_t b3 = r3 == 0 ? 2u : r3 - 1, b2 = (s - 1) & 1, m0 = (s - 1) * K;
                if (m0 + K <= P)
                    fine_chunk_tier<R, INTEG, PROF, TF, true>(tier_f, c, p, h, hh, L, b3, b2, m0, P, lane);
                else
                    fine_chunk_tier<R, INTEG, PROF, TF, false>(tier_f, c, p, h, hh, L, b3, b2, m0, P, lane);
            }
        } else {
            if (s >= 2) {
                const uint32_t b3 = r3 == 2 ? 0u : r3 + 1, b2 = s & 1, m0 = (s - 2) * K;   // (s - 2) mod 3, mod 2
                coarse_chunk_tier<R, INTEG, PROF, TC>(tier_c, c, p, h2, h, L, b3, b2, m0, P, lane);
            }
        }
        r3 = r3 == 2 ? 0u : r3 + 1;
        __syncthreads();
    }
    if (wave == 3) {
        end_pc[lane] = qoi(kp, (double)p.x, (double)p.u);
        end_bad[lane] = p.bad ? 1 : 0;
    }
    __syncthreads();
    if (wave == 2 && active) {
        const double pf = qoi(kp, (double)p.x, (double)p.u);
        const double pc = end_pc[lane];
        const bool bad = p.bad || end_bad[lane] != 0 || !isfinite(pf) || !isfinite(pc);
        if (dump != nullptr) {
            dump[2 * local] = pf;
            dump[2 * local + 1] = pc;
        }
        accumulate(acc, pf, pc, bad);
    }
}

// Wave priority (s_setprio takes an immediate): the longest paths of a launch first.
// A PIPE block's samples, with o_step_expm1's tier per path from its own step (h fine, 2h
// coarse; PIPE levels are >= 1), as in run_sample. The coarse tier never exceeds the fine
// one, FP64 has no tier 2 and symplectic Euler none but 0. FP32 blocks fix the tiers for
// the whole block: the fine wave's chunk is then one straight run (level 12 of the single
// large workload 7 % faster). FP64 blocks choose them chunk by chunk: fixed tiers made FP64
// level 12 alone 5 % faster but the estimate, whose long levels share CUs with each other
// and with the short levels' launch, 3 % slower.
template <typename R, int INTEG, int PROF>
__device__ __forceinline__ void pipe_samples(const KProblem& kp, const Consts<R>& c,
                                             const KItem& item, uint32_t local_block, Acc& acc,
                                             double* dump, PipeLds<R>& L) {
    if constexpr (INTEG == KINTEG_SE) {
        pipe_samples_t<R, INTEG, PROF, 0, 0>(kp, c, item, local_block, acc, dump, L);
    } else if constexpr (sizeof(R) == 8) {
        pipe_samples_t<R, INTEG, PROF, -1, -1>(kp, c, item, local_block, acc, dump, L);
    } else {
        const double hd = kp.T / (double)((uint32_t)kp.M0 << item.level);
        const int tf = expm1_tier<R>(kp, INTEG, hd);
        const int tc = expm1_tier<R>(kp, INTEG, 2.0 * hd);
        if (tc == 2)
            pipe_samples_t<R, INTEG, PROF, 2, 2>(kp, c, item, local_block, acc, dump, L);
        else if (tf == 2)
            pipe_samples_t<R, INTEG, PROF, 2, 1>(kp, c, item, local_block, acc, dump, L);
        else if (tc >= 1)
            pipe_samples_t<R, INTEG, PROF, 1, 1>(kp, c, item, local_block, acc, dump, L);
        else if (tf >= 1)
            pipe_samples_t<R, INTEG, PROF, 1, 0>(kp, c, item, local_block, acc, dump, L);
        else
            pipe_samples_t<R, INTEG, PROF, 0, 0>(kp, c, item, local_block, acc, dump, L);
    }
}

__device__ __forceinline__ void set_priority(uint32_t prio) {
    switch (prio) {
        case 3: __builtin_amdgcn_s_setprio(3); break;
        case 2: __builtin_amdgcn_s_setprio(2); break;
        case 1: __builtin_amdgcn_s_setprio(1); break;
        default: __builtin_amdgcn_s_setprio(0); break;
    }
}

// One wave's samples with adaptive symplectic Euler steps (Sec. 7): the contiguous chunk
// [c_begin, c_end) of the item's range. Adaptive paths differ in length, so samples are
// handed out as lanes free up: every iteration the wave counts (ballot) the lanes whose
// sample ended, gives them the next indices of the chunk in lane order and moves its
// shared cursor on. A wave runs in lockstep, so the assignment, and with it each lane's
// order of accumulation, is a function of the inputs alone: results are reproducible
// bit for bit. The loop is flat: a lane finishes one sample and starts the next in the
// same iteration, and lanes go idle only once the chunk is used up.
//
// Normals: interval j takes normal j of the sample's stream (component j mod 2 of Philox
// block j / 2). A lane uses at most one per iteration; it keeps up to three in a queue and
// refills it (one block, two normals) only on its even iterations, when fewer than two
// are left, so the lanes of a wave generate blocks together on every other iteration
// instead of each on its own. A new sample enters with its first block drawn.
// T: tick counter type, 32 bits when T in ticks fits.
template <typename R, int PROF, typename T>
__device__ __forceinline__ void adaptive_lane(const KProblem& kp, const Consts<R>& c, const KItem& item,
                                              uint64_t c_begin, uint64_t c_end, Acc& acc, double* dump) {
    const int level = item.level;
    const bool coupled = level != 0;
    const uint64_t M = (uint64_t)kp.M0 << level;                   // M_l = M_0 2^l
    const uint32_t base = 1u << kTickBits;                         // h_l in ticks
    const T t_end = (T)(M << kTickBits);                           // T in ticks
    const R tick = (R)((kp.T / (double)M) / (double)base);
    // lambda(x_adapt) by the same arithmetic as lambda(X): with x_adapt at the cut-off no
    // path's lambda exceeds it, and the scheme is the uniform one exactly
    const R lam_a = acoef_at<R, PROF>(c, (R)kp.x_adapt).lam;

    Stream st = make_stream(kp.seed, kp.stream_id, level, 0);
    Path<R> f, g;
    ACoef<R> kf, kg;
    T tf = 0, tc = 0, ef = 0, ec = 0, tau = 0;
    uint32_t it = 0, blk = 0, cnt = 0;   // it: own iterations; blk: next Philox block
    R wf = (R)0, wc = (R)0, q0 = (R)0, q1 = (R)0, q2 = (R)0;
    uint64_t cur = 0, cursor = c_begin;  // the lane's sample; the wave's next free index
    bool fresh = true;
    for (;;) {
        // hand the next indices of the chunk to the lanes whose sample ended (all lanes
        // still in the loop take part, so every copy of the cursor stays the same)
        const bool need = fresh || (tf == t_end && (!coupled || tc == t_end));
        const uint64_t mask = __ballot(need);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const uint64_t mine = cursor + rank;
        cursor += (uint64_t)__popcll(mask);
        // one divergent branch per iteration: finish the sample that ended, start the next
        if (need) {
            if (!fresh) {
                const double pf = qoi(kp, (double)f.x, (double)f.u);
                const double pc = coupled ? qoi(kp, (double)g.x, (double)g.u) : 0.0;
                const bool bad = f.bad || (coupled && g.bad) || !isfinite(pf) || !isfinite(pc);
                if (dump != nullptr) {
                    dump[2 * cur] = pf;
                    dump[2 * cur + 1] = pc;
                }
                accumulate(acc, pf, pc, bad);
            }
            if (mine >= c_end) break;
            cur = mine;
            st = make_stream(kp.seed, kp.stream_id, level, item.sample_begin + cur);
            R x0, u0;
            initial_state<R, PROF>(kp, c, st, x0, u0);
            init_path<R, KINTEG_SE, PROF>(c, f, x0, u0, (R)0);
            init_path<R, KINTEG_SE, PROF>(c, g, x0, u0, (R)0);
            kf = acoef_at<R, PROF>(c, x0);
            kg = kf;
            tf = tc = tau = 0;
            wf = wc = (R)0;
            ef = adaptive_end(lam_a, kf.lam, (T)0, base, t_end);
            ec = coupled ? adaptive_end(lam_a, kg.lam, (T)0, 2u * base, t_end) : t_end;
            Normals<R>::pair(philox(st, 0u), q0, q1);
            blk = 1;
            cnt = 2;
            fresh = false;
        }
        if ((it & 1u) == 0u && cnt < 2u) {   // refill: append normals 2 blk, 2 blk + 1
            R a, b;
            Normals<R>::pair(philox(st, blk), a, b);
            ++blk;
            if (cnt == 0u) q0 = a;
            q1 = (cnt == 0u) ? b : a;
            q2 = b;
            cnt += 2u;
        }
        ++it;
        // the next event: the end of the fine step or of the coarse step, fine first on a tie
        const bool fine_ev = (tf < t_end) && (!coupled || ef <= ec);
        const T e = fine_ev ? ef : ec;
        // a new merged interval [tau, e] takes the next normal; an event at tau (the second
        // step ending at a shared time point) adds exact zeros
        const bool adv = e > tau;
        const R dW = q0 * Math<R>::sqrt_((R)(uint32_t)(e - tau) * tick);
        q0 = adv ? q1 : q0;
        q1 = adv ? q2 : q1;
        cnt -= adv ? 1u : 0u;
        wf += dW;
        wc += Math<R>::flip(dW, f.sgn);      // S_f at the start of the interval
        tau = e;
        // one step of the path whose step ends at e, field by field (no path copies)
        Path<R> p;
        p.x = fine_ev ? f.x : g.x;
        p.u = fine_ev ? f.u : g.u;
        p.sgn = fine_ev ? f.sgn : g.sgn;
        p.bad = fine_ev ? f.bad : g.bad;
        p.a = (R)0;
        p.b = (R)0;
        ACoef<R> kc;
        kc.su = fine_ev ? kf.su : kg.su;
        kc.lam = fine_ev ? kf.lam : kg.lam;
        kc.a = fine_ev ? kf.a : kg.a;
        kc.b = fine_ev ? kf.b : kg.b;
        const R h = (R)(uint32_t)(e - (fine_ev ? tf : tc)) * tick;
        const R dWs = fine_ev ? wf : Math<R>::flip(wc, g.sgn);
        se_step_dw(kc, h, dWs, c.H, p);
        const ACoef<R> kn = acoef_at<R, PROF>(c, p.x);
        const T en = adaptive_end(lam_a, kn.lam, e, fine_ev ? base : 2u * base, t_end);
        f.x = fine_ev ? p.x : f.x;
        f.u = fine_ev ? p.u : f.u;
        f.sgn = fine_ev ? p.sgn : f.sgn;
        f.bad = fine_ev ? p.bad : f.bad;
        g.x = fine_ev ? g.x : p.x;
        g.u = fine_ev ? g.u : p.u;
        g.sgn = fine_ev ? g.sgn : p.sgn;
        g.bad = fine_ev ? g.bad : p.bad;
        kf.su = fine_ev ? kn.su : kf.su;
        kf.lam = fine_ev ? kn.lam : kf.lam;
        kf.a = fine_ev ? kn.a : kf.a;
        kf.b = fine_ev ? kn.b : kf.b;
        kg.su = fine_ev ? kg.su : kn.su;
        kg.lam = fine_ev ? kg.lam : kn.lam;
        kg.a = fine_ev ? kg.a : kn.a;
        kg.b = fine_ev ? kg.b : kn.b;
        tf = fine_ev ? e : tf;
        ef = fine_ev ? en : ef;
        wf = fine_ev ? (R)0 : wf;
        tc = fine_ev ? tc : e;
        ec = fine_ev ? ec : en;
        wc = fine_ev ? wc : (R)0;
    }
}

// The wave's share of an adaptive item: a chunk of 64 spl samples per wave, in block and
// wave order. WIDE: 64-bit tick counters (else T in ticks plus the longest step, 2^21
// ticks, fits 32 bits: the host picks the kernel).
template <typename R, int PROF, bool WIDE>
__device__ __forceinline__ void adaptive_samples(const KProblem& kp, const Consts<R>& c, const KItem& item,
                                                 uint32_t local_block, Acc& acc, double* dump) {
    const uint64_t chunk = 64ull * item.spl;
    const uint64_t wave = (uint64_t)local_block * (kBlock / 64) + (threadIdx.x >> 6);
    const uint64_t c_begin = wave * chunk;
    if (c_begin >= item.n_samples) return;
    const uint64_t c_end = (c_begin + chunk < item.n_samples) ? c_begin + chunk : item.n_samples;
    if constexpr (WIDE)
        adaptive_lane<R, PROF, uint64_t>(kp, c, item, c_begin, c_end, acc, dump);
    else
        adaptive_lane<R, PROF, uint32_t>(kp, c, item, c_begin, c_end, acc, dump);
}

// The work of one block: block `local_block` of `item`, in the item's mode. acc receives
// this block's sums (valid in thread 0 after block_reduce).
template <typename R, int INTEG, int PROF>
__device__ __forceinline__ void run_block(const KProblem& kp, const KItem& item,
                                          uint32_t local_block, Acc& acc, double* dump,
                                          PipeLds<R>& lds) {
    const Consts<R> c = make_consts<R>(kp);
    if constexpr (INTEG == KINTEG_SE_ADAPT || INTEG == KINTEG_SE_ADAPT_WIDE) {   // STREAM layout only
        adaptive_samples<R, PROF, INTEG == KINTEG_SE_ADAPT_WIDE>(kp, c, item, local_block, acc, dump);
    } else if (item.mode == KMODE_PIPE) {
        pipe_samples<R, INTEG, PROF>(kp, c, item, local_block, acc, dump, lds);
    } else {
        const uint64_t base = (uint64_t)local_block * (uint64_t)kBlock * item.spl;
        for (uint32_t k = 0; k < item.spl; ++k) {
            const uint64_t local = base + (uint64_t)k * kBlock + threadIdx.x;
            if (local < item.n_samples) {
                double pf, pc;
                bool bad;
                sample_qoi<R, INTEG, PROF>(kp, c, item.level, item.sample_begin + local, pf, pc, bad);
                if (dump != nullptr) {
                    dump[2 * local] = pf;
                    dump[2 * local + 1] = pc;
                }
                accumulate(acc, pf, pc, bad);
            }
        }
    }
}

// One kernel per (path precision, integrator, profile): all items of a launch share the
// problem, so the choice is made on the host and each kernel holds two path bodies only.
// At least 3 waves per SIMD (HIP's second bound): the FP64 bodies fit 168 registers
// without spilling; the FP32 bodies use far fewer.
template <typename R, int INTEG, int PROF>
__global__ __launch_bounds__(kBlock, 3) void level_kernel(const KArgs args,
                                                       ld_level_sums* __restrict__ partials,
                                                       double* __restrict__ dump) {
    const uint32_t b = blockIdx.x;
    int it = 0;
    while (it + 1 < args.n_items && b >= args.items[it].block_begin + args.items[it].n_blocks) ++it;
    const KItem item = args.items[it];
    set_priority(item.prio);
    Acc acc;
    acc_zero(acc);
    // the PIPE blocks' hand-off area. FP32: dynamic, a launch brings sizeof(PipeLds<float>)
    // bytes only if one of its items runs PIPE blocks (launch_levels), so that STREAM-only
    // launches keep the occupancy their registers allow (6 blocks per CU rather than the 4
    // that 34 KB allow). FP64: static (its blocks fit 3 per CU by registers anyway; the
    // dynamic form made the FP64 estimate 3 % slower)
    if constexpr (sizeof(R) == 4) {
        extern __shared__ __align__(16) unsigned char pipe_lds[];
        run_block<R, INTEG, PROF>(args.prob, item, b - item.block_begin, acc, dump,
                                  *reinterpret_cast<PipeLds<R>*>(pipe_lds));
    } else {
        __shared__ PipeLds<R> lds;
        run_block<R, INTEG, PROF>(args.prob, item, b - item.block_begin, acc, dump, lds);
    }
    block_reduce(acc);
    if (threadIdx.x == 0) store_sums(&partials[b], acc);
}

// ---------------------------------------------------------------------------------
// Persistent multi-estimator kernel. Blocks take tiles (one block's work of one
// (query, level, range)) from a queue until it is empty; each tile writes its own
// partial, so the result does not depend on which block ran which tile. Integrators
// are chosen per tile (uniform per block); the profile is a template parameter.
// ADAPT: the queue of adaptive symplectic Euler tiles (neutral profile), each run as the
// level kernel runs that block, with 32- or 64-bit tick counters as its level needs.
// ---------------------------------------------------------------------------------
// One tile of a queue: its block of samples in the tile's mode, the block's sums written
// to the tile's partial. Both engine kernels below run tiles with this code, so a tile's
// partial does not depend on which of them ran it.
template <typename R, int PROF, bool ADAPT>
__device__ __forceinline__ void run_tile(const KQueue& q, uint32_t t, const KTile* __restrict__ tiles,
                                         const KProblem* __restrict__ problems,
                                         ld_level_sums* __restrict__ partials, PipeLds<R>& lds) {
    const KTile tile = tiles[q.first + t];
    const KProblem& kp = problems[tile.slot];
    KItem item;
    item.level = tile.level;
    item.spl = tile.spl;
    item.block_begin = 0;
    item.n_blocks = 0;
    item.sample_begin = tile.sample_begin;
    item.n_samples = tile.n_samples;
    item.out_slot = 0;
    item.mode = tile.mode;
    item.prio = tile.prio;
    set_priority(tile.prio);
    Acc acc;
    acc_zero(acc);
    if constexpr (ADAPT) {
        if (((uint64_t)kp.M0 << (tile.level + kAdaptTickBits)) + ((uint64_t)2 << kAdaptTickBits) <
            ((uint64_t)1 << 32))
            run_block<R, KINTEG_SE_ADAPT, PROF>(kp, item, tile.local_block, acc, nullptr, lds);
        else
            run_block<R, KINTEG_SE_ADAPT_WIDE, PROF>(kp, item, tile.local_block, acc, nullptr, lds);
    } else {
        switch (kp.integ) {
            case KINTEG_SE: run_block<R, KINTEG_SE, PROF>(kp, item, tile.local_block, acc, nullptr, lds); break;
            case KINTEG_GL: run_block<R, KINTEG_GL, PROF>(kp, item, tile.local_block, acc, nullptr, lds); break;
            default: run_block<R, KINTEG_BAOAB, PROF>(kp, item, tile.local_block, acc, nullptr, lds); break;
        }
    }
    block_reduce_all(acc);
    if (wave_index() == 0) store_sums(&partials[q.first + t], acc);   // same values from every lane
}

// Persistent form (a fixed grid, as a captured graph needs): blocks take tiles from the
// queue's counter until it is empty.
template <typename R, int PROF, bool ADAPT = false>
__global__ __launch_bounds__(kBlock) void persistent_kernel(const KHeader* __restrict__ hdr,
                                                            const KTile* __restrict__ tiles,
                                                            const KProblem* __restrict__ problems,
                                                            ld_level_sums* __restrict__ partials,
                                                            uint32_t* __restrict__ counters) {
    __shared__ uint32_t sh_tile;
    __shared__ PipeLds<R> lds;
    const KQueue q = hdr->queue[ADAPT ? (int)KQUEUE_ADAPT : PROF];
    const uint32_t wave = wave_index();
    const uint32_t lane = threadIdx.x & 63u;
    // The loop boundary holds no single-lane region (a divergent region there can be
    // turned into a loop exit for that lane alone, re-running the body for the other
    // lanes without fetching a new tile): wave 0 fetches the tile under a scalar
    // branch, every lane issuing the atomic with only lane 0 adding 1.
    for (;;) {
        if (wave == 0) {
            const uint32_t old = atomicAdd(&counters[q.counter], lane == 0 ? 1u : 0u);
            sh_tile = __builtin_amdgcn_readfirstlane(old);
        }
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(sh_tile);
        __syncthreads();
        if (t >= q.n_tiles) break;
        run_tile<R, PROF, ADAPT>(q, t, tiles, problems, partials, lds);
    }
}

// One block per tile (a grid of exactly the queue's tile count): blocks start in tile
// order, so the longest paths, first in the table, start first. At least three waves per
// SIMD, as for the level kernels (the FP64 body then fits 168 VGPRs without spilling).
template <typename R, int PROF, bool ADAPT = false>
__global__ __launch_bounds__(kBlock, 3) void tile_kernel(const KHeader* __restrict__ hdr,
                                                      const KTile* __restrict__ tiles,
                                                      const KProblem* __restrict__ problems,
                                                      ld_level_sums* __restrict__ partials) {
    __shared__ PipeLds<R> lds;
    const KQueue q = hdr->queue[ADAPT ? (int)KQUEUE_ADAPT : PROF];
    const uint32_t t = blockIdx.x;
    if (t >= q.n_tiles) return;
    run_tile<R, PROF, ADAPT>(q, t, tiles, problems, partials, lds);
}

// The tile table of an iteration from its ranges: tile b of a range is block b of it.
__global__ __launch_bounds__(kBlock) void expand_tiles_kernel(const KHeader* __restrict__ hdr,
                                                              const KRange* __restrict__ ranges,
                                                              KTile* __restrict__ tiles) {
    const uint32_t n_ranges = hdr->n_ranges;
    for (uint32_t r = blockIdx.x; r < n_ranges; r += gridDim.x) {
        const KRange rg = ranges[r];
        KTile t;
        t.slot = rg.slot;
        t.level = rg.level;
        t.sample_begin = rg.sample_begin;
        t.n_samples = rg.n_samples;
        t.spl = rg.spl;
        t.mode = rg.mode;
        t.prio = rg.prio;
        t.pad = 0;
        for (uint32_t b = threadIdx.x; b < rg.n_tiles; b += kBlock) {
            t.local_block = b;
            tiles[rg.tile_begin + b] = t;
        }
    }
}

// expand_tiles_kernel for a small iteration whose tables come as the argument: block 0
// stores the header, the ranges and the new problems for the kernels that follow (stream
// order), and every block writes its ranges' tiles from the argument.
__global__ __launch_bounds__(kBlock) void expand_inline_kernel(const KInline in, KHeader* __restrict__ hdr,
                                                               KRange* __restrict__ ranges,
                                                               KProblem* __restrict__ problems,
                                                               KTile* __restrict__ tiles) {
    const uint32_t n_ranges = in.hdr.n_ranges;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) *hdr = in.hdr;
        for (uint32_t r = threadIdx.x; r < n_ranges; r += kBlock) ranges[r] = in.ranges[r];
        for (uint32_t j = threadIdx.x; j < in.n_new; j += kBlock) problems[in.new_lo + j] = in.problems[j];
    }
    for (uint32_t r = blockIdx.x; r < n_ranges; r += gridDim.x) {
        const KRange& rg = in.ranges[r];
        KTile t;
        t.slot = rg.slot;
        t.level = rg.level;
        t.sample_begin = rg.sample_begin;
        t.n_samples = rg.n_samples;
        t.spl = rg.spl;
        t.mode = rg.mode;
        t.prio = rg.prio;
        t.pad = 0;
        for (uint32_t b = threadIdx.x; b < rg.n_tiles; b += kBlock) {
            t.local_block = b;
            tiles[rg.tile_begin + b] = t;
        }
    }
}

__global__ void reset_counters_kernel(uint32_t* counters, int n) {
    if ((int)threadIdx.x < n) counters[threadIdx.x] = 0u;
}

// Each range's tile partials, in tile order, are reduced and added to the running sums
// of (query slot, level); also written per range for the caller. The persistent kernels
// of the iteration have ended (stream order), so block 0 also sets the queue counters
// back to zero for the next iteration.
__global__ __launch_bounds__(kBlock) void merge_ranges_kernel(const KHeader* __restrict__ hdr,
                                                              const KRange* __restrict__ ranges,
                                                              const ld_level_sums* __restrict__ partials,
                                                              ld_level_sums* __restrict__ running,
                                                              ld_level_sums* __restrict__ range_out,
                                                              uint32_t* __restrict__ counters,
                                                              ld_level_sums* __restrict__ host_running) {
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)kNumQueues) counters[threadIdx.x] = 0u;
    const uint32_t n_ranges = hdr->n_ranges;
    for (uint32_t r = blockIdx.x; r < n_ranges; r += gridDim.x) {
        const KRange rg = ranges[r];
        Acc acc;
        acc_zero(acc);
        for (uint32_t j = threadIdx.x; j < rg.n_tiles; j += kBlock) {
            const ld_level_sums p = partials[rg.tile_begin + j];
#pragma unroll
            for (int k = 0; k < 4; ++k) neumaier_merge(acc.s[k], acc.c[k], p.s[k], p.c[k]);
            acc.n += p.n;
            acc.nbad += p.n_nonfinite;
        }
        block_reduce_all(acc);
        if (wave_index() == 0) {   // scalar branch; every lane computes and stores the same values
            store_sums(&range_out[r], acc);
            ld_level_sums* run = &running[rg.slot * LD_MAX_LEVELS + rg.level];
            // a fresh level adds to zeros: the same arithmetic as after clearing it
            Acc tot;
            if (rg.fresh) {
                acc_zero(tot);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    tot.s[k] = run->s[k];
                    tot.c[k] = run->c[k];
                }
                tot.n = run->n;
                tot.nbad = run->n_nonfinite;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) neumaier_merge(tot.s[k], tot.c[k], acc.s[k], acc.c[k]);
            tot.n += acc.n;
            tot.nbad += acc.nbad;
            store_sums(run, tot);
            // the same row into the host's pinned copy (one lane: a posted write over the
            // bus), which the host reads after the stream synchronises
            if (host_running != nullptr && (threadIdx.x & 63) == 0)
                store_sums(&host_running[rg.slot * LD_MAX_LEVELS + rg.level], tot);
        }
    }
}

__global__ void clear_sums_kernel(ld_level_sums* sums, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        ld_level_sums z;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            z.s[k] = 0.0;
            z.c[k] = 0.0;
        }
        z.n = 0;
        z.n_nonfinite = 0;
        sums[i] = z;
    }
}

__global__ __launch_bounds__(kBlock) void merge_kernel(const KArgs args,
                                                       const ld_level_sums* __restrict__ partials,
                                                       ld_level_sums* __restrict__ out) {
    const KItem item = args.items[blockIdx.x];
    Acc acc;
    acc_zero(acc);
    for (uint32_t j = threadIdx.x; j < item.n_blocks; j += kBlock) {
        const ld_level_sums p = partials[item.block_begin + j];
#pragma unroll
        for (int k = 0; k < 4; ++k) neumaier_merge(acc.s[k], acc.c[k], p.s[k], p.c[k]);
        acc.n += p.n;
        acc.nbad += p.n_nonfinite;
    }
    block_reduce(acc);
    if (threadIdx.x == 0) store_sums(&out[item.out_slot], acc);
}

// ---------------------------------------------------------------------------------
// Binned concentration (vector QoI of Sec. 6.4). The path kernels dump the terminal
// positions (X_f, X_c) of a range (NaN for a path that ran away); pdf_bins_kernel then
// forms, per bin, compensated sums of Y_i = P_i(X_f) - P_i(X_c), Y_i^2, P_i(X_f) and
// its square, with P_i the box of Eq. (34) or its smoothing by Eq. (37). A wave holds
// floor(64 / n_bins) samples side by side, one lane per (sample, bin); each block takes
// kPdfChunk consecutive samples and reduces its sample streams per bin in a fixed
// order, and pdf_merge_kernel folds the blocks of each bin in a fixed tree.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ double box_qoi(const KProblem& kp, double x, double a, double b) {
    if (kp.r == 0) return (x <= b ? 1.0 : 0.0) - (x <= a ? 1.0 : 0.0);
    return g_r(kp, (x - b) * kp.inv_delta) - g_r(kp, (x - a) * kp.inv_delta);
}

__global__ __launch_bounds__(kBlock) void pdf_bins_kernel(const KBins bins, const KProblem kp,
                                                          const double* __restrict__ dump,
                                                          ld_level_sums* __restrict__ partials) {
    const int k = bins.n_bins;
    const int spw = 64 / k;                              // sample streams per wave
    const int lane = threadIdx.x & 63, wave = (int)wave_index();
    const int sub = lane / k, bin = lane - sub * k;
    const bool on = sub < spw;
    const int streams = (kBlock / 64) * spw;
    const int stream = wave * spw + sub;
    const uint64_t lo = (uint64_t)blockIdx.x * kPdfChunk;
    const uint64_t hi = lo + kPdfChunk < bins.n ? lo + kPdfChunk : bins.n;
    const double a = bins.a0 + (double)bin * bins.width;
    const double b = bins.a0 + (double)(bin + 1) * bins.width;
    Acc acc;
    acc_zero(acc);
    if (on) {
        for (uint64_t j = lo + (uint64_t)stream; j < hi; j += (uint64_t)streams) {
            const double xf = dump[2 * j], xc = dump[2 * j + 1];
            const bool bad = !isfinite(xf) || (bins.level != 0 && !isfinite(xc));
            const double pf = box_qoi(kp, xf, a, b);
            const double pc = (bins.level == 0) ? 0.0 : box_qoi(kp, xc, a, b);
            accumulate(acc, pf, pc, bad);
        }
    }
    __shared__ Acc sh[kBlock];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < (unsigned)k) {
        Acc t;
        acc_zero(t);
        for (int st = 0; st < streams; ++st) {               // fixed order of the streams
            const Acc& o = sh[(st / spw) * 64 + (st % spw) * k + (int)threadIdx.x];
#pragma unroll
            for (int q = 0; q < 4; ++q) neumaier_merge(t.s[q], t.c[q], o.s[q], o.c[q]);
            t.n += o.n;
            t.nbad += o.nbad;
        }
        store_sums(&partials[(uint64_t)blockIdx.x * k + threadIdx.x], t);
    }
}

// One block per bin: the block partials of that bin, strided over the threads and
// reduced in the fixed tree of block_reduce.
__global__ __launch_bounds__(kBlock) void pdf_merge_kernel(const ld_level_sums* __restrict__ partials,
                                                           uint32_t n_blocks, int32_t n_bins,
                                                           ld_level_sums* __restrict__ out) {
    const int bin = blockIdx.x;
    Acc acc;
    acc_zero(acc);
    for (uint32_t j = threadIdx.x; j < n_blocks; j += kBlock) {
        const ld_level_sums p = partials[(uint64_t)j * n_bins + bin];
#pragma unroll
        for (int q = 0; q < 4; ++q) neumaier_merge(acc.s[q], acc.c[q], p.s[q], p.c[q]);
        acc.n += p.n;
        acc.nbad += p.n_nonfinite;
    }
    block_reduce(acc);
    if (threadIdx.x == 0) store_sums(&out[bin], acc);
}

int launch_pdf_bins(const KBins& bins, const KProblem& kp, const double* d_dump,
                    ld_level_sums* d_partials, ld_level_sums* d_out, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const uint32_t nb = pdf_blocks(bins.n);
    if (nb > 0) {
        hipLaunchKernelGGL(pdf_bins_kernel, dim3(nb), dim3(kBlock), 0, s, bins, kp, d_dump, d_partials);
        if (hipGetLastError() != hipSuccess) return LD_EDEVICE;
    }
    hipLaunchKernelGGL(pdf_merge_kernel, dim3(bins.n_bins), dim3(kBlock), 0, s, d_partials, nb, bins.n_bins,
                       d_out);
    return hipGetLastError() == hipSuccess ? LD_OK : LD_EDEVICE;
}

// Partials of mlmc_level_sums_noalloc. In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the address that scratch_partials looks up.
static __device__ __align__(256) ld_level_sums scratch[kScratchPartials];

constexpr int kMaxDevices = 64;

int scratch_partials(ld_level_sums** out) {
    static std::mutex mu;
    static ld_level_sums* addr[kMaxDevices] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return LD_ENODEVICE;
    if (dev >= kMaxDevices) return LD_EDEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return LD_EDEVICE;
        addr[dev] = (ld_level_sums*)p;
    }
    *out = addr[dev];
    return LD_OK;
}

using LevelKernel = void (*)(const KArgs, ld_level_sums*, double*);

template <typename R>
LevelKernel pick_kernel(int integ, int profile, bool adaptive, bool wide) {
    if (adaptive)   // neutral profile only
        return wide ? level_kernel<R, KINTEG_SE_ADAPT_WIDE, KPROFILE_NEUTRAL> : level_kernel<R, KINTEG_SE_ADAPT, KPROFILE_NEUTRAL>;
    switch (integ * 2 + profile) {
        case KINTEG_SE * 2 + KPROFILE_HOMOGENEOUS: return level_kernel<R, KINTEG_SE, KPROFILE_HOMOGENEOUS>;
        case KINTEG_SE * 2 + KPROFILE_NEUTRAL: return level_kernel<R, KINTEG_SE, KPROFILE_NEUTRAL>;
        case KINTEG_GL * 2 + KPROFILE_HOMOGENEOUS: return level_kernel<R, KINTEG_GL, KPROFILE_HOMOGENEOUS>;
        case KINTEG_GL * 2 + KPROFILE_NEUTRAL: return level_kernel<R, KINTEG_GL, KPROFILE_NEUTRAL>;
        case KINTEG_BAOAB * 2 + KPROFILE_HOMOGENEOUS: return level_kernel<R, KINTEG_BAOAB, KPROFILE_HOMOGENEOUS>;
        default: return level_kernel<R, KINTEG_BAOAB, KPROFILE_NEUTRAL>;
    }
}

int launch_levels(const KArgs& args, uint32_t total_blocks, ld_level_sums* d_partials,
                  ld_level_sums* d_out, double* d_dump, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (total_blocks > 0) {
        // adaptive steps: 64-bit tick counters if some item's T in ticks plus a coarse step
        // (2^21 ticks) does not fit 32 bits
        bool wide = false;
        for (int i = 0; i < args.n_items; ++i)
            wide |= (((uint64_t)args.prob.M0 << (args.items[i].level + kAdaptTickBits)) +
                     ((uint64_t)2 << kAdaptTickBits)) >= ((uint64_t)1 << 32);
        const LevelKernel k = (args.precision == LD_FP32)
                                  ? pick_kernel<float>(args.prob.integ, args.prob.profile, args.prob.adaptive, wide)
                                  : pick_kernel<double>(args.prob.integ, args.prob.profile, args.prob.adaptive, wide);
        bool pipe = false;
        for (int i = 0; i < args.n_items; ++i) pipe |= args.items[i].mode == KMODE_PIPE;
        const size_t lds = (pipe && args.precision == LD_FP32) ? sizeof(PipeLds<float>) : 0;
        hipLaunchKernelGGL(k, dim3(total_blocks), dim3(kBlock), lds, s, args, d_partials, d_dump);
        if (hipGetLastError() != hipSuccess) return LD_EDEVICE;
    }
    hipLaunchKernelGGL(merge_kernel, dim3(args.n_items), dim3(kBlock), 0, s, args, d_partials, d_out);
    if (hipGetLastError() != hipSuccess) return LD_EDEVICE;
    return LD_OK;
}

template <typename R, int PROF, bool ADAPT>
void launch_queue(bool persistent, uint32_t grid, hipStream_t s, const KHeader* d_hdr, const KTile* d_tiles,
                  const KProblem* d_problems, ld_level_sums* d_partials, uint32_t* d_counters) {
    if (persistent)
        hipLaunchKernelGGL((persistent_kernel<R, PROF, ADAPT>), dim3(grid), dim3(kBlock), 0, s, d_hdr, d_tiles,
                           d_problems, d_partials, d_counters);
    else
        hipLaunchKernelGGL((tile_kernel<R, PROF, ADAPT>), dim3(grid), dim3(kBlock), 0, s, d_hdr, d_tiles,
                           d_problems, d_partials);
}

template <typename R>
void launch_queues(bool persistent, const uint32_t* grid, uint32_t mask, hipStream_t s, const KHeader* d_hdr,
                   const KTile* d_tiles, const KProblem* d_problems, ld_level_sums* d_partials,
                   uint32_t* d_counters) {
    if ((mask >> KPROFILE_NEUTRAL) & 1u)
        launch_queue<R, KPROFILE_NEUTRAL, false>(persistent, grid[KPROFILE_NEUTRAL], s, d_hdr, d_tiles, d_problems,
                                                 d_partials, d_counters);
    if ((mask >> KPROFILE_HOMOGENEOUS) & 1u)
        launch_queue<R, KPROFILE_HOMOGENEOUS, false>(persistent, grid[KPROFILE_HOMOGENEOUS], s, d_hdr, d_tiles,
                                                     d_problems, d_partials, d_counters);
    if ((mask >> KQUEUE_ADAPT) & 1u)
        launch_queue<R, KPROFILE_NEUTRAL, true>(persistent, grid[KQUEUE_ADAPT], s, d_hdr, d_tiles, d_problems,
                                                d_partials, d_counters);
}

int launch_engine_iteration(int precision, bool persistent, const uint32_t* grid_blocks, uint32_t queue_mask,
                            const KHeader* d_hdr, const KTile* d_tiles, const KProblem* d_problems,
                            ld_level_sums* d_partials, uint32_t* d_counters,
                            const KRange* d_ranges, ld_level_sums* d_running,
                            ld_level_sums* d_range_out, ld_level_sums* h_running, void* stream,
                            const KInline* inl) {
    hipStream_t s = (hipStream_t)stream;
    if (inl != nullptr)
        hipLaunchKernelGGL(expand_inline_kernel, dim3(inl->hdr.n_ranges > 0 ? inl->hdr.n_ranges : 1u), dim3(kBlock),
                           0, s, *inl, const_cast<KHeader*>(d_hdr), const_cast<KRange*>(d_ranges),
                           const_cast<KProblem*>(d_problems), const_cast<KTile*>(d_tiles));
    else
        hipLaunchKernelGGL(expand_tiles_kernel, dim3(kMergeGrid), dim3(kBlock), 0, s, d_hdr, d_ranges,
                           (KTile*)d_tiles);
    if (precision == LD_FP32)
        launch_queues<float>(persistent, grid_blocks, queue_mask, s, d_hdr, d_tiles, d_problems, d_partials,
                             d_counters);
    else
        launch_queues<double>(persistent, grid_blocks, queue_mask, s, d_hdr, d_tiles, d_problems, d_partials,
                              d_counters);
    hipLaunchKernelGGL(merge_ranges_kernel, dim3(kMergeGrid), dim3(kBlock), 0, s, d_hdr, d_ranges, d_partials,
                       d_running, d_range_out, d_counters, h_running);
    return hipGetLastError() == hipSuccess ? LD_OK : LD_EDEVICE;
}

int launch_reset_counters(uint32_t* d_counters, void* stream) {
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, d_counters, (int)kNumQueues);
    return hipGetLastError() == hipSuccess ? LD_OK : LD_EDEVICE;
}

int launch_clear_sums(ld_level_sums* d_sums, uint32_t n, void* stream) {
    if (n == 0) return LD_OK;
    hipLaunchKernelGGL(clear_sums_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_sums, n);
    return hipGetLastError() == hipSuccess ? LD_OK : LD_EDEVICE;
}

}  // namespace ldm
