// kernels.hip -- level-sum kernels for gfx950.
//
// level_kernel: one coupled sample per lane at a time (each lane runs `spl` samples of
// its block's range), the fine and coarse paths entirely in registers; no input
// arrays. Each lane keeps Neumaier (compensated) FP64 sums of Y_l, Y_l^2, P_l, P_l^2
// (Eq. 16); a wave combines them with xor-shuffles, the four waves of a block through
// LDS, and the block writes one 80-byte partial. merge_kernel then combines each
// item's partials in a fixed order. No atomics: results are bitwise reproducible.
#include <hip/hip_runtime.h>

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
// normals of alternate coarse steps of a chunk, wave 2 advances the fine paths over
// the chunk before and passes (S xi_2m, S xi_2m+1, e^{-lambda h}) on, wave 3 advances
// the coarse paths over the chunk before that. Double-buffered LDS, one barrier per
// chunk of kPipeChunk coarse steps; the arithmetic per path is that of STREAM mode.
template <typename R>
struct PipeLds {
    R nrm[2][kPipeChunk][2][64];   // normals of a chunk, double-buffered
    R msg[2][kPipeChunk][3][64];   // fine -> coarse: S xi_2m, S xi_2m+1, e^{-lambda h}
    double end_pc[64];
    int end_bad[64];
};

template <typename R, int INTEG, int PROF>
__device__ __forceinline__ void pipe_samples(const KProblem& kp, const Consts<R>& c,
                                             const KItem& item, uint32_t local_block, Acc& acc,
                                             double* dump, PipeLds<R>& L) {
    constexpr int K = kPipeChunk;
    auto& nrm = L.nrm;
    auto& msg = L.msg;
    auto& end_pc = L.end_pc;
    auto& end_bad = L.end_bad;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t local = (uint64_t)local_block * 64 + lane;
    const bool active = local < item.n_samples;
    const int level = item.level;
    const uint32_t M = (uint32_t)kp.M0 << level;
    const uint32_t P = M / 2;
    const uint32_t nch = (P + K - 1) / K;
    const double hd = kp.T / (double)M;
    const R h = (R)hd, hh = (R)(0.5 * hd), h2 = (R)(2.0 * hd);
    const Stream st = make_stream(kp.seed, kp.stream_id, level, item.sample_begin + local);
    Path<R> p;
    if (wave >= 2) {
        R x0, u0;
        initial_state<R, PROF>(kp, c, st, x0, u0);
        init_path<R, INTEG, PROF>(c, p, x0, u0);
    }
    for (uint32_t s = 0; s < nch + 2; ++s) {
        if (wave < 2) {
            if (s < nch) {
                const uint32_t b = s & 1;
#pragma unroll
                for (int j = 0; j < K; j += 2) {
                    const uint32_t m = s * K + j + wave;
                    if (m < P) {
                        R z0, z1;
                        Normals<R>::pair(philox(st, m), z0, z1);
                        nrm[b][j + wave][0][lane] = z0;
                        nrm[b][j + wave][1][lane] = z1;
                    }
                }
            }
        } else if (wave == 2) {
            if (s >= 1 && s <= nch) {
                const uint32_t b = (s - 1) & 1;
                for (int j = 0; j < K; ++j) {
                    const uint32_t m = (s - 1) * K + j;
                    if (m < P) {
                        R ta, tb, wa, wb;
                        step<R, INTEG, PROF, false>(c, p, h, hh, nrm[b][j][0][lane], ta, wa);
                        step<R, INTEG, PROF, false>(c, p, h, hh, nrm[b][j][1][lane], tb, wb);
                        msg[b][j][0][lane] = ta;
                        msg[b][j][1][lane] = tb;
                        msg[b][j][2][lane] = wa;
                    }
                }
            }
        } else {
            if (s >= 2) {
                const uint32_t b = s & 1;   // == (s - 2) & 1
                for (int j = 0; j < K; ++j) {
                    const uint32_t m = (s - 2) * K + j;
                    if (m < P) {
                        const R ta = msg[b][j][0][lane], tb = msg[b][j][1][lane];
                        R xi_c;
                        if (INTEG == KINTEG_SE) {
                            xi_c = (ta + tb) * (R)0.70710678118654752440;             // Eq. (18)
                        } else {
                            const R wa = msg[b][j][2][lane];
                            xi_c = (wa * ta + tb) * Math<R>::rsqrt(wa * wa + (R)1);  // Eq. (19)
                        }
                        R unused_t, unused_w;
                        step<R, INTEG, PROF, true>(c, p, h2, h, xi_c, unused_t, unused_w);
                    }
                }
            }
        }
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
__device__ __forceinline__ void set_priority(uint32_t prio) {
    switch (prio) {
        case 3: __builtin_amdgcn_s_setprio(3); break;
        case 2: __builtin_amdgcn_s_setprio(2); break;
        case 1: __builtin_amdgcn_s_setprio(1); break;
        default: break;
    }
}

// One kernel per (path precision, integrator, profile): all items of a launch share the
// problem, so the choice is made on the host and each kernel holds two path bodies only.
template <typename R, int INTEG, int PROF>
__global__ __launch_bounds__(kBlock) void level_kernel(const KArgs args,
                                                       ld_level_sums* __restrict__ partials,
                                                       double* __restrict__ dump) {
    const uint32_t b = blockIdx.x;
    int it = 0;
    while (it + 1 < args.n_items && b >= args.items[it].block_begin + args.items[it].n_blocks) ++it;
    const KItem item = args.items[it];
    const KProblem& kp = args.prob;
    const Consts<R> c = make_consts<R>(kp);
    set_priority(item.prio);
    Acc acc;
    acc_zero(acc);
    if (item.mode == KMODE_PIPE) {
        __shared__ PipeLds<R> lds;
        pipe_samples<R, INTEG, PROF>(kp, c, item, b - item.block_begin, acc, dump, lds);
    } else {
        const uint64_t base = (uint64_t)(b - item.block_begin) * (uint64_t)kBlock * item.spl;
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
    block_reduce(acc);
    if (threadIdx.x == 0) store_sums(&partials[b], acc);
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

using LevelKernel = void (*)(const KArgs, ld_level_sums*, double*);

template <typename R>
LevelKernel pick_kernel(int integ, int profile) {
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
        const LevelKernel k = (args.precision == LD_FP32)
                                  ? pick_kernel<float>(args.prob.integ, args.prob.profile)
                                  : pick_kernel<double>(args.prob.integ, args.prob.profile);
        hipLaunchKernelGGL(k, dim3(total_blocks), dim3(kBlock), 0, s, args, d_partials, d_dump);
        if (hipGetLastError() != hipSuccess) return LD_EDEVICE;
    }
    hipLaunchKernelGGL(merge_kernel, dim3(args.n_items), dim3(kBlock), 0, s, args, d_partials, d_out);
    if (hipGetLastError() != hipSuccess) return LD_EDEVICE;
    return LD_OK;
}

}  // namespace ldm
