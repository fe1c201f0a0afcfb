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

template <typename R>
__device__ __forceinline__ void dispatch(const KProblem& kp, const Consts<R>& c, int level,
                                         uint64_t sample, double& pf, double& pc, bool& bad) {
    switch (kp.integ * 2 + kp.profile) {
        case KINTEG_SE * 2 + KPROFILE_HOMOGENEOUS:
            sample_qoi<R, KINTEG_SE, KPROFILE_HOMOGENEOUS>(kp, c, level, sample, pf, pc, bad); break;
        case KINTEG_SE * 2 + KPROFILE_NEUTRAL:
            sample_qoi<R, KINTEG_SE, KPROFILE_NEUTRAL>(kp, c, level, sample, pf, pc, bad); break;
        case KINTEG_GL * 2 + KPROFILE_HOMOGENEOUS:
            sample_qoi<R, KINTEG_GL, KPROFILE_HOMOGENEOUS>(kp, c, level, sample, pf, pc, bad); break;
        case KINTEG_GL * 2 + KPROFILE_NEUTRAL:
            sample_qoi<R, KINTEG_GL, KPROFILE_NEUTRAL>(kp, c, level, sample, pf, pc, bad); break;
        case KINTEG_BAOAB * 2 + KPROFILE_HOMOGENEOUS:
            sample_qoi<R, KINTEG_BAOAB, KPROFILE_HOMOGENEOUS>(kp, c, level, sample, pf, pc, bad); break;
        default:
            sample_qoi<R, KINTEG_BAOAB, KPROFILE_NEUTRAL>(kp, c, level, sample, pf, pc, bad); break;
    }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void level_kernel(const KArgs args,
                                                       ld_level_sums* __restrict__ partials,
                                                       double* __restrict__ dump) {
    const uint32_t b = blockIdx.x;
    int it = 0;
    while (it + 1 < args.n_items && b >= args.items[it].block_begin + args.items[it].n_blocks) ++it;
    const KItem item = args.items[it];
    const KProblem& kp = args.prob;
    const Consts<R> c = make_consts<R>(kp);
    Acc acc;
    acc_zero(acc);
    const uint64_t base = (uint64_t)(b - item.block_begin) * (uint64_t)kBlock * item.spl;
    for (uint32_t k = 0; k < item.spl; ++k) {
        const uint64_t local = base + (uint64_t)k * kBlock + threadIdx.x;
        if (local < item.n_samples) {
            double pf, pc;
            bool bad;
            dispatch<R>(kp, c, item.level, item.sample_begin + local, pf, pc, bad);
            if (dump != nullptr) {
                dump[2 * local] = pf;
                dump[2 * local + 1] = pc;
            }
            if (bad) {
                acc.nbad += 1;
            } else {
                const double y = pf - pc;
                neumaier_add(acc.s[0], acc.c[0], y);
                neumaier_add(acc.s[1], acc.c[1], y * y);
                neumaier_add(acc.s[2], acc.c[2], pf);
                neumaier_add(acc.s[3], acc.c[3], pf * pf);
                acc.n += 1;
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

int launch_levels(const KArgs& args, uint32_t total_blocks, ld_level_sums* d_partials,
                  ld_level_sums* d_out, double* d_dump, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (total_blocks > 0) {
        if (args.precision == LD_FP32)
            hipLaunchKernelGGL(level_kernel<float>, dim3(total_blocks), dim3(kBlock), 0, s, args,
                               d_partials, d_dump);
        else
            hipLaunchKernelGGL(level_kernel<double>, dim3(total_blocks), dim3(kBlock), 0, s, args,
                               d_partials, d_dump);
        if (hipGetLastError() != hipSuccess) return LD_EDEVICE;
    }
    hipLaunchKernelGGL(merge_kernel, dim3(args.n_items), dim3(kBlock), 0, s, args, d_partials, d_out);
    if (hipGetLastError() != hipSuccess) return LD_EDEVICE;
    return LD_OK;
}

}  // namespace ldm
