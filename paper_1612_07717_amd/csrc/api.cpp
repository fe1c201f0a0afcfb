// api.cpp -- validation, launch planning and the level-sum entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "host_common.hpp"

namespace ldm {

namespace {
thread_local std::string g_last_error;


bool finite(double v) { return std::isfinite(v); }
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

double sigma_u_at(const ld_profile& prof, double x) {
    if (prof.kind == LD_PROFILE_HOMOGENEOUS) return prof.sigma_u;
    const double xc = std::min(std::max(x, prof.eps_reg), prof.H - prof.eps_reg);
    return prof.kappa_sigma * prof.u_star * std::pow(1.0 - xc / prof.H, 0.75);
}

double lambda_max(const ld_profile& prof) {
    if (prof.kind == LD_PROFILE_HOMOGENEOUS) return 1.0 / prof.tau;
    // lambda = sigma_U / (kappa_tau X) decreases with X; its maximum is at the cut-off.
    return sigma_u_at(prof, prof.eps_reg) / (prof.kappa_tau * prof.eps_reg);
}

double lambda_at(const ld_profile& prof, double x) {
    if (prof.kind == LD_PROFILE_HOMOGENEOUS) return 1.0 / prof.tau;
    const double xc = std::min(std::max(x, prof.eps_reg), prof.H - prof.eps_reg);
    return sigma_u_at(prof, xc) / (prof.kappa_tau * xc);
}

int validate_problem(const ld_problem* p) {
    if (p == nullptr) return fail(LD_EINVAL, "problem is NULL");
    const ld_profile& f = p->profile;
    if (!(finite(f.H) && f.H >= 1e-6 && f.H <= 1e30)) return fail(LD_EINVAL, "profile.H must be in [1e-6, 1e30]");
    if (f.kind == LD_PROFILE_HOMOGENEOUS) {
        if (!(finite(f.sigma_u) && f.sigma_u > 0 && finite(f.tau) && f.tau > 0))
            return fail(LD_EINVAL, "homogeneous profile needs sigma_u > 0 and tau > 0");
    } else if (f.kind == LD_PROFILE_NEUTRAL_BL) {
        if (!(finite(f.kappa_sigma) && f.kappa_sigma > 0 && finite(f.kappa_tau) &&
              f.kappa_tau > 0 && finite(f.u_star) && f.u_star > 0))
            return fail(LD_EINVAL, "neutral profile needs kappa_sigma, kappa_tau, u_star > 0");
        // the cut-off band must be resolved by the FP32 path arithmetic: with eps_reg
        // below H's rounding, H - eps_reg would round to H and the drift coefficients at
        // X = H, which would count as inside, would divide by zero
        if (!(finite(f.eps_reg) && f.eps_reg >= 1e-6 * f.H && f.eps_reg < 0.5 * f.H))
            return fail(LD_EINVAL, "neutral profile needs 1e-6 H <= eps_reg < H/2");
    } else {
        return fail(LD_EINVAL, "unknown profile kind");
    }
    const ld_release& r = p->release;
    if (r.kind != LD_RELEASE_FIXED_W && r.kind != LD_RELEASE_GAUSSIAN_W &&
        r.kind != LD_RELEASE_WELL_MIXED)
        return fail(LD_EINVAL, "unknown release kind");
    if (r.kind != LD_RELEASE_WELL_MIXED && !(finite(r.z0) && r.z0 >= 0 && r.z0 <= f.H))
        return fail(LD_EINVAL, "release.z0 must lie in [0, H]");
    if (r.kind == LD_RELEASE_FIXED_W && !finite(r.w0))
        return fail(LD_EINVAL, "release.w0 must be finite");
    const ld_qoi& q = p->qoi;
    if (q.kind < LD_QOI_MEAN_Z || q.kind > LD_QOI_VELOCITY_SQ)
        return fail(LD_EINVAL, "unknown qoi kind");
    if (q.kind == LD_QOI_P_ABOVE || q.kind == LD_QOI_P_BOX) {
        if (q.r < 0 || q.r > 8) return fail(LD_EINVAL, "qoi.r must lie in 0..8");
        if (!(finite(q.a) && finite(q.b))) return fail(LD_EINVAL, "qoi.a, qoi.b must be finite");
        if (q.r > 0 && !(finite(q.delta) && q.delta > 0))
            return fail(LD_EINVAL, "qoi.delta must be positive");
    }
    if (!(finite(p->T) && p->T > 0)) return fail(LD_EINVAL, "T must be positive");
    if (p->M0 < 1) return fail(LD_EINVAL, "M0 must be >= 1");
    if (p->stream_id >= (1u << 24)) return fail(LD_EINVAL, "stream_id must be < 2^24");
    if (!(finite(p->x_adapt) && p->x_adapt >= 0.0 && p->x_adapt <= f.H))
        return fail(LD_EINVAL, "x_adapt must lie in [0, H] (0: uniform steps)");
    return LD_OK;
}

int check_stability(const ld_problem* p, ld_integrator integ, int32_t level) {
    if (p->x_adapt > 0.0 && integ != LD_SE)
        return fail(LD_EINVAL, "adaptive steps (x_adapt > 0) are defined for symplectic Euler only");
    if (p->x_adapt > 0.0 && lambda_max(p->profile) > 64.0 * lambda_at(p->profile, p->x_adapt))
        return fail(LD_EINVAL, "x_adapt too high: steps would shrink more than 64 times");
    if (integ != LD_SE) return LD_OK;
    // the longest step of the level: h_0 on level 0, the coarse step 2 h_l above it; with
    // adaptive steps lambda h never exceeds lambda(x_adapt) h (Sec. 7)
    const double M = std::ldexp((double)p->M0, level);
    const double h = (level == 0) ? p->T / M : 2.0 * p->T / M;
    const double lam = (p->x_adapt > 0.0) ? lambda_at(p->profile, p->x_adapt) : lambda_max(p->profile);
    if (lam * h >= 2.0)
        return fail(LD_EUNSTABLE, "symplectic Euler unstable: lambda * h >= 2 (use a larger M0 or adapt)");
    return LD_OK;
}

int make_kproblem(const ld_problem* p, ld_integrator integ, KProblem* kp) {
    std::memset(kp, 0, sizeof *kp);
    const ld_profile& f = p->profile;
    kp->H = f.H;
    kp->profile = (f.kind == LD_PROFILE_HOMOGENEOUS) ? KPROFILE_HOMOGENEOUS : KPROFILE_NEUTRAL;
    if (kp->profile == KPROFILE_NEUTRAL) {
        kp->eps_reg = f.eps_reg;
        kp->ks = f.kappa_sigma * f.u_star;
        kp->kappa_tau = f.kappa_tau;
        kp->sigma_u = 1.0;   // unused
        kp->tau = 1.0;       // unused
        kp->ksH = kp->ks * std::pow(f.H, -0.75);
        kp->kl = kp->ksH / f.kappa_tau;
    } else {
        kp->eps_reg = 0.0;
        kp->ks = 0.0;
        kp->kappa_tau = 1.0; // unused
        kp->sigma_u = f.sigma_u;
        kp->tau = f.tau;
    }
    kp->T = p->T;
    kp->z0 = p->release.z0;
    kp->w0 = p->release.w0;
    kp->su_z0 = sigma_u_at(f, p->release.z0);
    kp->lam_max = lambda_max(f);
    kp->release = p->release.kind;
    kp->qoi_kind = p->qoi.kind;
    kp->r = p->qoi.r;
    kp->qa = p->qoi.a;
    kp->qb = p->qoi.b;
    kp->inv_delta = (p->qoi.r > 0) ? 1.0 / p->qoi.delta : 0.0;
    kp->ncoef = 0;
    if ((p->qoi.kind == LD_QOI_P_ABOVE || p->qoi.kind == LD_QOI_P_BOX) && p->qoi.r > 0) {
        if (smoothing_coefficients(p->qoi.r, kp->coef) != 0)
            return fail(LD_EINVAL, "smoothing polynomial failed");
        kp->ncoef = p->qoi.r + 2;
    }
    kp->integ = (int32_t)integ;
    // In homogeneous turbulence lambda is the same everywhere, so no step ever shortens and
    // the adaptive scheme is the uniform one: it runs as such.
    kp->adaptive = (integ == LD_SE && p->x_adapt > 0.0 && kp->profile == KPROFILE_NEUTRAL) ? 1 : 0;
    kp->x_adapt = p->x_adapt;
    kp->M0 = p->M0;
    kp->stream_id = p->stream_id;
    kp->seed = p->seed;
    return LD_OK;
}

void plan_item(uint64_t n_samples, uint32_t* spl, uint32_t* n_blocks, uint64_t target_blocks) {
    const uint64_t per_block = (uint64_t)kBlock;
    uint64_t s = 1;
    if (n_samples > per_block * target_blocks)
        s = (n_samples + per_block * target_blocks - 1) / (per_block * target_blocks);
    *spl = (uint32_t)s;
    *n_blocks = (uint32_t)((n_samples + per_block * s - 1) / (per_block * s));
}

uint32_t max_blocks(uint64_t n_samples) {
    uint32_t spl, nb;
    plan_item(n_samples, &spl, &nb);
    if (n_samples <= kPipeMaxSamples) nb = std::max<uint32_t>(nb, (uint32_t)((n_samples + 63) / 64));
    return nb;
}

int build_batch(const ld_problem* p, ld_integrator integ, ld_precision prec,
                const ld_level_range* ranges, int32_t n_ranges, KArgs* args,
                uint32_t* total_blocks) {
    if (ranges == nullptr || n_ranges < 1 || n_ranges > LD_MAX_LEVELS)
        return fail(LD_EINVAL, "need 1..LD_MAX_LEVELS ranges");
    if (integ != LD_SE && integ != LD_GL && integ != LD_BAOAB)
        return fail(LD_EINVAL, "unknown integrator");
    if (prec != LD_FP64 && prec != LD_FP32) return fail(LD_EINVAL, "unknown precision");
    int rc = validate_problem(p);
    if (rc != LD_OK) return rc;
    std::memset(args, 0, sizeof *args);
    rc = make_kproblem(p, integ, &args->prob);
    if (rc != LD_OK) return rc;
    args->precision = (int32_t)prec;
    args->n_items = n_ranges;
    // order: largest M_l first so the longest blocks start first
    int order[LD_MAX_LEVELS];
    for (int i = 0; i < n_ranges; ++i) order[i] = i;
    std::stable_sort(order, order + n_ranges,
                     [&](int a, int b) { return ranges[a].level > ranges[b].level; });
    uint64_t blocks = 0;
    const int32_t top_level = ranges[order[0]].level;
    for (int j = 0; j < n_ranges; ++j) {
        const ld_level_range& r = ranges[order[j]];
        if (r.level < 0 || r.level >= LD_MAX_LEVELS)
            return fail(LD_EINVAL, "level must lie in 0..LD_MAX_LEVELS-1");
        if (std::ldexp((double)p->M0, r.level) > 2147483648.0)
            return fail(LD_EINVAL, "M0 * 2^level must not exceed 2^31");
        if (r.sample_begin + r.n_samples < r.sample_begin)
            return fail(LD_EINVAL, "sample range overflows 64 bits");
        rc = check_stability(p, integ, r.level);
        if (rc != LD_OK) return rc;
        if (args->prob.adaptive && std::ldexp((double)p->M0, r.level) > 67108864.0)
            return fail(LD_EINVAL, "adaptive steps need M0 * 2^level <= 2^26");
        KItem& it = args->items[j];
        it.level = r.level;
        const uint64_t M = (uint64_t)p->M0 << r.level;
        if (r.level >= 1 && r.n_samples <= kPipeMaxSamples && M >= kPipeMinSteps && !args->prob.adaptive) {
            // long paths and few samples: latency-bound, use the wave-specialised blocks
            it.mode = KMODE_PIPE;
            it.spl = 1;
            it.n_blocks = (uint32_t)((r.n_samples + 63) / 64);
        } else {
            it.mode = KMODE_STREAM;
            const uint64_t target = !args->prob.adaptive ? kTargetBlocks
                                    : (prec == LD_FP32 ? kAdaptiveTargetBlocksFp32 : kAdaptiveTargetBlocksFp64);
            plan_item(r.n_samples, &it.spl, &it.n_blocks, target);
        }
        it.prio = (uint16_t)std::max(0, 3 - (top_level - r.level));
        it.block_begin = (uint32_t)blocks;
        it.sample_begin = r.sample_begin;
        it.n_samples = r.n_samples;
        it.out_slot = (uint32_t)order[j];
        blocks += it.n_blocks;
    }
    if (blocks > 0x7FFFFFFFull) return fail(LD_EINVAL, "too many blocks");
    *total_blocks = (uint32_t)blocks;
    return LD_OK;
}

int run_batch(const ld_problem* p, ld_integrator integ, ld_precision prec,
              const ld_level_range* ranges, int32_t n_ranges, ld_level_sums* d_out,
              void* d_workspace, size_t workspace_bytes, double* d_dump, void* stream) {
    KArgs args;
    uint32_t total = 0;
    int rc = build_batch(p, integ, prec, ranges, n_ranges, &args, &total);
    if (rc != LD_OK) return rc;
    if (d_out == nullptr) return fail(LD_EINVAL, "d_out is NULL");
    const size_t need = (size_t)total * sizeof(ld_level_sums);
    if (need > 0 && d_workspace == nullptr) return fail(LD_EINVAL, "d_workspace is NULL");
    if (workspace_bytes < need) return fail(LD_ENOMEM, "workspace smaller than required");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LD_ENODEVICE, "no HIP device");
    rc = launch_levels(args, total, (ld_level_sums*)d_workspace, d_out, d_dump, stream);
    if (rc != LD_OK) return fail(rc, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
    return LD_OK;
}

}  // namespace ldm

using namespace ldm;

extern "C" {

size_t mlmc_level_sums_workspace(uint64_t n_samples) {
    return ((size_t)max_blocks(n_samples) + 1) * sizeof(ld_level_sums);
}

int mlmc_level_sums(const ld_problem* problem, ld_integrator integrator, ld_precision precision,
                    int32_t level, uint64_t sample_begin, uint64_t n_samples, ld_level_sums* d_out,
                    void* d_workspace, size_t workspace_bytes, void* hip_stream) {
    ld_level_range r;
    std::memset(&r, 0, sizeof r);
    r.level = level;
    r.sample_begin = sample_begin;
    r.n_samples = n_samples;
    return run_batch(problem, integrator, precision, &r, 1, d_out, d_workspace, workspace_bytes,
                     nullptr, hip_stream);
}

int mlmc_level_sums_noalloc(const ld_problem* problem, ld_integrator integrator,
                            ld_precision precision, int32_t level, uint64_t sample_begin,
                            uint64_t n_samples, ld_level_sums* d_out, void* hip_stream) {
    ld_level_range r;
    std::memset(&r, 0, sizeof r);
    r.level = level;
    r.sample_begin = sample_begin;
    r.n_samples = n_samples;
    KArgs args;
    uint32_t total = 0;
    int rc = build_batch(problem, integrator, precision, &r, 1, &args, &total);
    if (rc != LD_OK) return rc;
    if (d_out == nullptr) return fail(LD_EINVAL, "d_out is NULL");
    if (total > kScratchPartials)
        return fail(LD_ENOMEM, "range needs " + std::to_string(total) + " block partials; the "
                    "library's own array holds " + std::to_string(kScratchPartials));
    ld_level_sums* d_scratch = nullptr;
    rc = scratch_partials(&d_scratch);
    if (rc != LD_OK) return fail(rc, "no device address for the library's partials array");
    rc = launch_levels(args, total, d_scratch, d_out, nullptr, hip_stream);
    if (rc != LD_OK) return fail(rc, std::string("kernel launch failed: ") + hipGetErrorString(hipGetLastError()));
    return LD_OK;
}

size_t mlmc_level_sums_batch_workspace(const ld_level_range* ranges, int32_t n_ranges) {
    if (ranges == nullptr || n_ranges < 1) return 0;
    size_t total = 0;
    for (int i = 0; i < n_ranges; ++i) total += max_blocks(ranges[i].n_samples);
    return total * sizeof(ld_level_sums);
}

int mlmc_level_sums_batch(const ld_problem* problem, ld_integrator integrator,
                          ld_precision precision, const ld_level_range* ranges, int32_t n_ranges,
                          ld_level_sums* d_out, void* d_workspace, size_t workspace_bytes,
                          void* hip_stream) {
    return run_batch(problem, integrator, precision, ranges, n_ranges, d_out, d_workspace,
                     workspace_bytes, nullptr, hip_stream);
}

int mlmc_level_samples(const ld_problem* problem, ld_integrator integrator, ld_precision precision,
                       int32_t level, uint64_t sample_begin, uint64_t n_samples, double* d_pf_pc,
                       void* d_workspace, size_t workspace_bytes, void* hip_stream) {
    if (d_pf_pc == nullptr && n_samples > 0) return fail(LD_EINVAL, "d_pf_pc is NULL");
    const uint32_t nb = max_blocks(n_samples);
    const size_t need = ((size_t)nb + 1) * sizeof(ld_level_sums);
    if (d_workspace == nullptr) return fail(LD_EINVAL, "d_workspace is NULL");
    if (workspace_bytes < need) return fail(LD_ENOMEM, "workspace smaller than required");
    ld_level_range r;
    std::memset(&r, 0, sizeof r);
    r.level = level;
    r.sample_begin = sample_begin;
    r.n_samples = n_samples;
    // the merged sums go to the last slot of the workspace
    ld_level_sums* d_sums = (ld_level_sums*)d_workspace + nb;
    return run_batch(problem, integrator, precision, &r, 1, d_sums, d_workspace,
                     (size_t)nb * sizeof(ld_level_sums), d_pf_pc, hip_stream);
}

const char* ld_strerror(int status) {
    switch (status) {
        case LD_OK: return "ok";
        case LD_WARN_NOT_CONVERGED: return "not converged (stopped at L_max or max_iter)";
        case LD_EINVAL: return "invalid argument";
        case LD_EUNSTABLE: return "symplectic Euler step unstable (lambda_max * h >= 2)";
        case LD_ENOMEM: return "workspace too small";
        case LD_EDEVICE: return "HIP device error";
        case LD_ENONFINITE: return "non-finite samples";
        case LD_ENODEVICE: return "no usable device";
        case LD_PENDING: return "query still running";
        case LD_EBUSY: return "no free query slot within the HBM budget";
        default: return "unknown status";
    }
}

const char* ld_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
