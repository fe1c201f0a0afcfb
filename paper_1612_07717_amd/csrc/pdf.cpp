// pdf.cpp -- the binned concentration (vector QoI of Sec. 6.4): per-bin level sums, the
// max-variance planner, and the MLMC and standard Monte Carlo drivers.
//
// A level's samples run in the ordinary path kernels with the position as QoI and a
// per-sample dump of (X_f, X_c); the bins kernel turns the dump into per-bin sums. Large
// ranges are cut into chunks of kChunk samples (the dump of a chunk is 16 B per sample),
// always at the same boundaries, so the summation order depends on the range alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.hpp"

using namespace ldm;

namespace {

constexpr uint64_t kChunk = (uint64_t)1 << 22;   // samples per dump

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct PdfWs {
    size_t dump, run, bins, total;
};

PdfWs pdf_layout(uint64_t n, int32_t k) {
    PdfWs w;
    w.dump = align256((size_t)16 * n);
    w.run = align256(((size_t)max_blocks(n) + 1) * sizeof(ld_level_sums));
    w.bins = align256((size_t)pdf_blocks(n) * (size_t)k * sizeof(ld_level_sums));
    w.total = w.dump + w.run + w.bins;
    return w;
}

int validate_bins(const ld_bins* b) {
    if (b == nullptr) return fail(LD_EINVAL, "bins is NULL");
    if (b->n_bins < 1 || b->n_bins > LD_MAX_BINS) return fail(LD_EINVAL, "need 1 <= n_bins <= LD_MAX_BINS");
    if (!(b->width > 0.0) || !std::isfinite(b->width) || !std::isfinite(b->a0))
        return fail(LD_EINVAL, "bins need a finite a0 and width > 0");
    return LD_OK;
}

// The problem as the path kernels see it (position as QoI), and as the bins kernel sees
// it (the box of the first bin carries r, delta and the smoothing coefficients).
int split_problem(const ld_problem* p, const ld_bins* b, ld_integrator integ, ld_problem* path, KProblem* kbox) {
    *path = *p;
    path->qoi.kind = LD_QOI_MEAN_Z;
    path->qoi.a = path->qoi.b = 0.0;
    ld_problem box = *p;
    box.qoi.kind = LD_QOI_P_BOX;
    box.qoi.a = b->a0;
    box.qoi.b = b->a0 + b->width;
    int rc = validate_problem(&box);
    if (rc != LD_OK) return rc;
    return make_kproblem(&box, integ, kbox);
}

int pdf_chunk(const ld_problem* path, const KProblem& kbox, ld_integrator integ, ld_precision prec,
              int32_t level, uint64_t begin, uint64_t n, const ld_bins* b, ld_level_sums* d_out, char* ws,
              const PdfWs& lay, hipStream_t stream) {
    double* d_dump = (double*)ws;
    ld_level_sums* d_run = (ld_level_sums*)(ws + lay.dump);
    ld_level_sums* d_run_out = d_run + max_blocks(n);
    ld_level_sums* d_bins = (ld_level_sums*)(ws + lay.dump + lay.run);
    ld_level_range r;
    std::memset(&r, 0, sizeof r);
    r.level = level;
    r.sample_begin = begin;
    r.n_samples = n;
    int rc = run_batch(path, integ, prec, &r, 1, d_run_out, d_run, lay.run - sizeof(ld_level_sums), d_dump, stream);
    if (rc != LD_OK) return rc;
    KBins kb;
    kb.a0 = b->a0;
    kb.width = b->width;
    kb.n_bins = b->n_bins;
    kb.level = level;
    kb.n = n;
    rc = launch_pdf_bins(kb, kbox, d_dump, d_bins, d_out, stream);
    if (rc != LD_OK) return fail(rc, "bins kernel launch failed");
    return LD_OK;
}

struct BinSums {
    double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    uint64_t n = 0, bad = 0;
    void add(const ld_level_sums& x) {
        for (int q = 0; q < 4; ++q) {
            const double t = s[q] + x.s[q];
            const double big = std::fabs(s[q]) >= std::fabs(x.s[q]) ? s[q] : x.s[q];
            const double small = std::fabs(s[q]) >= std::fabs(x.s[q]) ? x.s[q] : s[q];
            c[q] = (c[q] + x.c[q]) + ((big - t) + small);
            s[q] = t;
        }
        n += x.n;
        bad += x.n_nonfinite;
    }
    double value(int q) const { return s[q] + c[q]; }
};

void mean_var(uint64_t n_, double s1, double s2, double* mean, double* var) {
    const double n = (double)n_;
    *mean = n_ > 0 ? s1 / n : 0.0;
    *var = n_ > 1 ? (s2 - n * *mean * *mean) / (n - 1.0) : 0.0;
    if (!(*var > 0.0)) *var = 0.0;
}

// Draws samples [begin, begin + n) of `level` in chunks and adds their per-bin sums to
// acc[0..k). The chunk results come back through one pinned-free staging copy each.
int draw(const ld_problem* path, const KProblem& kbox, ld_integrator integ, ld_precision prec, int32_t level,
         uint64_t begin, uint64_t n, const ld_bins* b, char* ws, const PdfWs& lay, ld_level_sums* d_out,
         hipStream_t stream, BinSums* acc) {
    std::vector<ld_level_sums> h((size_t)b->n_bins);
    for (uint64_t off = 0; off < n; off += kChunk) {
        const uint64_t m = std::min(kChunk, n - off);
        int rc = pdf_chunk(path, kbox, integ, prec, level, begin + off, m, b, d_out, ws, lay, stream);
        if (rc != LD_OK) return rc;
        if (hipMemcpyAsync(h.data(), d_out, h.size() * sizeof(ld_level_sums), hipMemcpyDeviceToHost, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(LD_EDEVICE, std::string("pdf level sums failed: ") + hipGetErrorString(hipGetLastError()));
        for (int32_t i = 0; i < b->n_bins; ++i) acc[i].add(h[i]);
    }
    return LD_OK;
}

}  // namespace

extern "C" {

size_t mlmc_pdf_level_sums_workspace(uint64_t n_samples, int32_t n_bins) {
    if (n_bins < 1 || n_bins > LD_MAX_BINS) return 0;
    return pdf_layout(n_samples, n_bins).total;
}

size_t mlmc_estimate_pdf_workspace(int32_t n_bins) {
    if (n_bins < 1 || n_bins > LD_MAX_BINS) return 0;
    return pdf_layout(kChunk, n_bins).total + align256((size_t)n_bins * sizeof(ld_level_sums));
}

int mlmc_pdf_level_sums(const ld_problem* problem, ld_integrator integrator, ld_precision precision,
                        int32_t level, uint64_t sample_begin, uint64_t n_samples, const ld_bins* bins,
                        ld_level_sums* d_out, void* d_workspace, size_t workspace_bytes, void* hip_stream) {
    int rc = validate_bins(bins);
    if (rc != LD_OK) return rc;
    if (problem == nullptr) return fail(LD_EINVAL, "problem is NULL");
    if (d_out == nullptr) return fail(LD_EINVAL, "d_out is NULL");
    ld_problem path;
    KProblem kbox;
    rc = split_problem(problem, bins, integrator, &path, &kbox);
    if (rc != LD_OK) return rc;
    const PdfWs lay = pdf_layout(n_samples, bins->n_bins);
    if (d_workspace == nullptr) return fail(LD_EINVAL, "d_workspace is NULL");
    if (workspace_bytes < lay.total) return fail(LD_ENOMEM, "workspace smaller than mlmc_pdf_level_sums_workspace()");
    return pdf_chunk(&path, kbox, integrator, precision, level, sample_begin, n_samples, bins, d_out,
                     (char*)d_workspace, lay, (hipStream_t)hip_stream);
}

int mlmc_plan_pdf(const ld_pdf_plan_in* in, ld_pdf_plan_out* out) {
    if (in == nullptr || out == nullptr) return fail(LD_EINVAL, "NULL argument");
    if (in->L < 0 || in->L >= LD_MAX_LEVELS || in->M0 < 1 || !(in->eps > 0) || in->n_bins < 1 ||
        in->n_bins > LD_MAX_BINS)
        return fail(LD_EINVAL, "invalid planner input");
    std::memset(out, 0, sizeof *out);
    const int32_t L = in->L, k = in->n_bins;
    double Ymax[LD_MAX_LEVELS];
    static thread_local double Yhat[LD_MAX_LEVELS][LD_MAX_BINS];
    for (int32_t l = 0; l <= L; ++l) {
        out->V[l] = 0.0;
        Ymax[l] = 0.0;
        for (int32_t i = 0; i < k; ++i) {
            double mean, var;
            mean_var(in->n[l], in->sum1[l][i], in->sum2[l][i], &mean, &var);
            Yhat[l][i] = mean;
            out->estimate[i] += mean;
            out->V[l] = std::max(out->V[l], var);               // max_i Var[Y_{l,i}]
            Ymax[l] = std::max(Ymax[l], std::fabs(mean));
        }
    }
    for (int32_t i = 0; i < k; ++i) {                           // max_i sum_l V_{l,i} / N_l
        double sv = 0.0;
        for (int32_t l = 0; l <= L; ++l) {
            double mean, var;
            mean_var(in->n[l], in->sum1[l][i], in->sum2[l][i], &mean, &var);
            if (in->n[l] > 0) sv += var / (double)in->n[l];
        }
        out->stat_var = std::max(out->stat_var, sv);
    }
    const double alpha = (in->alpha > 0.0) ? in->alpha : fit_alpha(Ymax, L);
    out->alpha = alpha;
    const double r = std::pow(2.0, alpha);
    double bias = 0.0;
    if (L >= 1)
        for (int32_t i = 0; i < k; ++i)
            bias = std::max(bias, std::max(std::fabs(Yhat[L][i]), std::fabs(Yhat[L - 1][i]) / r) / (r - 1.0));
    out->bias_est = bias;
    ld_plan_in sc;
    std::memset(&sc, 0, sizeof sc);
    sc.L = L;
    sc.M0 = in->M0;
    for (int32_t l = 0; l <= L; ++l) sc.n[l] = in->n[l];
    sc.L_max = in->L_max;
    sc.fixed_L = in->fixed_L;
    sc.N_init = in->N_init;
    int32_t Lout = L;
    out->status = decide(&sc, out->V, bias, in->eps, out->dn, &Lout);
    out->L = Lout;
    return LD_OK;
}

int mlmc_estimate_pdf(double eps, const ld_bins* bins, const ld_qoi* qoi, ld_integrator integrator,
                      const ld_profile* profile, const ld_estimate_opts* opts_in, ld_estimator estimator,
                      ld_pdf_result* out) {
    const auto t_start = std::chrono::steady_clock::now();
    if (qoi == nullptr || profile == nullptr || out == nullptr) return fail(LD_EINVAL, "NULL argument");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(LD_EINVAL, "eps must be positive");
    if (estimator != LD_MLMC && estimator != LD_STMC) return fail(LD_EINVAL, "unknown estimator");
    int rc = validate_bins(bins);
    if (rc != LD_OK) return rc;
    ld_estimate_opts opts;
    if (opts_in)
        opts = *opts_in;
    else
        mlmc_estimate_default_opts(&opts);
    if (opts.eps_is_relative) return fail(LD_EINVAL, "the binned estimate takes an absolute eps");
    if (opts.N_init < 2) return fail(LD_EINVAL, "N_init must be >= 2");
    std::memset(out, 0, sizeof *out);
    out->estimator = estimator;
    const int32_t k = bins->n_bins;
    ld_problem prob;
    std::memset(&prob, 0, sizeof prob);
    prob.profile = *profile;
    prob.release = opts.release;
    prob.qoi = *qoi;
    prob.T = opts.T;
    prob.M0 = opts.M0;
    prob.stream_id = opts.stream_id;
    prob.seed = opts.seed;
    prob.x_adapt = opts.x_adapt;
    if (estimator == LD_STMC) {
        if (opts.fixed_L < 0 || opts.fixed_L >= LD_MAX_LEVELS) return fail(LD_EINVAL, "StMC needs 0 <= fixed_L");
        if (std::ldexp((double)opts.M0, opts.fixed_L) > 2147483648.0)
            return fail(LD_EINVAL, "M0 * 2^fixed_L must not exceed 2^31");
        prob.M0 = opts.M0 << opts.fixed_L;   // the single fine path of level L = level 0 of this
    } else {
        const int32_t L0 = opts.fixed_L >= 0 ? opts.fixed_L : opts.L_min;
        if (L0 < 0 || L0 >= LD_MAX_LEVELS || opts.L_max < L0 || opts.L_max >= LD_MAX_LEVELS)
            return fail(LD_EINVAL, "need 0 <= L_min <= L_max < LD_MAX_LEVELS");
    }
    rc = validate_problem(&prob);
    if (rc != LD_OK) return rc;
    rc = check_stability(&prob, integrator, 0);
    if (rc != LD_OK) return rc;
    ld_problem path;
    KProblem kbox;
    rc = split_problem(&prob, bins, integrator, &path, &kbox);
    if (rc != LD_OK) return rc;

    hipStream_t stream = (hipStream_t)opts.hip_stream;
    const PdfWs lay = pdf_layout(kChunk, k);
    char* ws = nullptr;
    ld_level_sums* d_out = nullptr;
    const bool own_ws = opts.d_workspace == nullptr;
    if (!own_ws) {
        if (opts.workspace_bytes < mlmc_estimate_pdf_workspace(k))
            return fail(LD_ENOMEM, "workspace smaller than mlmc_estimate_pdf_workspace()");
        ws = (char*)opts.d_workspace;
        d_out = (ld_level_sums*)(ws + lay.total);
    } else if (hipMalloc((void**)&ws, lay.total) != hipSuccess ||
               hipMalloc((void**)&d_out, (size_t)k * sizeof(ld_level_sums)) != hipSuccess) {
        if (ws) (void)hipFree(ws);
        return fail(LD_EDEVICE, "hipMalloc of the workspace failed");
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool timing = hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess;
    std::vector<BinSums> sums((size_t)LD_MAX_LEVELS * k);
    uint64_t drawn[LD_MAX_LEVELS] = {0};
    const int max_iter = opts.max_iter > 0 ? opts.max_iter : 100;
    int iter = 0;
    double device_s = 0.0;
    auto timed_draw = [&](int32_t level, uint64_t begin, uint64_t n, BinSums* acc) -> int {
        if (timing) (void)hipEventRecord(ev0, stream);
        const int r = draw(&path, kbox, integrator, opts.precision, level, begin, n, bins, ws, lay, d_out, stream, acc);
        if (r == LD_OK && timing) {
            (void)hipEventRecord(ev1, stream);
            (void)hipEventSynchronize(ev1);
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) device_s += 1e-3 * ms;
        }
        return r;
    };

    if (estimator == LD_STMC) {
        uint64_t dn = opts.N_init;
        double V = 0.0;
        for (;;) {
            rc = timed_draw(0, drawn[0], dn, sums.data());
            if (rc != LD_OK) break;
            drawn[0] += dn;
            ++iter;
            const uint64_t n = sums[0].n;
            V = 0.0;
            for (int32_t i = 0; i < k; ++i) {
                double mean, var;
                mean_var(n, sums[i].value(0), sums[i].value(1), &mean, &var);
                out->estimate[i] = mean;
                V = std::max(V, var);
            }
            const double target = std::ceil(2.0 * V / (eps * eps));
            dn = (target > (double)n) ? (uint64_t)target - n : 0;
            if (!((double)dn > 0.01 * (double)n) || iter >= max_iter) break;
        }
        if (rc == LD_OK) {
            out->L = opts.fixed_L;
            out->N[0] = drawn[0];
            out->V[0] = V;
            out->stat_var = V / (double)std::max<uint64_t>(sums[0].n, 1);
            out->rmse_est = std::sqrt(out->stat_var);
            out->status = 1;
            out->n_nonfinite = sums[0].bad;
            out->fine_steps = (double)drawn[0] * (double)prob.M0;
        }
    } else {
        static thread_local ld_pdf_plan_in pin;
        std::memset(&pin, 0, sizeof pin);
        pin.L = opts.fixed_L >= 0 ? opts.fixed_L : opts.L_min;
        pin.n_bins = k;
        pin.M0 = opts.M0;
        pin.L_max = opts.L_max;
        pin.eps = eps;
        pin.fixed_L = opts.fixed_L;
        pin.N_init = opts.N_init;
        pin.alpha = opts.alpha;
        uint64_t dn[LD_MAX_LEVELS] = {0};
        for (int32_t l = 0; l <= pin.L; ++l) dn[l] = opts.N_init;
        ld_pdf_plan_out plan;
        std::memset(&plan, 0, sizeof plan);
        for (;;) {
            for (int32_t l = 0; l <= pin.L && rc == LD_OK; ++l) {
                if (dn[l] == 0) continue;
                rc = timed_draw(l, drawn[l], dn[l], &sums[(size_t)l * k]);
                drawn[l] += dn[l];
            }
            if (rc != LD_OK) break;
            for (int32_t l = 0; l <= pin.L; ++l) {
                pin.n[l] = sums[(size_t)l * k].n;
                for (int32_t i = 0; i < k; ++i) {
                    pin.sum1[l][i] = sums[(size_t)l * k + i].value(0);
                    pin.sum2[l][i] = sums[(size_t)l * k + i].value(1);
                }
            }
            mlmc_plan_pdf(&pin, &plan);
            ++iter;
            if (plan.status != 0 || iter >= max_iter) break;
            pin.L = plan.L;
            std::memcpy(dn, plan.dn, sizeof dn);
        }
        if (rc == LD_OK) {
            for (int32_t i = 0; i < k; ++i) out->estimate[i] = plan.estimate[i];
            out->bias_est = plan.bias_est;
            out->stat_var = plan.stat_var;
            out->rmse_est = std::sqrt(plan.bias_est * plan.bias_est + plan.stat_var);
            out->L = plan.L;
            out->status = plan.status == 0 ? 2 : plan.status;
            for (int32_t l = 0; l <= plan.L; ++l) {
                out->N[l] = drawn[l];
                out->n_nonfinite += sums[(size_t)l * k].bad;
                out->V[l] = plan.V[l];
                out->fine_steps += (double)drawn[l] * std::ldexp((double)opts.M0, l);
            }
        }
    }
    if (timing) {
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    if (own_ws) {
        (void)hipFree(ws);
        (void)hipFree(d_out);
    }
    if (rc != LD_OK) return rc;
    out->iterations = iter;
    out->device_seconds = device_s;
    out->wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (out->n_nonfinite > 0) return fail(LD_ENONFINITE, "some samples were non-finite");
    return out->status == 1 ? LD_OK : LD_WARN_NOT_CONVERGED;
}

}  // extern "C"
