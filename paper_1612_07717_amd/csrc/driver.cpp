// driver.cpp -- the adaptive MLMC driver (host, FP64) and mlmc_estimate.
//
// The mean square error of the estimator (Eq. 17) is bias^2 + sum_l V_l / N_l; each
// part is held below eps^2 / 2 (Sec. 3.2, Sec. 6). For a cost C_l = M_l per sample
// (condition (iv) of the theorem of Sec. 3.3) the sample counts minimising
// sum_l N_l C_l under sum_l V_l / N_l = eps^2 / 2 are
//     N_l = 2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k)
// (Lagrange multipliers; Giles 2008, cited in Sec. 6). The bias is estimated from the
// finest level means with E[P_l - P] ~ c h_l^alpha (Sec. 6): then
// E[P_L - P] ~ Yhat_L / (2^alpha - 1), and Yhat_{L-1} 2^-alpha estimates the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "host_common.hpp"

using namespace ldm;

bool ldm::exceeds_budget(double max_fine_steps, int32_t M0, const uint64_t* drawn, const uint64_t* dn,
                         int32_t L) {
    if (!(max_fine_steps > 0.0)) return false;
    double cost = 0.0;
    for (int32_t l = 0; l <= L && l < LD_MAX_LEVELS; ++l)
        cost += ((double)drawn[l] + (double)dn[l]) * std::ldexp((double)M0, l);
    return cost > max_fine_steps;
}

namespace {

double cost_of_level(int32_t M0, int32_t l) { return std::ldexp((double)M0, l); }

// Samples needed on each level 0..L for the variance budget, minus those already
// drawn (0 if none are needed).
void variance_rule(const ld_plan_in* in, int32_t L, const double* V, double eps_abs,
                   uint64_t* dn) {
    double weighted = 0.0;
    for (int32_t l = 0; l <= L; ++l) weighted += std::sqrt(V[l] * cost_of_level(in->M0, l));
    const double scale = 2.0 * weighted / (eps_abs * eps_abs);
    for (int32_t l = 0; l <= L; ++l) {
        const double want = std::ceil(scale * std::sqrt(V[l] / cost_of_level(in->M0, l)));
        const uint64_t have = (l <= in->L) ? in->n[l] : 0;
        if (!(want > (double)have))
            dn[l] = 0;
        else if (want >= 4.0e18)
            dn[l] = (uint64_t)1 << 62;
        else
            dn[l] = (uint64_t)want - have;
    }
}

double fitted_alpha(const double* Yhat, int32_t L) {
    // least-squares slope of -log2 |Yhat_l| against l over l = 1..L
    int cnt = 0;
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    for (int32_t l = 1; l <= L; ++l) {
        const double a = std::fabs(Yhat[l]);
        if (!(a > 0.0)) continue;
        const double y = -std::log2(a);
        sx += l;
        sy += y;
        sxx += (double)l * l;
        sxy += l * y;
        ++cnt;
    }
    double alpha = 1.0;
    if (cnt >= 2) {
        const double den = cnt * sxx - sx * sx;
        if (den > 0) alpha = (cnt * sxy - sx * sy) / den;
    }
    return std::min(std::max(alpha, 0.5), 2.0);
}

struct HostSums {
    double s[4] = {0, 0, 0, 0}, c[4] = {0, 0, 0, 0};
    uint64_t n = 0, bad = 0;
};

void merge_into(HostSums& acc, const ld_level_sums& add) {
    for (int k = 0; k < 4; ++k) {
        const double t = acc.s[k] + add.s[k];
        const double big = std::fabs(acc.s[k]) >= std::fabs(add.s[k]) ? acc.s[k] : add.s[k];
        const double small = std::fabs(acc.s[k]) >= std::fabs(add.s[k]) ? add.s[k] : acc.s[k];
        acc.c[k] = (acc.c[k] + add.c[k]) + ((big - t) + small);
        acc.s[k] = t;
    }
    acc.n += add.n;
    acc.bad += add.n_nonfinite;
}

// Early top-up of the first iteration (ld_estimate_opts.early_topup). The levels are
// split at L0 - kEarlyGap: the long ones (L0 - kEarlyGap < l <= L0) run their first
// batch on the caller's stream, the short ones theirs on a second stream. As soon as the
// short levels' sums are back, the variance rule is applied to them alone: with the sum
// of sqrt(V_k C_k) over the short levels only, each N_l is at most what the full rule will
// ask once the long levels are known (for an absolute eps; for a relative one the short
// levels' partial estimate stands in, and the long levels' corrections are small). That
// many are drawn at once, on the second stream, while the long levels still run; the
// ordinary iterations follow. The sum of sqrt(V_k C_k) in that rule also counts the long
// levels, whose variances are not known yet, by extending the short levels' terms
// geometrically: term_k = term_Ls rho^(k - Ls), with rho the ratio of the last two short
// terms clamped to [kRhoMin, 1] (a variance that decays like 2^-beta l with beta between
// 1 and 3), times kLongMargin; and each short level's count is raised by three standard
// errors of its variance estimate, 3 sqrt(2 / n_l), so that the full rule, applied with
// the variances of all samples, rarely asks for more than its 1 % tolerance. Where the
// guess is high the short levels get a few more samples than the full rule asks, which
// run beside the long levels anyway; where it is low the first ordinary iteration draws
// the rest, as without the guess. The draws are
// the same (sample indices from 0 upward on every level), only their order in time
// changes, so the estimate is the plain MLMC estimate of whatever N_l end up drawn.
constexpr int32_t kEarlyGap = 5;
constexpr double kRhoMin = 0.5;
constexpr double kLongMargin = 1.25;

// The second stream and the events of an estimate, kept for reuse instead of being made
// and destroyed by every call. A kit belongs to one device and to one call at a time:
// calls take a free kit of their device from the pool (or make one) and return it when
// they end, so concurrent estimates never share a stream or an event. Kits live until
// the process ends. The second stream has the default priority and does not synchronise
// with the NULL stream by itself; every use orders it explicitly.
struct EstimateKit {
    int device = -1;
    hipStream_t s2 = nullptr;                         // the early top-up's second stream
    hipEvent_t ev0 = nullptr, ev1 = nullptr;          // kernel time on the caller's stream
    hipEvent_t e_start = nullptr;                     // the caller's stream before any launch
    hipEvent_t e_long = nullptr, e_short0 = nullptr, e_short = nullptr;
};

std::mutex g_kit_mutex;
std::vector<EstimateKit*> g_free_kits;

// A free kit of `device` (the current device), or a new one; nullptr if the device
// refuses a stream or an event.
EstimateKit* acquire_kit(int device) {
    {
        std::lock_guard<std::mutex> lock(g_kit_mutex);
        for (size_t i = 0; i < g_free_kits.size(); ++i) {
            if (g_free_kits[i]->device == device) {
                EstimateKit* k = g_free_kits[i];
                g_free_kits.erase(g_free_kits.begin() + (long)i);
                return k;
            }
        }
    }
    EstimateKit* k = new EstimateKit;
    k->device = device;
    bool ok = hipStreamCreateWithFlags(&k->s2, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t* e : {&k->ev0, &k->ev1, &k->e_start, &k->e_long, &k->e_short0, &k->e_short})
        ok = ok && hipEventCreate(e) == hipSuccess;
    if (!ok) {
        for (hipEvent_t e : {k->ev0, k->ev1, k->e_start, k->e_long, k->e_short0, k->e_short})
            if (e) (void)hipEventDestroy(e);
        if (k->s2) (void)hipStreamDestroy(k->s2);
        delete k;
        return nullptr;
    }
    return k;
}

void release_kit(EstimateKit* k) {
    if (k == nullptr) return;
    std::lock_guard<std::mutex> lock(g_kit_mutex);
    g_free_kits.push_back(k);
}

struct KitGuard {
    EstimateKit* k;
    ~KitGuard() { release_kit(k); }
};

struct Batch {
    ld_level_range r[LD_MAX_LEVELS];
    int32_t n = 0;
    void add(int32_t level, uint64_t begin, uint64_t count) {
        if (count == 0) return;
        r[n].level = level;
        r[n].reserved = 0;
        r[n].sample_begin = begin;
        r[n].n_samples = count;
        ++n;
    }
    size_t blocks() const { return n > 0 ? mlmc_level_sums_batch_workspace(r, n) / sizeof(ld_level_sums) : 0; }
};

}  // namespace

// The decision of one iteration (shared by the scalar and the vector planners), given
// each level's variance V[0..in->L], the bias estimate and the absolute tolerance:
// levels needing more than 1 % extra samples get them (status 0); otherwise the
// estimate has converged (1), or the bias test adds level L + 1 with V_{L+1} = V_L / 4
// (condition (iii)) and at least N_init samples (0), or L_max is reached (2).
int ldm::decide(const ld_plan_in* in, const double* Vl, double bias, double eps_abs, uint64_t* dn,
                int32_t* L_out) {
    const int32_t L = in->L;
    *L_out = L;
    variance_rule(in, L, Vl, eps_abs, dn);
    bool more = false;
    for (int32_t l = 0; l <= L; ++l)
        if ((double)dn[l] > 0.01 * (double)in->n[l]) more = true;
    if (more) return 0;
    for (int32_t l = 0; l <= L; ++l) dn[l] = 0;
    if (in->fixed_L >= 0 || L < 1 || bias <= eps_abs / std::sqrt(2.0)) return 1;
    if (L >= in->L_max || L + 1 >= LD_MAX_LEVELS) return 2;
    double V[LD_MAX_LEVELS];
    for (int32_t l = 0; l <= L; ++l) V[l] = Vl[l];
    V[L + 1] = V[L] / 4.0;
    variance_rule(in, L + 1, V, eps_abs, dn);
    dn[L + 1] = std::max(dn[L + 1], in->N_init);
    *L_out = L + 1;
    return 0;
}

double ldm::fit_alpha(const double* Yhat, int32_t L) { return fitted_alpha(Yhat, L); }

extern "C" {

int mlmc_plan(const ld_plan_in* in, ld_plan_out* out) {
    if (in == nullptr || out == nullptr) return fail(LD_EINVAL, "NULL argument");
    if (in->L < 0 || in->L >= LD_MAX_LEVELS || in->M0 < 1 || !(in->eps > 0))
        return fail(LD_EINVAL, "invalid planner input");
    std::memset(out, 0, sizeof *out);
    const int32_t L = in->L;
    double estimate = 0.0, stat_var = 0.0;
    for (int32_t l = 0; l <= L; ++l) {
        const double n = (double)in->n[l];
        const double mean = in->n[l] > 0 ? in->sum1[l] / n : 0.0;
        double var = in->n[l] > 1 ? (in->sum2[l] - n * mean * mean) / (n - 1.0) : 0.0;
        if (!(var > 0.0)) var = 0.0;   // unbiased sample variance, clamped at 0
        out->Yhat[l] = mean;
        out->V[l] = var;
        estimate += mean;
        if (in->n[l] > 0) stat_var += var / n;
    }
    out->estimate = estimate;
    out->stat_var = stat_var;
    out->eps_abs = in->eps_is_relative ? in->eps * std::fabs(estimate) : in->eps;
    const double alpha = (in->alpha > 0.0) ? in->alpha : fitted_alpha(out->Yhat, L);
    out->alpha = alpha;
    const double r = std::pow(2.0, alpha);
    out->bias_est = (L >= 1) ? std::max(std::fabs(out->Yhat[L]), std::fabs(out->Yhat[L - 1]) / r) / (r - 1.0)
                             : 0.0;
    out->L = L;
    if (in->fixed_N) {
        out->status = 1;
        return LD_OK;
    }
    if (!(out->eps_abs > 0.0)) {   // relative eps of a zero estimate: nothing to aim at
        out->status = 2;
        return LD_OK;
    }
    int32_t Lout = L;
    out->status = decide(in, out->V, out->bias_est, out->eps_abs, out->dn, &Lout);
    out->L = Lout;
    return LD_OK;
}

void mlmc_estimate_default_opts(ld_estimate_opts* o) {
    if (o == nullptr) return;
    std::memset(o, 0, sizeof *o);
    o->release.kind = LD_RELEASE_FIXED_W;   // the paper's Sec. 6 release: 50 m, 0.1 m/s
    o->release.z0 = 50.0;
    o->release.w0 = 0.1;
    o->T = 1000.0;
    o->M0 = 40;
    o->L_min = 2;
    o->L_max = 20;
    o->fixed_L = -1;
    o->fixed_N = 0;
    o->eps_is_relative = 0;
    o->N_init = 10000;
    o->alpha = 1.0;
    o->precision = LD_FP64;
    o->max_iter = 100;
}

size_t mlmc_estimate_workspace(void) {
    // per level: its sums plus at most the blocks plan_item gives any range
    uint32_t spl, nb;
    plan_item(~(uint64_t)0 >> 2, &spl, &nb);
    return (size_t)LD_MAX_LEVELS * (1 + (size_t)nb) * sizeof(ld_level_sums);
}

int mlmc_estimate(double eps, const ld_qoi* qoi, ld_integrator integrator, const ld_profile* profile,
                  const ld_estimate_opts* opts_in, ld_estimate_result* out) {
    const auto t_start = std::chrono::steady_clock::now();
    if (qoi == nullptr || profile == nullptr || out == nullptr) return fail(LD_EINVAL, "NULL argument");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(LD_EINVAL, "eps must be positive");
    ld_estimate_opts opts;
    if (opts_in)
        opts = *opts_in;
    else
        mlmc_estimate_default_opts(&opts);
    std::memset(out, 0, sizeof *out);
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
    int rc = validate_problem(&prob);
    if (rc != LD_OK) return rc;
    const int32_t L0 = opts.fixed_L >= 0 ? opts.fixed_L : opts.L_min;
    if (L0 < 0 || L0 >= LD_MAX_LEVELS || opts.L_max < L0 || opts.L_max >= LD_MAX_LEVELS)
        return fail(LD_EINVAL, "need 0 <= L_min <= L_max < LD_MAX_LEVELS");
    if (opts.N_init < 2) return fail(LD_EINVAL, "N_init must be >= 2");
    if (!(opts.max_fine_steps >= 0.0)) return fail(LD_EINVAL, "max_fine_steps must be >= 0");
    rc = check_stability(&prob, integrator, 0);
    if (rc != LD_OK) return rc;

    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(LD_ENODEVICE, "no HIP device");
    hipStream_t stream = (hipStream_t)opts.hip_stream;
    const size_t ws_need = mlmc_estimate_workspace();
    void* ws = opts.d_workspace;
    bool own_ws = false;
    if (ws == nullptr) {
        if (hipMalloc(&ws, ws_need) != hipSuccess) return fail(LD_EDEVICE, "hipMalloc of the workspace failed");
        own_ws = true;
    } else if (opts.workspace_bytes < ws_need) {
        return fail(LD_ENOMEM, "workspace smaller than mlmc_estimate_workspace()");
    }
    ld_level_sums* d_sums = (ld_level_sums*)ws;
    void* d_partials = (void*)(d_sums + LD_MAX_LEVELS);
    const size_t partial_bytes = ws_need - LD_MAX_LEVELS * sizeof(ld_level_sums);

    EstimateKit* kit = acquire_kit(device);
    if (kit == nullptr) {
        if (own_ws) (void)hipFree(ws);
        return fail(LD_EDEVICE, "no stream or event for the estimate");
    }
    KitGuard kit_guard{kit};
    hipEvent_t ev0 = kit->ev0, ev1 = kit->ev1;

    std::vector<HostSums> sums(LD_MAX_LEVELS);
    uint64_t drawn[LD_MAX_LEVELS] = {0};
    uint64_t dn[LD_MAX_LEVELS] = {0};
    ld_plan_in pin;
    std::memset(&pin, 0, sizeof pin);
    pin.L = L0;
    pin.M0 = opts.M0;
    pin.eps = eps;
    pin.alpha = opts.alpha;
    pin.eps_is_relative = opts.eps_is_relative;
    pin.L_max = opts.L_max;
    pin.fixed_L = opts.fixed_L;
    pin.fixed_N = opts.fixed_N;
    pin.N_init = opts.N_init;
    for (int32_t l = 0; l <= L0; ++l) dn[l] = opts.N_init;
    ld_plan_out plan;
    std::memset(&plan, 0, sizeof plan);
    const int max_iter = opts.max_iter > 0 ? opts.max_iter : 100;
    int iter = 0;
    double device_s = 0.0;
    ld_level_sums host_batch[LD_MAX_LEVELS];
    rc = LD_OK;
    if (opts.early_topup && !opts.fixed_N && L0 >= kEarlyGap) {
        const int32_t Ls = L0 - kEarlyGap;               // short levels 0..Ls
        Batch longb, shortb, topb;
        for (int32_t l = Ls + 1; l <= L0; ++l) longb.add(l, 0, opts.N_init);
        for (int32_t l = 0; l <= Ls; ++l) shortb.add(l, 0, opts.N_init);
        const size_t slots = partial_bytes / sizeof(ld_level_sums);
        const size_t off = longb.blocks();               // the second stream's partials follow
        hipStream_t s2 = kit->s2;
        hipEvent_t e_long = kit->e_long, e_short0 = kit->e_short0, e_short = kit->e_short;
        if (off + shortb.blocks() > slots) {
            rc = fail(LD_ENOMEM, "early top-up: workspace too small for two batches");
        } else {
            ld_level_sums* d_sums2 = d_sums + longb.n;
            void* d_part2 = (void*)((ld_level_sums*)d_partials + off);
            const size_t part2_bytes = partial_bytes - off * sizeof(ld_level_sums);
            ld_level_sums h_long[LD_MAX_LEVELS], h_short[LD_MAX_LEVELS], h_top[LD_MAX_LEVELS];
            // the second stream starts after everything the caller queued before this call
            // (its work may still use the workspace, e.g. memory a caching allocator
            // handed out again)
            if (hipEventRecord(kit->e_start, stream) != hipSuccess ||
                hipStreamWaitEvent(s2, kit->e_start, 0) != hipSuccess)
                rc = fail(LD_EDEVICE, "early top-up: cannot order the second stream");
            if (rc == LD_OK) (void)hipEventRecord(ev0, stream);
            if (rc == LD_OK)
                rc = run_batch(&prob, integrator, opts.precision, longb.r, longb.n, d_sums, d_partials,
                               off * sizeof(ld_level_sums), nullptr, stream);
            if (rc == LD_OK) (void)hipEventRecord(e_long, stream);
            // kernel time of the second stream: each of its batches between two events
            double s2_seconds = 0.0;
            auto s2_span = [&]() {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, e_short0, e_short) == hipSuccess) s2_seconds += ms * 1e-3;
            };
            if (rc == LD_OK) (void)hipEventRecord(e_short0, s2);
            if (rc == LD_OK)
                rc = run_batch(&prob, integrator, opts.precision, shortb.r, shortb.n, d_sums2, d_part2,
                               part2_bytes, nullptr, s2);
            if (rc == LD_OK) (void)hipEventRecord(e_short, s2);
            if (rc == LD_OK &&
                (hipMemcpyAsync(h_short, d_sums2, shortb.n * sizeof(ld_level_sums), hipMemcpyDeviceToHost, s2) !=
                     hipSuccess ||
                 hipStreamSynchronize(s2) != hipSuccess))
                rc = fail(LD_EDEVICE, "level sums failed (short levels)");
            if (rc == LD_OK) s2_span();
            if (rc == LD_OK) {
                for (int32_t j = 0; j < shortb.n; ++j) {
                    merge_into(sums[shortb.r[j].level], h_short[j]);
                    drawn[shortb.r[j].level] += shortb.r[j].n_samples;
                }
                // the variance rule over the short levels alone, no level added, no bias test
                ld_plan_in ps = pin;
                ps.L = Ls;
                ps.fixed_L = Ls;
                for (int32_t l = 0; l <= Ls; ++l) {
                    ps.n[l] = sums[l].n;
                    ps.sum1[l] = sums[l].s[0] + sums[l].c[0];
                    ps.sum2[l] = sums[l].s[1] + sums[l].c[1];
                }
                ld_plan_out po;
                mlmc_plan(&ps, &po);
                uint64_t dn_s[LD_MAX_LEVELS] = {0};
                // the variance rule with the long levels' terms extrapolated (see above)
                double term[LD_MAX_LEVELS], s_short = 0.0;
                for (int32_t l = 0; l <= Ls; ++l) {
                    term[l] = std::sqrt(std::max(po.V[l], 0.0) * std::ldexp((double)opts.M0, l));
                    s_short += term[l];
                }
                const double rho = (Ls >= 1 && term[Ls - 1] > 0.0)
                                       ? std::min(1.0, std::max(kRhoMin, term[Ls] / term[Ls - 1])) : 1.0;
                double s_long = 0.0, t = term[Ls];
                for (int32_t k = Ls + 1; k <= L0; ++k) s_long += (t *= rho);
                const double scale = 2.0 * (s_short + kLongMargin * s_long) / (po.eps_abs * po.eps_abs);
                for (int32_t l = 0; l <= Ls; ++l) {
                    const double margin = 1.0 + 3.0 * std::sqrt(2.0 / (double)std::max<uint64_t>(ps.n[l], 2));
                    const double want = std::ceil(margin * scale * std::sqrt(std::max(po.V[l], 0.0) /
                                                                             std::ldexp((double)opts.M0, l)));
                    dn_s[l] = (std::isfinite(want) && want > (double)ps.n[l])
                                  ? (uint64_t)std::min(want, 1e15) - ps.n[l] : 0;
                }
                if (po.eps_abs > 0.0 && !exceeds_budget(opts.max_fine_steps, opts.M0, drawn, dn_s, Ls))
                    for (int32_t l = 0; l <= Ls; ++l) topb.add(l, drawn[l], dn_s[l]);
                if (topb.n > 0) {
                    (void)hipEventRecord(e_short0, s2);
                    rc = run_batch(&prob, integrator, opts.precision, topb.r, topb.n, d_sums2, d_part2,
                                   part2_bytes, nullptr, s2);
                    if (rc == LD_OK) (void)hipEventRecord(e_short, s2);
                    if (rc == LD_OK &&
                        (hipMemcpyAsync(h_top, d_sums2, topb.n * sizeof(ld_level_sums), hipMemcpyDeviceToHost,
                                        s2) != hipSuccess ||
                         hipStreamSynchronize(s2) != hipSuccess))
                        rc = fail(LD_EDEVICE, "level sums failed (early top-up)");
                    if (rc == LD_OK) s2_span();
                }
            }
            if (rc == LD_OK &&
                (hipMemcpyAsync(h_long, d_sums, longb.n * sizeof(ld_level_sums), hipMemcpyDeviceToHost, stream) !=
                     hipSuccess ||
                 hipStreamSynchronize(stream) != hipSuccess || hipStreamSynchronize(s2) != hipSuccess))
                rc = fail(LD_EDEVICE, "level sums failed (long levels)");
            if (rc == LD_OK) {
                for (int32_t j = 0; j < longb.n; ++j) {
                    merge_into(sums[longb.r[j].level], h_long[j]);
                    drawn[longb.r[j].level] += longb.r[j].n_samples;
                }
                for (int32_t j = 0; j < topb.n; ++j) {
                    merge_into(sums[topb.r[j].level], h_top[j]);
                    drawn[topb.r[j].level] += topb.r[j].n_samples;
                }
                out->launches += topb.n > 0 ? 3 : 2;
                {   // kernel time of both streams, summed as for one stream
                    float a = 0.f;
                    if (hipEventElapsedTime(&a, ev0, e_long) == hipSuccess) device_s += a * 1e-3;
                    device_s += s2_seconds;
                }
                std::memset(dn, 0, sizeof dn);               // the loop below starts by planning
            }
        }
        if (rc != LD_OK) {   // work already queued may still use the workspace
            (void)hipStreamSynchronize(stream);
            (void)hipStreamSynchronize(s2);
        }
    }
    for (;;) {
        if (rc != LD_OK) break;
        ld_level_range ranges[LD_MAX_LEVELS];
        int32_t nr = 0;
        for (int32_t l = 0; l <= pin.L; ++l) {
            if (dn[l] == 0) continue;
            ranges[nr].level = l;
            ranges[nr].reserved = 0;
            ranges[nr].sample_begin = drawn[l];
            ranges[nr].n_samples = dn[l];
            ++nr;
        }
        if (nr > 0) {
            (void)hipEventRecord(ev0, stream);
            rc = run_batch(&prob, integrator, opts.precision, ranges, nr, d_sums, d_partials,
                           partial_bytes, nullptr, stream);
            if (rc != LD_OK) break;
            (void)hipEventRecord(ev1, stream);
            if (hipMemcpyAsync(host_batch, d_sums, nr * sizeof(ld_level_sums), hipMemcpyDeviceToHost,
                               stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess) {
                rc = fail(LD_EDEVICE, std::string("level sums failed: ") + hipGetErrorString(hipGetLastError()));
                break;
            }
            {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess) device_s += ms * 1e-3;
            }
            out->launches += 1;
            for (int32_t j = 0; j < nr; ++j) {
                merge_into(sums[ranges[j].level], host_batch[j]);
                drawn[ranges[j].level] += ranges[j].n_samples;
            }
        }
        for (int32_t l = 0; l <= pin.L; ++l) {
            pin.n[l] = sums[l].n;
            pin.sum1[l] = sums[l].s[0] + sums[l].c[0];
            pin.sum2[l] = sums[l].s[1] + sums[l].c[1];
        }
        mlmc_plan(&pin, &plan);
        ++iter;
        if (plan.status != 0 || iter >= max_iter) break;
        if (exceeds_budget(opts.max_fine_steps, opts.M0, drawn, plan.dn, plan.L)) break;
        pin.L = plan.L;
        std::memcpy(dn, plan.dn, sizeof dn);
    }
    if (own_ws) (void)hipFree(ws);
    if (rc != LD_OK) return rc;

    out->estimate = plan.estimate;
    out->eps_abs = plan.eps_abs;
    out->bias_est = plan.bias_est;
    out->stat_var = plan.stat_var;
    out->rmse_est = std::sqrt(plan.bias_est * plan.bias_est + plan.stat_var);
    out->alpha = plan.alpha;
    out->L = plan.L;
    out->iterations = iter;
    out->status = plan.status == 0 ? 2 : plan.status;
    for (int32_t l = 0; l <= plan.L; ++l) {
        out->N[l] = drawn[l];
        out->n_nonfinite += sums[l].bad;
        out->Yhat[l] = plan.Yhat[l];
        out->V[l] = plan.V[l];
        const double M = cost_of_level(opts.M0, l);
        out->fine_steps += (double)drawn[l] * M;
        out->integrator_steps += (double)drawn[l] * (l == 0 ? M : 1.5 * M);
    }
    out->device_seconds = device_s;
    out->wall_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    if (out->n_nonfinite > 0) return fail(LD_ENONFINITE, "some samples were non-finite");
    return out->status == 1 ? LD_OK : LD_WARN_NOT_CONVERGED;
}

}  // extern "C"
