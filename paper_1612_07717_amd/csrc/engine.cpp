// engine.cpp -- many MLMC estimates in one launch per iteration.
//
// Each active query owns a slot: its problem parameters and its running level sums
// (LD_MAX_LEVELS ld_level_sums) live in device memory for the query's lifetime.
// Submission touches no device: the problem waits in a pinned host table and goes up
// with the next iteration's tables, and a slot's level sums restart from zero at the
// merge of its first range. An iteration gathers every query's planned (level, range)
// pairs and plans each range's tiles with a rule that depends on the range alone; the
// range table goes up in one copy (with the new problems), and the device writes the
// tile table from it, runs the tiles of each queue present (profile kind, or adaptive
// symplectic Euler) - one block per tile, or persistent blocks taking tiles from the
// queue's counter when the iteration is a captured graph (use_graph) - and merges each
// range's partials into the running sums. The running sums of the
// touched slots come back and each query's planner (mlmc_plan, Sec. 3.3 / Sec. 6)
// decides its next samples; converged queries leave, new ones are admitted between
// iterations (continuous batching).
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

double now_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Query {
    bool used = false;
    bool done = false;
    int64_t handle = -1;
    ld_query q;
    ld_problem prob;
    KProblem kp;
    int32_t L = 0;
    uint64_t drawn[LD_MAX_LEVELS];
    uint64_t dn[LD_MAX_LEVELS];
    ld_plan_out plan;
    int32_t iterations = 0;
    int status = LD_PENDING;
    double t_submit = 0, t_done = 0;
    uint32_t fresh_levels = 0;   // levels whose running sums no range has reached yet
    ld_level_sums sums[LD_MAX_LEVELS];
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct ld_engine {
    ld_engine_opts opts;
    int device = 0;
    int n_cu = 256;
    uint32_t grid = 0;
    int32_t slots = 0;
    uint64_t max_tiles = 0;
    uint32_t max_ranges = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* d_base = nullptr;
    KProblem* d_problems = nullptr;
    ld_level_sums* d_running = nullptr;
    KHeader* d_hdr = nullptr;
    uint32_t* d_counters = nullptr;
    KRange* d_ranges = nullptr;
    ld_level_sums* d_range_out = nullptr;
    KTile* d_tiles = nullptr;
    ld_level_sums* d_partials = nullptr;
    KHeader* h_hdr = nullptr;              // pinned: the header, then the ranges at rng_off,
    KRange* h_ranges = nullptr;            // laid out as d_hdr and d_ranges (one upload)
    size_t rng_off = 0;
    KProblem* h_problems = nullptr;        // pinned copy of every slot's problem
    int32_t new_lo = 0, new_hi = -1;       // slots whose problems await upload
    ld_level_sums* h_running = nullptr;    // pinned, coherent: the range merge writes it
    ld_level_sums* h_running_dev = nullptr;   // its address on the device
    hipGraphExec_t graph[1 << kNumQueues] = {};   // by queue mask
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<Query> q;        // by slot
    int64_t next_handle = 0;
    double device_seconds = 0.0;
    int64_t iterations = 0;
    double fine_steps = 0.0;
};

namespace ldm {

int validate_query(const ld_query* qq) {
    if (qq == nullptr) return fail(LD_EINVAL, "query is NULL");
    int rc = validate_problem(&qq->problem);
    if (rc != LD_OK) return rc;
    if (qq->integrator != LD_SE && qq->integrator != LD_GL && qq->integrator != LD_BAOAB)
        return fail(LD_EINVAL, "unknown integrator");
    if (!(qq->eps > 0.0) || !std::isfinite(qq->eps)) return fail(LD_EINVAL, "eps must be positive");
    const int32_t L0 = qq->fixed_L >= 0 ? qq->fixed_L : qq->L_min;
    if (L0 < 0 || L0 >= LD_MAX_LEVELS || qq->L_max < L0 || qq->L_max >= LD_MAX_LEVELS)
        return fail(LD_EINVAL, "need 0 <= L_min <= L_max < LD_MAX_LEVELS");
    if (qq->N_init < 2) return fail(LD_EINVAL, "N_init must be >= 2");
    if (!(qq->max_fine_steps >= 0.0)) return fail(LD_EINVAL, "max_fine_steps must be >= 0");
    if (qq->problem.x_adapt > 0.0 && std::ldexp((double)qq->problem.M0, qq->L_max) > 67108864.0)
        return fail(LD_EINVAL, "adaptive steps need M0 * 2^L_max <= 2^26");
    if (std::ldexp((double)qq->problem.M0, qq->L_max) > 2147483648.0)
        return fail(LD_EINVAL, "M0 * 2^L_max must not exceed 2^31");
    return check_stability(&qq->problem, qq->integrator, 0);
}

}  // namespace ldm

namespace {

void release_resources(ld_engine* e) {
    for (hipGraphExec_t g : e->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    if (e->d_base) (void)hipFree(e->d_base);
    if (e->h_hdr) (void)hipHostFree(e->h_hdr);
    if (e->h_problems) (void)hipHostFree(e->h_problems);
    if (e->h_running) (void)hipHostFree(e->h_running);
    if (e->own_stream && e->stream) (void)hipStreamDestroy(e->stream);
}

// STREAM tiles of a range: 256 lanes x spl samples each. Adaptive symplectic Euler takes
// the level kernel's plan for its precision (one resident round of blocks), so its tiles
// are that kernel's blocks and a query's sums are the same bit for bit.
void stream_tiles(const ld_engine* e, const Query& qu, uint64_t n, uint32_t* spl, uint32_t* nb) {
    if (qu.kp.adaptive) {
        plan_item(n, spl, nb, e->opts.precision == LD_FP32 ? kAdaptiveTargetBlocksFp32 : kAdaptiveTargetBlocksFp64);
        return;
    }
    const uint64_t per = (uint64_t)kBlock;
    const uint64_t T = std::max<uint64_t>(1, e->opts.target_tiles);
    const uint64_t s = (n > per * T) ? (n + per * T - 1) / (per * T) : 1;
    *spl = (uint32_t)s;
    *nb = (uint32_t)((n + per * s - 1) / (per * s));
}

// How a range is cut into tiles (the rule depends on the range alone): its mode, samples
// per lane and tile count.
uint64_t plan_range(const ld_engine* e, const Query& qu, int32_t level, uint64_t n, uint16_t* mode,
                    uint32_t* spl) {
    const uint64_t M = (uint64_t)qu.prob.M0 << level;
    if (level >= 1 && n <= e->opts.pipe_max_samples && M >= e->opts.pipe_min_steps && !qu.kp.adaptive) {
        *mode = KMODE_PIPE;
        *spl = 1;
        return (n + 63) / 64;
    }
    uint32_t nb = 0;
    stream_tiles(e, qu, n, spl, &nb);
    *mode = KMODE_STREAM;
    return nb;
}

// One graph per set of profiles present (the persistent kernel of a profile without
// tiles is left out rather than launched empty).
int capture_graph(ld_engine* e, uint32_t mask) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(LD_EDEVICE, "hipStreamBeginCapture failed");
    const uint32_t grids[kNumQueues] = {e->grid, e->grid, e->grid};
    int rc = launch_engine_iteration(e->opts.precision, true, grids, mask, e->d_hdr, e->d_tiles, e->d_problems,
                                     e->d_partials, e->d_counters, e->d_ranges, e->d_running,
                                     e->d_range_out, e->h_running_dev, e->stream);
    const hipError_t ec = hipStreamEndCapture(e->stream, &g);
    if (rc != LD_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LD_EDEVICE, "graph capture failed");
    }
    const hipError_t ei = hipGraphInstantiate(&e->graph[mask], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(LD_EDEVICE, "hipGraphInstantiate failed");
    return LD_OK;
}

void finish_query(Query& qu, int plan_status) {
    qu.done = true;
    qu.t_done = now_seconds();
    if (plan_status == 1)
        qu.status = LD_OK;
    else
        qu.status = LD_WARN_NOT_CONVERGED;
    uint64_t bad = 0;
    for (int32_t l = 0; l <= qu.plan.L && l < LD_MAX_LEVELS; ++l) bad += qu.sums[l].n_nonfinite;
    if (bad > 0) qu.status = LD_ENONFINITE;
}

}  // namespace

extern "C" {

void ld_engine_default_opts(ld_engine_opts* o) {
    if (o == nullptr) return;
    std::memset(o, 0, sizeof *o);
    o->precision = LD_FP32;
    o->max_queries = 256;
    o->hbm_budget_bytes = (size_t)1 << 30;
    o->blocks_per_cu = 8;
    o->target_tiles = 32768;
    o->pipe_max_samples = kPipeMaxSamples;
    o->pipe_min_steps = kPipeMinSteps;
    o->use_graph = 0;
    o->hip_stream = nullptr;
}

int ld_engine_create(const ld_engine_opts* opts_in, ld_engine** out) {
    if (out == nullptr) return fail(LD_EINVAL, "out is NULL");
    *out = nullptr;
    ld_engine_opts o;
    if (opts_in)
        o = *opts_in;
    else
        ld_engine_default_opts(&o);
    if (o.precision != LD_FP32 && o.precision != LD_FP64) return fail(LD_EINVAL, "unknown precision");
    if (o.max_queries < 1 || o.blocks_per_cu < 1 || o.blocks_per_cu > 64 || o.target_tiles < 1)
        return fail(LD_EINVAL, "invalid engine options");
    ld_engine* e = new ld_engine();
    e->opts = o;
    if (hipGetDevice(&e->device) != hipSuccess) {
        delete e;
        return fail(LD_ENODEVICE, "no HIP device");
    }
    (void)hipDeviceGetAttribute(&e->n_cu, hipDeviceAttributeMultiprocessorCount, e->device);
    e->grid = (uint32_t)(o.blocks_per_cu * std::max(1, e->n_cu));
    // memory: fixed per-slot parts, then tiles fill the rest of the budget
    const size_t per_slot = sizeof(KProblem) + LD_MAX_LEVELS * sizeof(ld_level_sums) +
                            LD_MAX_LEVELS * (sizeof(KRange) + sizeof(ld_level_sums));
    const size_t fixed = 4096;
    const size_t min_tiles = 4096;
    const size_t per_tile = sizeof(KTile) + sizeof(ld_level_sums);
    if (o.hbm_budget_bytes < fixed + per_slot + min_tiles * per_tile) {
        delete e;
        return fail(LD_ENOMEM, "hbm_budget_bytes cannot hold one query");
    }
    size_t slots = (size_t)o.max_queries;
    // at most half of the budget for slots, the rest for tiles
    while (slots > 1 && fixed + slots * per_slot > o.hbm_budget_bytes / 2) slots /= 2;
    e->slots = (int32_t)slots;
    e->max_ranges = (uint32_t)(slots * LD_MAX_LEVELS);
    e->max_tiles = (o.hbm_budget_bytes - fixed - slots * per_slot) / per_tile;
    e->max_tiles = std::min<uint64_t>(e->max_tiles, (uint64_t)1 << 31);
    size_t off = 0;
    // the header and the range table back to back, as in the pinned staging: one upload
    const size_t o_hdr = off; off = align_up(off + sizeof(KHeader), 256);
    const size_t o_rng = off; off = align_up(off + e->max_ranges * sizeof(KRange), 256);
    const size_t o_cnt = off; off = align_up(off + 64, 256);
    const size_t o_prob = off; off = align_up(off + slots * sizeof(KProblem), 256);
    const size_t o_run = off; off = align_up(off + slots * LD_MAX_LEVELS * sizeof(ld_level_sums), 256);
    const size_t o_rout = off; off = align_up(off + e->max_ranges * sizeof(ld_level_sums), 256);
    const size_t o_tile = off; off = align_up(off + e->max_tiles * sizeof(KTile), 256);
    const size_t o_part = off; off = align_up(off + e->max_tiles * sizeof(ld_level_sums), 256);
    if (hipMalloc(&e->d_base, off) != hipSuccess) {
        delete e;
        return fail(LD_ENOMEM, "hipMalloc of the engine buffers failed");
    }
    char* b = (char*)e->d_base;
    e->d_hdr = (KHeader*)(b + o_hdr);
    e->d_counters = (uint32_t*)(b + o_cnt);
    e->d_problems = (KProblem*)(b + o_prob);
    e->d_running = (ld_level_sums*)(b + o_run);
    e->d_ranges = (KRange*)(b + o_rng);
    e->d_range_out = (ld_level_sums*)(b + o_rout);
    e->d_tiles = (KTile*)(b + o_tile);
    e->d_partials = (ld_level_sums*)(b + o_part);
    e->rng_off = o_rng - o_hdr;
    if (hipHostMalloc((void**)&e->h_hdr, e->rng_off + e->max_ranges * sizeof(KRange)) != hipSuccess ||
        hipHostMalloc((void**)&e->h_running, slots * LD_MAX_LEVELS * sizeof(ld_level_sums),
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void**)&e->h_running_dev, e->h_running, 0) != hipSuccess ||
        hipHostMalloc((void**)&e->h_problems, slots * sizeof(KProblem)) != hipSuccess) {
        release_resources(e);
        delete e;
        return fail(LD_ENOMEM, "pinned host staging allocation failed");
    }
    e->h_ranges = (KRange*)((char*)e->h_hdr + e->rng_off);
    std::memset(e->h_problems, 0, slots * sizeof(KProblem));
    std::memset(e->h_running, 0, slots * LD_MAX_LEVELS * sizeof(ld_level_sums));
    if (o.hip_stream != nullptr) {
        e->stream = (hipStream_t)o.hip_stream;
    } else {
        if (hipStreamCreate(&e->stream) != hipSuccess) {
            release_resources(e);
            delete e;
            return fail(LD_EDEVICE, "hipStreamCreate failed");
        }
        e->own_stream = true;
    }
    if (hipEventCreate(&e->ev0) != hipSuccess || hipEventCreate(&e->ev1) != hipSuccess) {
        release_resources(e);
        delete e;
        return fail(LD_EDEVICE, "hipEventCreate failed");
    }
    e->q.resize(slots);
    if (launch_clear_sums(e->d_running, (uint32_t)(slots * LD_MAX_LEVELS), e->stream) != LD_OK ||
        launch_reset_counters(e->d_counters, e->stream) != LD_OK ||
        hipStreamSynchronize(e->stream) != hipSuccess) {
        release_resources(e);
        delete e;
        return fail(LD_EDEVICE, "clearing the running sums failed");
    }
    *out = e;
    return LD_OK;
}

void ld_engine_destroy(ld_engine* e) {
    if (e == nullptr) return;
    if (e->stream) (void)hipStreamSynchronize(e->stream);
    release_resources(e);
    delete e;
}

int ld_engine_submit(ld_engine* e, const ld_query* qq, int64_t* handle) {
    if (e == nullptr || handle == nullptr) return fail(LD_EINVAL, "NULL argument");
    int rc = validate_query(qq);
    if (rc != LD_OK) return rc;
    int32_t slot = -1;
    for (int32_t s = 0; s < e->slots; ++s)
        if (!e->q[s].used) {
            slot = s;
            break;
        }
    if (slot < 0) return fail(LD_EBUSY, "no free query slot within the HBM budget");
    Query& qu = e->q[slot];
    qu = Query();
    qu.used = true;
    qu.handle = e->next_handle++;
    qu.q = *qq;
    qu.prob = qq->problem;
    rc = make_kproblem(&qu.prob, qq->integrator, &qu.kp);
    if (rc != LD_OK) {
        qu.used = false;
        return rc;
    }
    qu.L = qq->fixed_L >= 0 ? qq->fixed_L : qq->L_min;
    std::memset(qu.drawn, 0, sizeof qu.drawn);
    std::memset(qu.dn, 0, sizeof qu.dn);
    std::memset(qu.sums, 0, sizeof qu.sums);
    std::memset(&qu.plan, 0, sizeof qu.plan);
    for (int32_t l = 0; l <= qu.L; ++l) qu.dn[l] = qq->N_init;
    qu.fresh_levels = ~0u;
    qu.t_submit = now_seconds();
    // no device work here: the problem goes up with the next iteration's tables (the
    // previous iteration's copies from this staging have completed)
    e->h_problems[slot] = qu.kp;
    e->new_lo = (e->new_hi < 0) ? slot : std::min(e->new_lo, slot);
    e->new_hi = std::max(e->new_hi, slot);
    *handle = qu.handle;
    return LD_OK;
}

int ld_engine_step(ld_engine* e, int32_t* n_active) {
    if (e == nullptr) return fail(LD_EINVAL, "engine is NULL");
    // 1. ranges of every active query, most expensive paths first
    struct Pending {
        int32_t slot, level;
        uint64_t begin, n;
    };
    std::vector<Pending> pend;
    for (int32_t s = 0; s < e->slots; ++s) {
        Query& qu = e->q[s];
        if (!qu.used || qu.done) continue;
        for (int32_t l = 0; l <= qu.L; ++l)
            if (qu.dn[l] > 0) pend.push_back({s, l, qu.drawn[l], qu.dn[l]});
    }
    if (pend.empty()) {
        if (n_active) *n_active = 0;
        return LD_OK;
    }
    auto steps_of = [&](const Pending& p) { return (double)((uint64_t)e->q[p.slot].prob.M0 << p.level); };
    std::stable_sort(pend.begin(), pend.end(),
                     [&](const Pending& a, const Pending& b) { return steps_of(a) > steps_of(b); });
    const double top = steps_of(pend.front());
    // 2. the ranges that fit, grouped by queue (profile kind, or adaptive SE); ranges
    //    that do not fit wait for the next iteration
    struct Taken {
        Pending p;
        int qi;
        uint64_t nt;
        uint16_t prio;
    };
    std::vector<Taken> taken;
    uint64_t count[kNumQueues] = {0, 0, 0};
    uint64_t total = 0;
    for (const Pending& p : pend) {
        const Query& qu = e->q[p.slot];
        uint16_t mode;
        uint32_t spl;
        const uint64_t nt = plan_range(e, qu, p.level, p.n, &mode, &spl);
        if (total + nt > e->max_tiles || taken.size() >= e->max_ranges) continue;
        const int qi = qu.kp.adaptive ? (int)KQUEUE_ADAPT : qu.kp.profile;
        const uint16_t prio = (uint16_t)std::max(0, 3 - (int)std::lround(std::log2(top / steps_of(p))));
        taken.push_back({p, qi, nt, prio});
        count[qi] += nt;
        total += nt;
    }
    if (total == 0) return fail(LD_ENOMEM, "a single range exceeds the engine's tile budget");
    int rc = LD_OK;
    // the queues one after the other in the tile table: neutral, homogeneous, adaptive;
    // the ranges go into the pinned staging and the device writes the tiles from them
    const int order[kNumQueues] = {KPROFILE_NEUTRAL, KPROFILE_HOMOGENEOUS, KQUEUE_ADAPT};
    std::memset(e->h_hdr, 0, sizeof(KHeader));
    uint32_t mask = 0;
    uint64_t first = 0;
    std::vector<Pending> pall;
    uint32_t nr = 0;
    for (int qi : order) {
        e->h_hdr->queue[qi] = KQueue{(uint32_t)first, (uint32_t)count[qi], (uint32_t)qi, 0};
        if (count[qi] > 0) mask |= 1u << qi;
        uint64_t cursor = first;
        for (const Taken& t : taken) {
            if (t.qi != qi) continue;
            Query& qu = e->q[t.p.slot];
            KRange& r = e->h_ranges[nr++];
            std::memset(&r, 0, sizeof r);
            r.slot = (uint32_t)t.p.slot;
            r.level = t.p.level;
            r.tile_begin = (uint32_t)cursor;
            r.n_tiles = (uint32_t)plan_range(e, qu, t.p.level, t.p.n, &r.mode, &r.spl);
            r.sample_begin = t.p.begin;
            r.n_samples = t.p.n;
            r.prio = t.prio;
            r.fresh = (qu.fresh_levels >> t.p.level) & 1u;
            cursor += r.n_tiles;
            pall.push_back(t.p);
        }
        first += count[qi];
    }
    e->h_hdr->n_ranges = nr;
    // 3. the tables of a small iteration go as the expand kernel's argument (no copy
    //    queued); larger ones, and captured graphs, upload new problems, then header and
    //    ranges, one copy each
    const int32_t n_new = e->new_hi >= 0 ? e->new_hi - e->new_lo + 1 : 0;
    const bool small = !e->opts.use_graph && nr <= (uint32_t)kInlineRanges && n_new <= kInlineProblems;
    KInline inl;
    if (small) {
        std::memset(&inl, 0, sizeof inl);
        inl.hdr = *e->h_hdr;
        inl.new_lo = (uint32_t)(n_new > 0 ? e->new_lo : 0);
        inl.n_new = (uint32_t)n_new;
        std::memcpy(inl.ranges, e->h_ranges, nr * sizeof(KRange));
        if (n_new > 0) std::memcpy(inl.problems, &e->h_problems[e->new_lo], (size_t)n_new * sizeof(KProblem));
    } else {
        if (n_new > 0 &&
            hipMemcpyAsync(&e->d_problems[e->new_lo], &e->h_problems[e->new_lo], (size_t)n_new * sizeof(KProblem),
                           hipMemcpyHostToDevice, e->stream) != hipSuccess)
            return fail(LD_EDEVICE, "uploading the new problems failed");
        if (hipMemcpyAsync(e->d_hdr, e->h_hdr, e->rng_off + nr * sizeof(KRange), hipMemcpyHostToDevice,
                           e->stream) != hipSuccess)
            return fail(LD_EDEVICE, "uploading the tile tables failed");
    }
    e->new_lo = 0;
    e->new_hi = -1;
    if (e->opts.use_graph && e->graph[mask] == nullptr) {
        rc = capture_graph(e, mask);
        if (rc != LD_OK) return rc;
    }
    (void)hipEventRecord(e->ev0, e->stream);
    if (e->opts.use_graph) {
        if (hipGraphLaunch(e->graph[mask], e->stream) != hipSuccess)
            return fail(LD_EDEVICE, "hipGraphLaunch failed");
    } else {
        // no captured grid to keep: one block per tile, in tile order
        uint32_t grids[kNumQueues];
        for (int qi = 0; qi < kNumQueues; ++qi) grids[qi] = (uint32_t)std::max<uint64_t>(1, count[qi]);
        rc = launch_engine_iteration(e->opts.precision, false, grids, mask, e->d_hdr, e->d_tiles, e->d_problems,
                                         e->d_partials, e->d_counters, e->d_ranges, e->d_running,
                                         e->d_range_out, e->h_running_dev, e->stream, small ? &inl : nullptr);
        if (rc != LD_OK) return fail(rc, "engine launch failed");
    }
    (void)hipEventRecord(e->ev1, e->stream);
    // the range merge wrote every updated row into h_running as well
    const size_t row = LD_MAX_LEVELS * sizeof(ld_level_sums);
    if (hipStreamSynchronize(e->stream) != hipSuccess)
        return fail(LD_EDEVICE, std::string("engine iteration failed: ") + hipGetErrorString(hipGetLastError()));
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e->ev0, e->ev1) == hipSuccess) e->device_seconds += 1e-3 * ms;
    e->iterations += 1;
    // 4. plan the queries that ran
    std::vector<int32_t> ran;
    for (const Pending& p : pall) {
        Query& qu = e->q[p.slot];
        qu.drawn[p.level] += p.n;
        qu.dn[p.level] = 0;
        qu.fresh_levels &= ~(1u << p.level);
        e->fine_steps += (double)p.n * (double)((uint64_t)qu.prob.M0 << p.level);
        ran.push_back(p.slot);
    }
    std::sort(ran.begin(), ran.end());
    ran.erase(std::unique(ran.begin(), ran.end()), ran.end());
    for (int32_t s : ran) {
        Query& qu = e->q[s];
        bool waiting = false;
        for (int32_t l = 0; l <= qu.L; ++l)
            if (qu.dn[l] > 0) waiting = true;   // a range of this query did not fit: plan later
        if (waiting) continue;
        std::memcpy(qu.sums, &e->h_running[s * LD_MAX_LEVELS], row);
        ld_plan_in pin;
        std::memset(&pin, 0, sizeof pin);
        pin.L = qu.L;
        pin.M0 = qu.prob.M0;
        for (int32_t l = 0; l <= qu.L; ++l) {
            pin.n[l] = qu.sums[l].n;
            pin.sum1[l] = qu.sums[l].s[0] + qu.sums[l].c[0];
            pin.sum2[l] = qu.sums[l].s[1] + qu.sums[l].c[1];
        }
        pin.eps = qu.q.eps;
        pin.alpha = qu.q.alpha;
        pin.eps_is_relative = qu.q.eps_is_relative;
        pin.L_max = qu.q.L_max;
        pin.fixed_L = qu.q.fixed_L;
        pin.fixed_N = 0;
        pin.N_init = qu.q.N_init;
        mlmc_plan(&pin, &qu.plan);
        qu.iterations += 1;
        const int max_iter = qu.q.max_iter > 0 ? qu.q.max_iter : 100;
        if (qu.plan.status != 0 || qu.iterations >= max_iter ||
            exceeds_budget(qu.q.max_fine_steps, qu.prob.M0, qu.drawn, qu.plan.dn, qu.plan.L)) {
            finish_query(qu, qu.plan.status);
        } else {
            qu.L = qu.plan.L;
            std::memcpy(qu.dn, qu.plan.dn, sizeof qu.dn);
        }
    }
    int32_t active = 0;
    for (int32_t s = 0; s < e->slots; ++s)
        if (e->q[s].used && !e->q[s].done) ++active;
    if (n_active) *n_active = active;
    return LD_OK;
}

int ld_engine_result(ld_engine* e, int64_t handle, ld_estimate_result* out) {
    if (e == nullptr || out == nullptr) return fail(LD_EINVAL, "NULL argument");
    for (int32_t s = 0; s < e->slots; ++s) {
        const Query& qu = e->q[s];
        if (!qu.used || qu.handle != handle) continue;
        if (!qu.done) return LD_PENDING;
        std::memset(out, 0, sizeof *out);
        const ld_plan_out& p = qu.plan;
        out->estimate = p.estimate;
        out->eps_abs = p.eps_abs;
        out->bias_est = p.bias_est;
        out->stat_var = p.stat_var;
        out->rmse_est = std::sqrt(p.bias_est * p.bias_est + p.stat_var);
        out->alpha = p.alpha;
        out->L = p.L;
        out->iterations = qu.iterations;
        out->status = p.status == 0 ? 2 : p.status;
        for (int32_t l = 0; l <= p.L; ++l) {
            out->N[l] = qu.drawn[l];
            out->n_nonfinite += qu.sums[l].n_nonfinite;
            out->Yhat[l] = p.Yhat[l];
            out->V[l] = p.V[l];
            const double M = std::ldexp((double)qu.prob.M0, l);
            out->fine_steps += (double)qu.drawn[l] * M;
            out->integrator_steps += (double)qu.drawn[l] * (l == 0 ? M : 1.5 * M);
        }
        out->wall_seconds = qu.t_done - qu.t_submit;
        out->launches = qu.iterations;
        return qu.status;
    }
    return fail(LD_EINVAL, "unknown query handle");
}

int ld_engine_release(ld_engine* e, int64_t handle) {
    if (e == nullptr) return fail(LD_EINVAL, "engine is NULL");
    for (int32_t s = 0; s < e->slots; ++s) {
        Query& qu = e->q[s];
        if (qu.used && qu.handle == handle) {
            qu.used = false;
            return LD_OK;
        }
    }
    return fail(LD_EINVAL, "unknown query handle");
}

int ld_engine_stats(ld_engine* e, double* device_seconds, int64_t* iterations, double* fine_steps) {
    if (e == nullptr) return fail(LD_EINVAL, "engine is NULL");
    if (device_seconds) *device_seconds = e->device_seconds;
    if (iterations) *iterations = e->iterations;
    if (fine_steps) *fine_steps = e->fine_steps;
    return LD_OK;
}

// Submits queries[0..n) to an engine as slots free up and steps it until every one has a
// result in out[]; releases each handle. Returns the worst status (an error, else a
// warning, else LD_OK). On an error the engine may still hold admitted queries.
static int run_to_completion(ld_engine* e, const ld_query* queries, int32_t n, ld_estimate_result* out) {
    std::vector<int64_t> handle(n, -1);
    std::vector<bool> got(n, false);
    int32_t next = 0, remaining = n;
    int worst = LD_OK;
    while (remaining > 0) {
        while (next < n) {
            int64_t h;
            const int s = ld_engine_submit(e, &queries[next], &h);
            if (s == LD_EBUSY) break;
            if (s != LD_OK) return s;
            handle[next++] = h;
        }
        int32_t active = 0;
        const int rc = ld_engine_step(e, &active);
        if (rc != LD_OK) return rc;
        for (int32_t i = 0; i < next; ++i) {
            if (got[i]) continue;
            const int s = ld_engine_result(e, handle[i], &out[i]);
            if (s == LD_PENDING) continue;
            got[i] = true;
            --remaining;
            (void)ld_engine_release(e, handle[i]);
            if (s < 0 && (worst >= 0 || s < worst)) worst = s;
            if (s > 0 && worst == LD_OK) worst = s;
        }
    }
    return worst;
}

int ld_engine_run(ld_engine* e, const ld_query* queries, int32_t n, ld_estimate_result* out) {
    if (e == nullptr) return fail(LD_EINVAL, "engine is NULL");
    if (queries == nullptr || out == nullptr || n < 1) return fail(LD_EINVAL, "need n >= 1 queries");
    for (int32_t i = 0; i < n; ++i) {
        const int rc = validate_query(&queries[i]);
        if (rc != LD_OK) return rc;
    }
    return run_to_completion(e, queries, n, out);
}

int mlmc_estimate_batch(const ld_query* queries, int32_t n, const ld_engine_opts* opts,
                        ld_estimate_result* out) {
    if (queries == nullptr || out == nullptr || n < 1) return fail(LD_EINVAL, "need n >= 1 queries");
    for (int32_t i = 0; i < n; ++i) {
        const int rc = validate_query(&queries[i]);
        if (rc != LD_OK) return rc;
    }
    ld_engine* e = nullptr;
    const int rc = ld_engine_create(opts, &e);
    if (rc != LD_OK) return rc;
    const int r = run_to_completion(e, queries, n, out);
    ld_engine_destroy(e);
    return r;
}

int ld_engine_autotune(const ld_query* queries, int32_t n, const ld_engine_opts* base, int32_t reps,
                       ld_engine_opts* best, double* best_seconds) {
    if (queries == nullptr || n < 1 || best == nullptr) return fail(LD_EINVAL, "invalid autotune arguments");
    ld_engine_opts b;
    if (base)
        b = *base;
    else
        ld_engine_default_opts(&b);
    const int32_t grids[] = {2, 4, 6, 8, 12, 16};
    const uint64_t tiles[] = {4096, 8192, 16384, 32768, 65536};
    const uint64_t pipes[] = {0, kPipeMaxSamples};
    const int32_t graphs[] = {0, 1};
    std::vector<ld_estimate_result> res(n);
    double best_t = 1e300;
    ld_engine_opts best_o = b;
    reps = std::max(1, reps);
    for (int32_t g : grids)
        for (uint64_t t : tiles)
            for (uint64_t pm : pipes)
                for (int32_t ug : graphs) {
                    ld_engine_opts o = b;
                    o.blocks_per_cu = g;
                    o.target_tiles = t;
                    o.pipe_max_samples = pm;
                    o.use_graph = ug;
                    // one engine per configuration, so that its allocation stays out of the
                    // timings (as for a server, which keeps its engine)
                    ld_engine* e = nullptr;
                    int rc = ld_engine_create(&o, &e);
                    if (rc != LD_OK) return rc;
                    std::vector<double> times;
                    for (int32_t r = 0; r < reps; ++r) {
                        const double t0 = now_seconds();
                        rc = run_to_completion(e, queries, n, res.data());
                        if (rc < 0 && rc != LD_ENONFINITE) {
                            ld_engine_destroy(e);
                            return rc;
                        }
                        times.push_back(now_seconds() - t0);
                    }
                    ld_engine_destroy(e);
                    std::sort(times.begin(), times.end());
                    const double med = times[times.size() / 2];
                    if (med < best_t) {
                        best_t = med;
                        best_o = o;
                    }
                }
    *best = best_o;
    if (best_seconds) *best_seconds = best_t;
    return LD_OK;
}

}  // extern "C"
