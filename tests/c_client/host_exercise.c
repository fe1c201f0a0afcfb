/* A C client that drives every host-side subsystem of libldmlmc through the C ABI on
 * the GPU: the MLMC driver in both path precisions and both schedules, the engine (its
 * own API and mlmc_estimate_batch), the request server in both policies, and the
 * binned-concentration estimator (MLMC and StMC). Neutral boundary layer as in
 * estimate.c, loose tolerances so the whole run takes well under a second of device
 * time. It is built with AddressSanitizer and UndefinedBehaviorSanitizer against a
 * library whose host code carries them too; it exits non-zero on any error status or
 * broken invariant, and the sanitizers end it on any report.
 *
 *   host_exercise
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ldmlmc.h"

static int failures = 0;

static void check(int ok, const char* what) {
    if (!ok) {
        fprintf(stderr, "FAILED: %s (%s)\n", what, ld_last_error());
        ++failures;
    }
}

static ld_profile neutral(void) {
    ld_profile p;
    memset(&p, 0, sizeof p);
    p.kind = LD_PROFILE_NEUTRAL_BL;
    p.H = 1000.0;
    p.kappa_sigma = 1.3;
    p.kappa_tau = 0.5;
    p.u_star = 0.2;
    p.eps_reg = 10.0;
    return p;
}

static ld_query query(double z0, ld_integrator integ, double eps, uint64_t seed) {
    ld_query q;
    memset(&q, 0, sizeof q);
    q.problem.profile = neutral();
    q.problem.release.kind = LD_RELEASE_GAUSSIAN_W;
    q.problem.release.z0 = z0;
    q.problem.qoi.kind = LD_QOI_MEAN_Z;
    q.problem.T = 1000.0;
    q.problem.M0 = 40;
    q.problem.seed = seed;
    q.integrator = integ;
    q.eps_is_relative = 1;
    q.eps = eps;
    q.L_min = 2;
    q.L_max = 8;
    q.fixed_L = -1;
    q.max_iter = 100;
    q.N_init = 1000;
    q.alpha = 1.0;
    return q;
}

static void driver(void) {
    const ld_profile prof = neutral();
    ld_qoi qoi;
    memset(&qoi, 0, sizeof qoi);
    qoi.kind = LD_QOI_MEAN_Z;
    for (int prec = 0; prec < 2; ++prec) {
        for (int early = 0; early < 2; ++early) {
            ld_estimate_opts o;
            mlmc_estimate_default_opts(&o);
            o.release.kind = LD_RELEASE_GAUSSIAN_W;
            o.release.z0 = 500.0;
            o.T = 1000.0;
            o.M0 = 8;
            o.eps_is_relative = 1;
            o.N_init = 2000;
            o.L_min = early ? 6 : 2;
            o.L_max = 8;
            o.early_topup = early;
            o.precision = prec ? LD_FP32 : LD_FP64;
            ld_estimate_result r;
            memset(&r, 0, sizeof r);
            const int rc = mlmc_estimate(1e-2, &qoi, LD_BAOAB, &prof, &o, &r);
            check(rc == LD_OK, "mlmc_estimate");
            check(r.estimate > 400.0 && r.estimate < 560.0, "mlmc_estimate value");
            printf("estimate prec=%d early=%d: %.6f L=%d launches=%d\n", prec, early, r.estimate, r.L,
                   r.launches);
        }
    }
}

enum { NQ = 6 };

static void engine(void) {
    ld_query qs[NQ];
    const ld_integrator integ[3] = {LD_SE, LD_GL, LD_BAOAB};
    for (int i = 0; i < NQ; ++i) qs[i] = query(150.0 + 120.0 * i, integ[i % 3], 1e-2, 7 + i);
    ld_engine_opts eo;
    ld_engine_default_opts(&eo);
    eo.precision = LD_FP32;
    eo.max_queries = 4;                         /* fewer slots than queries: re-admission */
    ld_engine* e = NULL;
    check(ld_engine_create(&eo, &e) == LD_OK && e != NULL, "ld_engine_create");
    if (e == NULL) return;
    int64_t handle[NQ];
    ld_estimate_result res[NQ];
    memset(res, 0, sizeof res);
    int done[NQ] = {0}, submitted = 0, finished = 0;
    for (int it = 0; it < 400 && finished < NQ; ++it) {
        while (submitted < NQ) {
            const int rc = ld_engine_submit(e, &qs[submitted], &handle[submitted]);
            if (rc == LD_EBUSY) break;
            check(rc == LD_OK, "ld_engine_submit");
            if (rc != LD_OK) break;
            ++submitted;
        }
        int32_t active = 0;
        check(ld_engine_step(e, &active) == LD_OK, "ld_engine_step");
        for (int i = 0; i < submitted; ++i) {
            if (done[i]) continue;
            const int rc = ld_engine_result(e, handle[i], &res[i]);
            if (rc == LD_PENDING) continue;
            check(rc == LD_OK, "ld_engine_result");
            check(ld_engine_release(e, handle[i]) == LD_OK, "ld_engine_release");
            done[i] = 1;
            ++finished;
        }
    }
    check(finished == NQ, "engine finished every query");
    double dev = 0.0, steps = 0.0;
    int64_t iters = 0;
    check(ld_engine_stats(e, &dev, &iters, &steps) == LD_OK && iters > 0, "ld_engine_stats");
    ld_engine_destroy(e);
    ld_estimate_result batch[NQ];
    memset(batch, 0, sizeof batch);
    check(mlmc_estimate_batch(qs, NQ, &eo, batch) == LD_OK, "mlmc_estimate_batch");
    for (int i = 0; i < NQ; ++i)
        check(batch[i].estimate == res[i].estimate && batch[i].L == res[i].L,
              "batch equals engine, bit for bit");
    printf("engine: %d queries in %lld iterations, first estimate %.6f\n", NQ, (long long)iters,
           res[0].estimate);
}

static void server(int policy, ld_precision prec, int n) {
    ld_server_opts so;
    ld_server_default_opts(&so);
    so.policy = policy;
    so.engine.precision = prec;
    ld_server* s = NULL;
    check(ld_server_create(&so, &s) == LD_OK && s != NULL, "ld_server_create");
    if (s == NULL) return;
    int64_t tickets[16];
    for (int i = 0; i < n; ++i) {
        const ld_query q = query(100.0 + 100.0 * i, i % 2 ? LD_BAOAB : LD_GL, 1e-2, 100 + i);
        check(ld_server_submit(s, &q, &tickets[i]) == LD_OK, "ld_server_submit");
    }
    for (int i = 0; i < n; ++i) {
        ld_estimate_result r;
        ld_request_times t;
        memset(&t, 0, sizeof t);
        check(ld_server_wait(s, tickets[i], 120.0, &r, &t) == LD_OK, "ld_server_wait");
        check(t.t_done >= t.t_admit && t.t_admit >= t.t_submit, "request times ordered");
    }
    ld_server_stats st;
    memset(&st, 0, sizeof st);
    check(ld_server_stats_get(s, &st) == LD_OK && st.completed == n, "ld_server_stats_get");
    ld_server_destroy(s);
    printf("server policy=%d: %lld completed in %lld iterations\n", policy, (long long)st.completed,
           (long long)st.iterations);
}

static void pdf(void) {
    const ld_profile prof = neutral();
    ld_qoi qoi;
    memset(&qoi, 0, sizeof qoi);
    qoi.kind = LD_QOI_P_BOX;
    qoi.r = 4;
    qoi.delta = 100.0;
    ld_bins bins;
    memset(&bins, 0, sizeof bins);
    bins.a0 = 0.0;
    bins.width = 50.0;
    bins.n_bins = 20;
    for (int est = 0; est < 2; ++est) {
        ld_estimate_opts o;
        mlmc_estimate_default_opts(&o);
        o.release.kind = LD_RELEASE_GAUSSIAN_W;
        o.release.z0 = 200.0;
        o.T = 1000.0;
        o.M0 = 40;
        o.N_init = 2000;
        o.L_max = 6;
        o.fixed_L = est ? 2 : -1;
        o.precision = LD_FP32;
        ld_pdf_result r;
        memset(&r, 0, sizeof r);
        const int rc = mlmc_estimate_pdf(5e-3, &bins, &qoi, LD_BAOAB, &prof, &o, est ? LD_STMC : LD_MLMC, &r);
        check(rc == LD_OK, "mlmc_estimate_pdf");
        double mass = 0.0;
        for (int i = 0; i < bins.n_bins; ++i) mass += r.estimate[i];
        check(mass > 0.8 && mass < 1.2, "p.d.f. mass near 1");
        printf("pdf estimator=%d: mass %.4f L=%d\n", est, mass, r.L);
    }
}

int main(void) {
    setvbuf(stdout, NULL, _IONBF, 0);   /* a sanitizer report at exit must not swallow it */
    driver();
    engine();
    server(LD_SERVE_BATCH, LD_FP32, 8);
    server(LD_SERVE_FIFO, LD_FP64, 3);
    pdf();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host exercise ok\n");
    return 0;
}
