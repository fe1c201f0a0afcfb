/*
 * oracle.c -- plain, slow, obviously correct CPU FP64 oracle of the MLMC
 * Lagrangian-dispersion hot path.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library. It shares no code with the GPU library.
 *
 * Paper: Katsiolides, Mueller, Scheichl, Shardlow, Giles, Thomson, "Multilevel Monte
 * Carlo and improved timestepping methods in atmospheric dispersion modelling",
 * arXiv:1612.07717. Equation numbers below are the paper's; each citation also names
 * the section and what the equation is, so it can be found if numbering differs.
 *
 * Everything is written in the paper's order and notation: one path at a time, one
 * step at a time, every coefficient re-evaluated from its definition, no blocking or
 * fusion. Parallelism (OpenMP) is only over independent samples; sums are merged in a
 * fixed order so results do not depend on the thread count.
 *
 * Readings where the paper is silent (listed with reasons in the design notes):
 *  - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by the
 *    seed, counter = (block, sample_lo, sample_hi, level | stream << 8); Box-Muller
 *    (Box & Muller 1958) turns one block into two normals;
 *  - reflection folds repeatedly until the position lies in [0, H] (the periodic
 *    extension of Sec. 4.1.1 implies this); 0 and H themselves are inside;
 *  - BAOAB folds after each A half-step, so every coefficient is evaluated in [0, H];
 *  - the sign S that multiplies a noise is the one in force when that noise enters
 *    the velocity (Eqs. 28-32), also for the coarse path;
 *  - the GL/BAOAB coupling weight uses lambda where the first fine O-step of the pair
 *    evaluated it (X_n for GL, X_{n+1/2} for BAOAB; Eq. 19 and the remark after it);
 *  - 1 - exp(-2 lambda h) is evaluated as -expm1(-2 lambda h) (same number, no
 *    cancellation);
 *  - inside the cut-off layers of Eq. (7) sigma_U is constant, so dsigma_U^2/dX = 0
 *    there and the well-mixed drift vanishes.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846
/* A fold needing more than this many reflections means the step ran away (a position
   many boundary-layer depths outside the domain); the sample is marked non-finite. */
#define ORACLE_FOLD_MAX 16
/* Reserved Philox blocks for the initial state. */
#define ORACLE_BLOCK_INIT_W 0xFFFFFFFFu
#define ORACLE_BLOCK_INIT_X 0xFFFFFFFEu
/* Samples per chunk of the fixed-order level reduction. */
#define ORACLE_CHUNK 1024

/* ================================================================================== */
/* Philox4x32-10: ten rounds of the Philox S-box on a 4x32-bit counter with a 2x32-bit */
/* key, the key advanced by the Weyl increments between rounds (Salmon et al., SC'11). */
/* ================================================================================== */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_block(const oracle_problem* p, int32_t level, uint64_t sample,
                         uint32_t block, uint32_t out[4]) {
    uint32_t ctr[4] = {block, (uint32_t)sample, (uint32_t)(sample >> 32),
                       ((uint32_t)level & 0xFFu) | (p->stream_id << 8)};
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* Uniform on the open interval (0, 1) from the top 52 bits of the 64-bit word hi:lo:
   (2m + 1) 2^-53 is exact in binary64 and never 0 or 1. */
static double uniform_open(uint32_t hi, uint32_t lo) {
    uint64_t m = (((uint64_t)hi << 32) | (uint64_t)lo) >> 12;
    return (double)(2u * m + 1u) * 0x1p-53;
}

void oracle_normals(const oracle_problem* p, int32_t level, uint64_t sample,
                    uint32_t block, double out[2]) {
    uint32_t r[4];
    philox_block(p, level, sample, block, r);
    double u = uniform_open(r[1], r[0]);
    double v = uniform_open(r[3], r[2]);
    double rho = sqrt(-2.0 * log(u));       /* Box-Muller */
    double theta = 2.0 * ORACLE_PI * v;
    out[0] = rho * cos(theta);
    out[1] = rho * sin(theta);
}

/* ================================================================================== */
/* Model: Sec. 2.                                                                      */
/* ================================================================================== */

/* Eq. (5) (neutral boundary-layer profiles) with the hard cut-off of Eq. (7). */
void oracle_profile(const oracle_problem* p, double x, double* sigma_u, double* tau) {
    if (p->profile_kind == ORACLE_PROFILE_HOMOGENEOUS) {
        *sigma_u = p->sigma_u;
        *tau = p->tau;
        return;
    }
    double xr = x;
    if (x < p->eps_reg) xr = p->eps_reg;
    if (x > p->H - p->eps_reg) xr = p->H - p->eps_reg;
    double su = p->kappa_sigma * p->u_star * pow(1.0 - xr / p->H, 0.75);
    *sigma_u = su;
    *tau = p->kappa_tau * xr / su;
}

/* d(sigma_U^2)/dX. From Eq. (5): sigma_U^2 = (kappa_sigma u_*)^2 (1 - X/H)^(3/2), so the
   derivative is -(3/2)(kappa_sigma u_*)^2 (1 - X/H)^(1/2) / H; it is zero where Eq. (7)
   freezes sigma_U. */
static double dsigma2_dx(const oracle_problem* p, double x) {
    if (p->profile_kind == ORACLE_PROFILE_HOMOGENEOUS) return 0.0;
    if (x < p->eps_reg || x > p->H - p->eps_reg) return 0.0;
    double ks = p->kappa_sigma * p->u_star;
    return -1.5 * ks * ks * sqrt(1.0 - x / p->H) / p->H;
}

/* V(X, U) = -1/2 [sigma_U^2 + U^2 log(sigma_U^2 / sigma_U^2(X_ref))] (after Eq. 3), so
   dV/dX = -1/2 [d sigma_U^2/dX + U^2 (d sigma_U^2/dX) / sigma_U^2]. */
double oracle_dVdX(const oracle_problem* p, double x, double u) {
    double su, tau;
    oracle_profile(p, x, &su, &tau);
    double d = dsigma2_dx(p, x);
    return -0.5 * (d + u * u * d / (su * su));
}

/* lambda = 1/tau and sigma = sqrt(2 sigma_U^2 / tau) (definitions after Eq. 3). */
static void coefficients(const oracle_problem* p, double x, double* lambda, double* sigma) {
    double su, tau;
    oracle_profile(p, x, &su, &tau);
    *lambda = 1.0 / tau;
    *sigma = sqrt(2.0 * su * su / tau);
}

/* Elastic reflection at 0 and H (Eq. 6 and the rule of Sec. 4): X -> -X or 2H - X,
   U -> -U, and the reflection count's sign S flips (Eq. 20). */
static int fold(double H, double* x, double* u, double* s) {
    int count = 0;
    while (*x < 0.0 || *x > H) {
        if (++count > ORACLE_FOLD_MAX) {
            *x = NAN;
            *u = NAN;
            return -1;
        }
        if (*x < 0.0)
            *x = -*x;
        else
            *x = 2.0 * H - *x;
        *u = -*u;
        *s = -*s;
    }
    return 0;
}

/* Physical noise entering now, and the extended-variable noise that it corresponds to. */
static double enter_noise(const oracle_problem* p, double sign, double xi,
                          int32_t noise_is_tilde, double* tilde) {
    double s = (p->coupling == ORACLE_COUPLING_NAIVE) ? 1.0 : sign;
    double physical = noise_is_tilde ? s * xi : xi;
    *tilde = s * physical;
    return physical;
}

/* Symplectic Euler, Eq. (8). */
static int step_se(const oracle_problem* p, double h, double st[3], double xi,
                   int32_t noise_is_tilde, double* tilde, double* lam_o) {
    double x = st[0], u = st[1], s = st[2];
    double lambda, sigma;
    coefficients(p, x, &lambda, &sigma);
    double noise = enter_noise(p, s, xi, noise_is_tilde, tilde);
    double u1 = (1.0 - lambda * h) * u - oracle_dVdX(p, x, u) * h + sigma * sqrt(h) * noise;
    double x1 = x + u1 * h;
    int rc = fold(p->H, &x1, &u1, &s);
    st[0] = x1; st[1] = u1; st[2] = s;
    *lam_o = lambda;
    return rc;
}

/* Geometric Langevin (OBA), Eq. (9). */
static int step_gl(const oracle_problem* p, double h, double st[3], double xi,
                   int32_t noise_is_tilde, double* tilde, double* lam_o) {
    double x = st[0], u = st[1], s = st[2];
    double lambda, sigma;
    coefficients(p, x, &lambda, &sigma);
    double noise = enter_noise(p, s, xi, noise_is_tilde, tilde);
    double ustar = exp(-lambda * h) * u +
                   sigma * sqrt(-expm1(-2.0 * lambda * h) / (2.0 * lambda)) * noise;  /* O */
    double u1 = ustar - oracle_dVdX(p, x, ustar) * h;                                /* B */
    double x1 = x + u1 * h;                                                          /* A */
    int rc = fold(p->H, &x1, &u1, &s);
    st[0] = x1; st[1] = u1; st[2] = s;
    *lam_o = lambda;
    return rc;
}

/* BAOAB, Eq. (10), folding after each A half-step. */
static int step_baoab(const oracle_problem* p, double h, double st[3], double xi,
                      int32_t noise_is_tilde, double* tilde, double* lam_o) {
    double x = st[0], u = st[1], s = st[2];
    int rc = 0;
    double uh = u - oracle_dVdX(p, x, u) * (h / 2.0);                                /* B */
    double xh = x + uh * (h / 2.0);                                                  /* A */
    rc |= fold(p->H, &xh, &uh, &s);
    double lambda, sigma;
    coefficients(p, xh, &lambda, &sigma);
    double noise = enter_noise(p, s, xi, noise_is_tilde, tilde);
    double ustar = exp(-lambda * h) * uh +
                   sigma * sqrt(-expm1(-2.0 * lambda * h) / (2.0 * lambda)) * noise;  /* O */
    double x1 = xh + ustar * (h / 2.0);                                              /* A */
    rc |= fold(p->H, &x1, &ustar, &s);
    double u1 = ustar - oracle_dVdX(p, x1, ustar) * (h / 2.0);                       /* B */
    st[0] = x1; st[1] = u1; st[2] = s;
    *lam_o = lambda;
    return rc;
}

int oracle_step(const oracle_problem* p, double h, double state[3], double xi,
                int32_t noise_is_tilde, double* tilde, double* lam_o) {
    int rc;
    switch (p->integrator) {
        case ORACLE_SE: rc = step_se(p, h, state, xi, noise_is_tilde, tilde, lam_o); break;
        case ORACLE_GL: rc = step_gl(p, h, state, xi, noise_is_tilde, tilde, lam_o); break;
        default: rc = step_baoab(p, h, state, xi, noise_is_tilde, tilde, lam_o); break;
    }
    if (!isfinite(state[0]) || !isfinite(state[1])) rc = -1;
    return rc;
}

/* ================================================================================== */
/* Quantities of interest: Sec. 2 and Sec. 5.                                          */
/* ================================================================================== */

/* p_r of Eq. (35): degree <= r + 1, p_r(-1) = 1, p_r(1) = 0, and
   int_{-1}^{1} s^j p_r(s) ds = (-1)^j / (j + 1) for j = 0 .. r - 1. The (r+2)x(r+2)
   system is solved by Gaussian elimination with partial pivoting in long double. */
int oracle_smoothing_poly(int32_t r, double* coef) {
    if (r < 1 || r > 8) return -1;
    int n = r + 2;
    long double a[10][11];
    for (int k = 0; k < n; ++k) {
        a[0][k] = (k % 2 == 0) ? 1.0L : -1.0L;          /* p(-1) = 1 */
        a[1][k] = 1.0L;                                  /* p(1) = 0 */
    }
    a[0][n] = 1.0L;
    a[1][n] = 0.0L;
    for (int j = 0; j < r; ++j) {
        for (int k = 0; k < n; ++k)   /* int_{-1}^{1} s^(j+k) ds */
            a[2 + j][k] = ((j + k) % 2 == 0) ? 2.0L / (long double)(j + k + 1) : 0.0L;
        a[2 + j][n] = ((j % 2 == 0) ? 1.0L : -1.0L) / (long double)(j + 1);
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int row = col + 1; row < n; ++row)
            if (fabsl(a[row][col]) > fabsl(a[piv][col])) piv = row;
        if (piv != col)
            for (int k = 0; k <= n; ++k) {
                long double t = a[col][k]; a[col][k] = a[piv][k]; a[piv][k] = t;
            }
        for (int row = 0; row < n; ++row) {
            if (row == col) continue;
            long double f = a[row][col] / a[col][col];
            for (int k = col; k <= n; ++k) a[row][k] -= f * a[col][k];
        }
    }
    for (int k = 0; k < n; ++k) coef[k] = (double)(a[k][n] / a[k][k]);
    return 0;
}

typedef struct {
    oracle_problem p;
    double coef[10];
    int ncoef;
} context;

static void make_context(const oracle_problem* p, context* ctx) {
    ctx->p = *p;
    ctx->ncoef = 0;
    if ((p->qoi_kind == ORACLE_QOI_P_ABOVE || p->qoi_kind == ORACLE_QOI_P_BOX) && p->r > 0) {
        oracle_smoothing_poly(p->r, ctx->coef);
        ctx->ncoef = p->r + 2;
    }
}

/* g_r of Eq. (35). */
static double g_r(const context* ctx, double s) {
    if (s < -1.0) return 1.0;
    if (s > 1.0) return 0.0;
    double v = 0.0;
    for (int k = ctx->ncoef - 1; k >= 0; --k) v = v * s + ctx->coef[k];
    return v;
}

/* theta of Eq. (34): 1 for X <= 0, else 0. */
static double theta(double s) { return s <= 0.0 ? 1.0 : 0.0; }

static double qoi(const context* ctx, double x, double u) {
    const oracle_problem* p = &ctx->p;
    switch (p->qoi_kind) {
        case ORACLE_QOI_MEAN_Z: return x;
        case ORACLE_QOI_VELOCITY: return u;
        case ORACLE_QOI_VELOCITY_SQ: return u * u;
        case ORACLE_QOI_P_ABOVE:
            if (p->r == 0) return 1.0 - theta(x - p->qa);
            return 1.0 - g_r(ctx, (x - p->qa) / p->delta);
        case ORACLE_QOI_P_BOX:   /* Eq. (34), smoothed as Eq. (37) */
            if (p->r == 0) return theta(x - p->qb) - theta(x - p->qa);
            return g_r(ctx, (x - p->qb) / p->delta) - g_r(ctx, (x - p->qa) / p->delta);
        default: return NAN;
    }
}

double oracle_qoi(const oracle_problem* p, double x, double u) {
    context ctx;
    make_context(p, &ctx);
    return qoi(&ctx, x, u);
}

/* ================================================================================== */
/* One coupled sample on level l (Sec. 3.3, Eqs. 14-19, with Eqs. 31-32).             */
/* ================================================================================== */

static void initial_state(const oracle_problem* p, int32_t level, uint64_t sample,
                          double* x0, double* u0) {
    double z[2];
    switch (p->release_kind) {
        case ORACLE_RELEASE_FIXED_W:
            *x0 = p->z0;
            *u0 = p->w0;
            return;
        case ORACLE_RELEASE_GAUSSIAN_W: {
            double su, tau;
            oracle_profile(p, p->z0, &su, &tau);
            oracle_normals(p, level, sample, ORACLE_BLOCK_INIT_W, z);
            *x0 = p->z0;
            *u0 = su * z[0];
            return;
        }
        default: {   /* well mixed: X_0 ~ U[0, H], U_0 ~ N(0, sigma_U(X_0)^2) (Sec. 2) */
            uint32_t r[4];
            philox_block(p, level, sample, ORACLE_BLOCK_INIT_X, r);
            *x0 = p->H * uniform_open(r[1], r[0]);
            double su, tau;
            oracle_profile(p, *x0, &su, &tau);
            oracle_normals(p, level, sample, ORACLE_BLOCK_INIT_W, z);
            *u0 = su * z[0];
            return;
        }
    }
}

/* ================================================================================== */
/* Adaptive, non-nested timesteps for symplectic Euler (Sec. 7).                        */
/* ================================================================================== */

/* Eq. (8) driven by the Brownian increment dW of the step (dW replaces sqrt(h) xi). */
static int step_se_dw(const oracle_problem* p, double h, double st[3], double dW) {
    double x = st[0], u = st[1], s = st[2];
    double lambda, sigma;
    coefficients(p, x, &lambda, &sigma);
    double u1 = (1.0 - lambda * h) * u - oracle_dVdX(p, x, u) * h + sigma * dW;
    double x1 = x + u1 * h;
    int rc = fold(p->H, &x1, &u1, &s);
    st[0] = x1; st[1] = u1; st[2] = s;
    return rc;
}

/* End (in ticks) of the step a path at x starts at tick t: base step `base` ticks,
   shortened to floor(lambda(X_adapt) / lambda(x) base) below the reference height. */
static uint64_t adaptive_end(const oracle_problem* p, double lam_adapt, double x, uint64_t t,
                             uint64_t base, uint64_t t_end) {
    double lambda, sigma;
    coefficients(p, x, &lambda, &sigma);
    double ratio = lam_adapt / lambda;
    uint64_t k = base;
    if (ratio < 1.0) {                          /* also false for a NaN state */
        k = (uint64_t)floor(ratio * (double)base);
        if (k < 1) k = 1;
    }
    return (t + k < t_end) ? t + k : t_end;
}

/* One coupled sample with adaptive steps. The merged time grid tau_j is the union of
   the fine and the coarse time points; interval j gets xi_j (draw j mod 2 of Philox block
   j / 2, as the uniform scheme's step j). The fine path's increment over its step is the
   sum of xi_j sqrt(tau_{j+1} - tau_j) over the intervals it covers; the coarse path's is
   S^(c) times the sum of S_j^(f) xi_j sqrt(tau_{j+1} - tau_j) (Eq. for the adaptive Euler
   increment), S_j^(f) being the fine path's reflection sign at tau_j. */
static int run_sample_adaptive(const context* ctx, int32_t level, uint64_t sample,
                               double fine[3], double coarse[3]) {
    const oracle_problem* p = &ctx->p;
    const uint64_t M = (uint64_t)p->M0 << level;
    const double h = p->T / (double)M;                       /* h_l */
    const uint64_t tick_base = (uint64_t)1 << ORACLE_TICK_BITS;
    const double tick = h / (double)tick_base;
    const uint64_t t_end = M * tick_base;                    /* T in ticks */
    double lam_adapt, sigma_unused;
    coefficients(p, p->x_adapt, &lam_adapt, &sigma_unused);
    double x0, u0;
    initial_state(p, level, sample, &x0, &u0);
    fine[0] = x0; fine[1] = u0; fine[2] = 1.0;
    coarse[0] = x0; coarse[1] = u0; coarse[2] = 1.0;
    const int naive = (p->coupling == ORACLE_COUPLING_NAIVE);
    int bad = 0;
    uint64_t tf = 0, tc = 0, tau = 0, j = 0;
    uint64_t ef = adaptive_end(p, lam_adapt, fine[0], 0, tick_base, t_end);
    uint64_t ec = (level == 0) ? t_end : adaptive_end(p, lam_adapt, coarse[0], 0, 2 * tick_base, t_end);
    double wf = 0.0, wc = 0.0, z[2];
    while (tf < t_end || (level != 0 && tc < t_end)) {
        uint64_t next = t_end;
        if (tf < t_end && ef < next) next = ef;
        if (level != 0 && tc < t_end && ec < next) next = ec;
        if (j % 2 == 0) oracle_normals(p, level, sample, (uint32_t)(j / 2), z);
        double dW = z[j % 2] * sqrt((double)(next - tau) * tick);
        wf += dW;
        wc += (naive ? 1.0 : fine[2]) * dW;
        tau = next;
        ++j;
        if (tf < t_end && tau == ef) {
            bad |= step_se_dw(p, (double)(ef - tf) * tick, fine, wf);
            tf = ef;
            wf = 0.0;
            if (tf < t_end) ef = adaptive_end(p, lam_adapt, fine[0], tf, tick_base, t_end);
        }
        if (level != 0 && tc < t_end && tau == ec) {
            bad |= step_se_dw(p, (double)(ec - tc) * tick, coarse, (naive ? 1.0 : coarse[2]) * wc);
            tc = ec;
            wc = 0.0;
            if (tc < t_end) ec = adaptive_end(p, lam_adapt, coarse[0], tc, 2 * tick_base, t_end);
        }
    }
    return bad;
}

/* Runs sample `sample` of `level`; fills the terminal fine and coarse states. */
static int run_sample(const context* ctx, int32_t level, uint64_t sample,
                      double fine[3], double coarse[3]) {
    const oracle_problem* p = &ctx->p;
    if (p->integrator == ORACLE_SE && p->x_adapt > 0.0)
        return run_sample_adaptive(ctx, level, sample, fine, coarse);
    uint64_t M = (uint64_t)p->M0 << level;     /* M_l = M_0 2^l */
    double h = p->T / (double)M;               /* h_l = T / M_l */
    double x0, u0;
    initial_state(p, level, sample, &x0, &u0);
    fine[0] = x0; fine[1] = u0; fine[2] = 1.0;
    coarse[0] = x0; coarse[1] = u0; coarse[2] = 1.0;
    int bad = 0;
    double z[2], tilde_a, tilde_b, lam_a, lam_b, unused;
    if (level == 0) {
        /* Level 0: one path of M_0 steps, xi_k is draw (k mod 2) of block floor(k/2). */
        for (uint64_t k = 0; k < M; ++k) {
            if (k % 2 == 0) oracle_normals(p, level, sample, (uint32_t)(k / 2), z);
            bad |= oracle_step(p, h, fine, z[k % 2], 0, &tilde_a, &lam_a);
        }
        return bad;
    }
    for (uint64_t m = 0; m < M / 2; ++m) {
        oracle_normals(p, level, sample, (uint32_t)m, z);
        bad |= oracle_step(p, h, fine, z[0], 0, &tilde_a, &lam_a);   /* fine step 2m   */
        bad |= oracle_step(p, h, fine, z[1], 0, &tilde_b, &lam_b);   /* fine step 2m+1 */
        double xi_c;
        if (p->integrator == ORACLE_SE) {
            /* Eq. (18) in extended variables (Eq. 31) */
            xi_c = (tilde_a + tilde_b) / sqrt(2.0);
        } else {
            /* Eq. (19) in extended variables (Eq. 32) */
            double w = exp(-lam_a * h);
            xi_c = (w * tilde_a + tilde_b) / sqrt(exp(-2.0 * lam_a * h) + 1.0);
        }
        bad |= oracle_step(p, 2.0 * h, coarse, xi_c, 1, &unused, &lam_b);
    }
    return bad;
}

int oracle_sample(const oracle_problem* p, int32_t level, uint64_t sample,
                  double* pf, double* pc) {
    context ctx;
    make_context(p, &ctx);
    double fine[3], coarse[3];
    int bad = run_sample(&ctx, level, sample, fine, coarse);
    *pf = qoi(&ctx, fine[0], fine[1]);
    *pc = (level == 0) ? 0.0 : qoi(&ctx, coarse[0], coarse[1]);
    return (bad || !isfinite(*pf) || !isfinite(*pc)) ? 1 : 0;
}

void oracle_level_samples(const oracle_problem* p, int32_t level, uint64_t begin,
                          uint64_t n, double* out) {
    context ctx;
    make_context(p, &ctx);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        double fine[3], coarse[3];
        run_sample(&ctx, level, begin + (uint64_t)k, fine, coarse);
        out[2 * k] = qoi(&ctx, fine[0], fine[1]);
        out[2 * k + 1] = (level == 0) ? 0.0 : qoi(&ctx, coarse[0], coarse[1]);
    }
}

void oracle_level_states(const oracle_problem* p, int32_t level, uint64_t begin,
                         uint64_t n, double* out) {
    context ctx;
    make_context(p, &ctx);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        double fine[3], coarse[3];
        run_sample(&ctx, level, begin + (uint64_t)k, fine, coarse);
        out[4 * k + 0] = fine[0];
        out[4 * k + 1] = fine[1];
        out[4 * k + 2] = (level == 0) ? NAN : coarse[0];
        out[4 * k + 3] = (level == 0) ? NAN : coarse[1];
    }
}

/* ================================================================================== */
/* Compensated level sums (Neumaier's improvement of Kahan summation).                 */
/* ================================================================================== */

static void neumaier_add(double* s, double* c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

static void sums_merge(oracle_sums* into, const oracle_sums* from) {
    for (int k = 0; k < 4; ++k) {
        neumaier_add(&into->s[k], &into->c[k], from->s[k]);
        into->c[k] += from->c[k];
    }
    into->n += from->n;
    into->n_nonfinite += from->n_nonfinite;
}

double oracle_sums_value(const oracle_sums* s, int32_t k) { return s->s[k] + s->c[k]; }

void oracle_level_sums(const oracle_problem* p, int32_t level, uint64_t begin,
                       uint64_t n, oracle_sums* out) {
    context ctx;
    make_context(p, &ctx);
    uint64_t nchunks = (n + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    oracle_sums* part = (oracle_sums*)calloc(nchunks ? nchunks : 1, sizeof(oracle_sums));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < (int64_t)nchunks; ++ch) {
        oracle_sums acc;
        memset(&acc, 0, sizeof acc);
        uint64_t lo = (uint64_t)ch * ORACLE_CHUNK;
        uint64_t hi = lo + ORACLE_CHUNK < n ? lo + ORACLE_CHUNK : n;
        for (uint64_t k = lo; k < hi; ++k) {
            double fine[3], coarse[3];
            int bad = run_sample(&ctx, level, begin + k, fine, coarse);
            double pf = qoi(&ctx, fine[0], fine[1]);
            double pc = (level == 0) ? 0.0 : qoi(&ctx, coarse[0], coarse[1]);
            double y = pf - pc;   /* Y_l = P_l - P_{l-1}, Eq. (16) */
            if (bad || !isfinite(pf) || !isfinite(pc)) {
                acc.n_nonfinite++;
                continue;
            }
            neumaier_add(&acc.s[0], &acc.c[0], y);
            neumaier_add(&acc.s[1], &acc.c[1], y * y);
            neumaier_add(&acc.s[2], &acc.c[2], pf);
            neumaier_add(&acc.s[3], &acc.c[3], pf * pf);
            acc.n++;
        }
        part[ch] = acc;
    }
    memset(out, 0, sizeof *out);
    for (uint64_t ch = 0; ch < nchunks; ++ch) sums_merge(out, &part[ch]);
    free(part);
}

/* ================================================================================== */
/* MLMC driver.                                                                        */
/*                                                                                     */
/* The MSE of Eq. (17) is split evenly: sum_l V_l / N_l <= eps^2 / 2 and bias <=       */
/* eps / sqrt(2) (Sec. 3.2 and the opening of Sec. 6). N_l minimises the cost         */
/* sum_l N_l C_l (C_l = M_l, condition (iv) of the theorem in Sec. 3.3) under the      */
/* variance constraint, which gives                                                    */
/*     N_l = ceil( 2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k) )                      */
/* (Giles 2008, cited in Sec. 6). After each batch, levels that need more than 1%     */
/* extra samples get them; once none does, the bias is estimated from the finest two  */
/* level means, E[P_L - P] ~ Yhat_L / (2^alpha - 1), with alpha the weak order: the   */
/* paper's first order (Sec. 3.1) by default, or a least-squares fit of log2 |Yhat_l| */
/* (Sec. 6 fits c_1 h^alpha). If it exceeds eps / sqrt(2), a level is added whose     */
/* variance is extrapolated with the quadratic decay of condition (iii).              */
/* ================================================================================== */

static double level_cost(int32_t M0, int32_t l) { return (double)M0 * ldexp(1.0, l); }

static void optimal_dn(const oracle_plan_in* in, int32_t L, const double* V, double eps_abs,
                       uint64_t* dn) {
    double total = 0.0;
    for (int32_t l = 0; l <= L; ++l) total += sqrt(V[l] * level_cost(in->M0, l));
    for (int32_t l = 0; l <= L; ++l) {
        double target = ceil(2.0 * total * sqrt(V[l] / level_cost(in->M0, l)) / (eps_abs * eps_abs));
        uint64_t have = (l <= in->L) ? in->n[l] : 0;
        if (!(target > (double)have))   /* also catches NaN */
            dn[l] = 0;
        else if (target >= 1.8e19)
            dn[l] = (uint64_t)1 << 62;
        else
            dn[l] = (uint64_t)target - have;
    }
}

void oracle_plan(const oracle_plan_in* in, oracle_plan_out* out) {
    memset(out, 0, sizeof *out);
    int32_t L = in->L;
    double estimate = 0.0, stat_var = 0.0;
    for (int32_t l = 0; l <= L; ++l) {
        double n = (double)in->n[l];
        double mean = in->n[l] > 0 ? in->sum1[l] / n : 0.0;
        double var = 0.0;
        if (in->n[l] > 1) var = (in->sum2[l] - n * mean * mean) / (n - 1.0);
        if (!(var > 0.0)) var = 0.0;
        out->Yhat[l] = mean;
        out->V[l] = var;
        estimate += mean;
        if (in->n[l] > 0) stat_var += var / n;
    }
    out->estimate = estimate;
    out->stat_var = stat_var;
    out->eps_abs = in->eps_is_relative ? in->eps * fabs(estimate) : in->eps;

    /* weak order alpha: given, or the least-squares slope of -log2 |Yhat_l| over l = 1..L */
    double alpha = in->alpha;
    if (!(alpha > 0.0)) {
        alpha = 1.0;
        double sl = 0, sy = 0, sll = 0, sly = 0;
        int cnt = 0;
        for (int32_t l = 1; l <= L; ++l) {
            if (!(fabs(out->Yhat[l]) > 0.0)) continue;
            double y = -log2(fabs(out->Yhat[l]));
            sl += l; sy += y; sll += (double)l * l; sly += l * y;
            cnt++;
        }
        if (cnt >= 2) {
            double den = cnt * sll - sl * sl;
            if (den > 0) alpha = (cnt * sly - sl * sy) / den;
        }
        if (!(alpha >= 0.5)) alpha = 0.5;
        if (alpha > 2.0) alpha = 2.0;
    }
    out->alpha = alpha;
    double bias = 0.0;
    if (L >= 1) {
        double a = fabs(out->Yhat[L]);
        double b = fabs(out->Yhat[L - 1]) / pow(2.0, alpha);
        bias = (a > b ? a : b) / (pow(2.0, alpha) - 1.0);
    }
    out->bias_est = bias;
    out->L = L;

    if (in->fixed_N) {
        out->status = 1;
        return;
    }
    optimal_dn(in, L, out->V, out->eps_abs, out->dn);
    int more = 0;
    for (int32_t l = 0; l <= L; ++l)
        if ((double)out->dn[l] > 0.01 * (double)in->n[l]) more = 1;
    if (more) {
        out->status = 0;
        return;
    }
    for (int32_t l = 0; l <= L; ++l) out->dn[l] = 0;
    if (in->fixed_L >= 0 || L < 1 || bias <= out->eps_abs / sqrt(2.0)) {
        out->status = 1;
        return;
    }
    if (L >= in->L_max || L + 1 >= ORACLE_MAX_LEVELS) {
        out->status = 2;
        return;
    }
    /* add level L + 1 with V_{L+1} = V_L / 4 */
    double V[ORACLE_MAX_LEVELS];
    for (int32_t l = 0; l <= L; ++l) V[l] = out->V[l];
    V[L + 1] = V[L] / 4.0;
    optimal_dn(in, L + 1, V, out->eps_abs, out->dn);
    if (out->dn[L + 1] < in->N_init) out->dn[L + 1] = in->N_init;
    out->L = L + 1;
    out->status = 0;
}

int oracle_estimate(double eps, const oracle_problem* p, const oracle_opts* opts,
                    oracle_result* out) {
    memset(out, 0, sizeof *out);
    if (!(eps > 0.0)) return -1;
    oracle_sums sums[ORACLE_MAX_LEVELS];
    uint64_t drawn[ORACLE_MAX_LEVELS];
    memset(sums, 0, sizeof sums);
    memset(drawn, 0, sizeof drawn);
    oracle_plan_in in;
    memset(&in, 0, sizeof in);
    in.L = opts->fixed_L >= 0 ? opts->fixed_L : opts->L_min;
    in.M0 = p->M0;
    in.eps = eps;
    in.eps_is_relative = opts->eps_is_relative;
    in.L_max = opts->L_max;
    in.fixed_L = opts->fixed_L;
    in.fixed_N = opts->fixed_N;
    in.N_init = opts->N_init;
    in.alpha = opts->alpha;
    uint64_t dn[ORACLE_MAX_LEVELS];
    memset(dn, 0, sizeof dn);
    for (int32_t l = 0; l <= in.L; ++l) dn[l] = opts->N_init;
    oracle_plan_out plan;
    memset(&plan, 0, sizeof plan);
    int iter = 0;
    int max_iter = opts->max_iter > 0 ? opts->max_iter : 100;
    for (;;) {
        for (int32_t l = 0; l <= in.L; ++l) {
            if (dn[l] == 0) continue;
            oracle_sums add;
            oracle_level_sums(p, l, drawn[l], dn[l], &add);
            sums_merge(&sums[l], &add);
            drawn[l] += dn[l];
        }
        for (int32_t l = 0; l <= in.L; ++l) {
            in.n[l] = sums[l].n;
            in.sum1[l] = oracle_sums_value(&sums[l], 0);
            in.sum2[l] = oracle_sums_value(&sums[l], 1);
        }
        oracle_plan(&in, &plan);
        ++iter;
        if (plan.status != 0 || iter >= max_iter) break;
        in.L = plan.L;
        memcpy(dn, plan.dn, sizeof dn);
    }
    out->estimate = plan.estimate;
    out->eps_abs = plan.eps_abs;
    out->bias_est = plan.bias_est;
    out->stat_var = plan.stat_var;
    out->rmse_est = sqrt(plan.bias_est * plan.bias_est + plan.stat_var);
    out->alpha = plan.alpha;
    out->L = plan.L;
    out->iterations = iter;
    out->status = plan.status == 0 ? 2 : plan.status;
    for (int32_t l = 0; l <= plan.L; ++l) {
        out->N[l] = drawn[l];
        out->n_nonfinite += sums[l].n_nonfinite;
        out->Yhat[l] = plan.Yhat[l];
        out->V[l] = plan.V[l];
        double M = level_cost(p->M0, l);
        out->fine_steps += (double)drawn[l] * M;
        out->integrator_steps += (double)drawn[l] * (l == 0 ? M : 1.5 * M);
    }
    return out->n_nonfinite ? -5 : 0;
}

/* ================================================================================== */
/* Vector QoI: the binned concentration of Sec. 6.4.                                  */
/* ================================================================================== */

void oracle_pdf_level_sums(const oracle_problem* p, int32_t level, uint64_t begin,
                           uint64_t n, double a0, double width, int32_t n_bins,
                           oracle_sums* out) {
    /* one scalar context per bin: the box [a_i, a_{i+1}] of Eq. (34) / (37) */
    context* box = (context*)malloc((size_t)n_bins * sizeof(context));
    for (int32_t i = 0; i < n_bins; ++i) {
        oracle_problem q = *p;
        q.qoi_kind = ORACLE_QOI_P_BOX;
        q.qa = a0 + (double)i * width;
        q.qb = a0 + (double)(i + 1) * width;
        make_context(&q, &box[i]);
    }
    context ctx;
    make_context(p, &ctx);
    uint64_t nchunks = (n + ORACLE_CHUNK - 1) / ORACLE_CHUNK;
    oracle_sums* part = (oracle_sums*)calloc((nchunks ? nchunks : 1) * (size_t)n_bins,
                                             sizeof(oracle_sums));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < (int64_t)nchunks; ++ch) {
        oracle_sums* acc = &part[(size_t)ch * n_bins];
        uint64_t lo = (uint64_t)ch * ORACLE_CHUNK;
        uint64_t hi = lo + ORACLE_CHUNK < n ? lo + ORACLE_CHUNK : n;
        for (uint64_t k = lo; k < hi; ++k) {
            double fine[3], coarse[3];
            int bad = run_sample(&ctx, level, begin + k, fine, coarse);
            if (bad || !isfinite(fine[0]) || (level != 0 && !isfinite(coarse[0]))) {
                for (int32_t i = 0; i < n_bins; ++i) acc[i].n_nonfinite++;
                continue;
            }
            for (int32_t i = 0; i < n_bins; ++i) {
                double pf = qoi(&box[i], fine[0], fine[1]);
                double pc = (level == 0) ? 0.0 : qoi(&box[i], coarse[0], coarse[1]);
                double y = pf - pc;
                neumaier_add(&acc[i].s[0], &acc[i].c[0], y);
                neumaier_add(&acc[i].s[1], &acc[i].c[1], y * y);
                neumaier_add(&acc[i].s[2], &acc[i].c[2], pf);
                neumaier_add(&acc[i].s[3], &acc[i].c[3], pf * pf);
                acc[i].n++;
            }
        }
    }
    for (int32_t i = 0; i < n_bins; ++i) {
        memset(&out[i], 0, sizeof out[i]);
        for (uint64_t ch = 0; ch < nchunks; ++ch) sums_merge(&out[i], &part[ch * n_bins + i]);
    }
    free(part);
    free(box);
}

static void mean_var(uint64_t n_, double s1, double s2, double* mean, double* var) {
    double n = (double)n_;
    *mean = n_ > 0 ? s1 / n : 0.0;
    *var = 0.0;
    if (n_ > 1) *var = (s2 - n * *mean * *mean) / (n - 1.0);
    if (!(*var > 0.0)) *var = 0.0;
}

void oracle_pdf_plan(const oracle_pdf_plan_in* in, oracle_pdf_plan_out* out) {
    memset(out, 0, sizeof *out);
    int32_t L = in->L, k = in->n_bins;
    double Yhat[ORACLE_MAX_LEVELS][ORACLE_MAX_BINS];
    double Ymax[ORACLE_MAX_LEVELS];
    double stat_var = 0.0;
    for (int32_t i = 0; i < k; ++i) out->estimate[i] = 0.0;
    for (int32_t l = 0; l <= L; ++l) {
        out->V[l] = 0.0;
        Ymax[l] = 0.0;
        for (int32_t i = 0; i < k; ++i) {
            double mean, var;
            mean_var(in->n[l], in->sum1[l][i], in->sum2[l][i], &mean, &var);
            Yhat[l][i] = mean;
            out->estimate[i] += mean;
            if (var > out->V[l]) out->V[l] = var;           /* max_i Var[Y_{l,i}] */
            if (fabs(mean) > Ymax[l]) Ymax[l] = fabs(mean);
        }
    }
    for (int32_t i = 0; i < k; ++i) {                       /* max_i sum_l V_{l,i} / N_l */
        double sv = 0.0;
        for (int32_t l = 0; l <= L; ++l) {
            double mean, var;
            mean_var(in->n[l], in->sum1[l][i], in->sum2[l][i], &mean, &var);
            if (in->n[l] > 0) sv += var / (double)in->n[l];
        }
        if (sv > stat_var) stat_var = sv;
    }
    out->stat_var = stat_var;
    double alpha = in->alpha;
    if (!(alpha > 0.0)) {                                   /* fit on max_i |Yhat_{l,i}| */
        alpha = 1.0;
        double sl = 0, sy = 0, sll = 0, sly = 0;
        int cnt = 0;
        for (int32_t l = 1; l <= L; ++l) {
            if (!(Ymax[l] > 0.0)) continue;
            double y = -log2(Ymax[l]);
            sl += l; sy += y; sll += (double)l * l; sly += l * y;
            cnt++;
        }
        if (cnt >= 2) {
            double den = cnt * sll - sl * sl;
            if (den > 0) alpha = (cnt * sly - sl * sy) / den;
        }
        if (!(alpha >= 0.5)) alpha = 0.5;
        if (alpha > 2.0) alpha = 2.0;
    }
    out->alpha = alpha;
    double bias = 0.0;
    if (L >= 1) {
        for (int32_t i = 0; i < k; ++i) {
            double a = fabs(Yhat[L][i]);
            double b = fabs(Yhat[L - 1][i]) / pow(2.0, alpha);
            double bi = (a > b ? a : b) / (pow(2.0, alpha) - 1.0);
            if (bi > bias) bias = bi;
        }
    }
    out->bias_est = bias;
    out->L = L;
    /* the scalar decision with V_l = max_i Var[Y_{l,i}] */
    oracle_plan_in sc;
    memset(&sc, 0, sizeof sc);
    sc.L = L;
    sc.M0 = in->M0;
    for (int32_t l = 0; l <= L; ++l) sc.n[l] = in->n[l];
    optimal_dn(&sc, L, out->V, in->eps, out->dn);
    int more = 0;
    for (int32_t l = 0; l <= L; ++l)
        if ((double)out->dn[l] > 0.01 * (double)in->n[l]) more = 1;
    if (more) {
        out->status = 0;
        return;
    }
    for (int32_t l = 0; l <= L; ++l) out->dn[l] = 0;
    if (in->fixed_L >= 0 || L < 1 || bias <= in->eps / sqrt(2.0)) {
        out->status = 1;
        return;
    }
    if (L >= in->L_max || L + 1 >= ORACLE_MAX_LEVELS) {
        out->status = 2;
        return;
    }
    double V[ORACLE_MAX_LEVELS];
    for (int32_t l = 0; l <= L; ++l) V[l] = out->V[l];
    V[L + 1] = V[L] / 4.0;
    optimal_dn(&sc, L + 1, V, in->eps, out->dn);
    if (out->dn[L + 1] < in->N_init) out->dn[L + 1] = in->N_init;
    out->L = L + 1;
    out->status = 0;
}

int oracle_estimate_pdf(double eps, const oracle_problem* p, const oracle_opts* opts,
                        double a0, double width, int32_t n_bins, int32_t estimator,
                        oracle_pdf_result* out) {
    memset(out, 0, sizeof *out);
    if (!(eps > 0.0) || n_bins < 1 || n_bins > ORACLE_MAX_BINS) return -1;
    out->estimator = estimator;
    int max_iter = opts->max_iter > 0 ? opts->max_iter : 100;
    oracle_sums* sums = (oracle_sums*)calloc((size_t)ORACLE_MAX_LEVELS * n_bins, sizeof(oracle_sums));
    oracle_sums* add = (oracle_sums*)calloc((size_t)n_bins, sizeof(oracle_sums));
    uint64_t drawn[ORACLE_MAX_LEVELS];
    memset(drawn, 0, sizeof drawn);
    int iter = 0;
    if (estimator == ORACLE_STMC) {
        /* the single fine path of level L: level 0 of the problem with M0 2^L steps */
        if (opts->fixed_L < 0) { free(sums); free(add); return -1; }
        oracle_problem q = *p;
        q.M0 = p->M0 << opts->fixed_L;
        uint64_t dn = opts->N_init;
        double V = 0.0;
        for (;;) {
            oracle_pdf_level_sums(&q, 0, drawn[0], dn, a0, width, n_bins, add);
            for (int32_t i = 0; i < n_bins; ++i) sums_merge(&sums[i], &add[i]);
            drawn[0] += dn;
            ++iter;
            uint64_t n = sums[0].n;
            V = 0.0;
            for (int32_t i = 0; i < n_bins; ++i) {
                double mean, var;
                mean_var(n, oracle_sums_value(&sums[i], 0), oracle_sums_value(&sums[i], 1), &mean, &var);
                out->estimate[i] = mean;
                if (var > V) V = var;
            }
            double target = ceil(2.0 * V / (eps * eps));
            dn = (target > (double)n) ? (uint64_t)target - n : 0;
            if (!((double)dn > 0.01 * (double)n) || iter >= max_iter) break;
        }
        out->L = opts->fixed_L;
        out->N[0] = drawn[0];
        out->V[0] = V;
        out->stat_var = V / (double)(sums[0].n ? sums[0].n : 1);
        out->rmse_est = sqrt(out->stat_var);
        out->status = 1;
        out->iterations = iter;
        out->n_nonfinite = sums[0].n_nonfinite;
        out->fine_steps = (double)drawn[0] * (double)q.M0;
        free(sums);
        free(add);
        return out->n_nonfinite ? -5 : 0;
    }
    oracle_pdf_plan_in* in = (oracle_pdf_plan_in*)calloc(1, sizeof *in);
    in->L = opts->fixed_L >= 0 ? opts->fixed_L : opts->L_min;
    in->n_bins = n_bins;
    in->M0 = p->M0;
    in->eps = eps;
    in->L_max = opts->L_max;
    in->fixed_L = opts->fixed_L;
    in->N_init = opts->N_init;
    in->alpha = opts->alpha;
    uint64_t dn[ORACLE_MAX_LEVELS];
    memset(dn, 0, sizeof dn);
    for (int32_t l = 0; l <= in->L; ++l) dn[l] = opts->N_init;
    oracle_pdf_plan_out plan;
    memset(&plan, 0, sizeof plan);
    for (;;) {
        for (int32_t l = 0; l <= in->L; ++l) {
            if (dn[l] == 0) continue;
            oracle_pdf_level_sums(p, l, drawn[l], dn[l], a0, width, n_bins, add);
            for (int32_t i = 0; i < n_bins; ++i) sums_merge(&sums[(size_t)l * n_bins + i], &add[i]);
            drawn[l] += dn[l];
        }
        for (int32_t l = 0; l <= in->L; ++l) {
            in->n[l] = sums[(size_t)l * n_bins].n;
            for (int32_t i = 0; i < n_bins; ++i) {
                in->sum1[l][i] = oracle_sums_value(&sums[(size_t)l * n_bins + i], 0);
                in->sum2[l][i] = oracle_sums_value(&sums[(size_t)l * n_bins + i], 1);
            }
        }
        oracle_pdf_plan(in, &plan);
        ++iter;
        if (plan.status != 0 || iter >= max_iter) break;
        in->L = plan.L;
        memcpy(dn, plan.dn, sizeof dn);
    }
    for (int32_t i = 0; i < n_bins; ++i) out->estimate[i] = plan.estimate[i];
    out->bias_est = plan.bias_est;
    out->stat_var = plan.stat_var;
    out->rmse_est = sqrt(plan.bias_est * plan.bias_est + plan.stat_var);
    out->L = plan.L;
    out->iterations = iter;
    out->status = plan.status == 0 ? 2 : plan.status;
    for (int32_t l = 0; l <= plan.L; ++l) {
        out->N[l] = drawn[l];
        out->n_nonfinite += sums[(size_t)l * n_bins].n_nonfinite;
        out->V[l] = plan.V[l];
        out->fine_steps += (double)drawn[l] * level_cost(p->M0, l);
    }
    free(in);
    free(sums);
    free(add);
    return out->n_nonfinite ? -5 : 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (n >= 1); results do not depend on it. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
