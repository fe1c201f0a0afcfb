/*
 * oracle.h -- C ABI of the plain CPU FP64 oracle.
 *
 * TEST INFRASTRUCTURE. This library exists to check the GPU library against the
 * paper; it is not part of the product. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header, helper or
 * constant table with the GPU library (whose ABI is include/ldmlmc.h).
 *
 * Paper: G. Katsiolides, E. H. Mueller, R. Scheichl, T. Shardlow, M. B. Giles,
 * D. J. Thomson, "Multilevel Monte Carlo and improved timestepping methods in
 * atmospheric dispersion modelling", arXiv:1612.07717 (J. Comput. Phys. 2018).
 *
 * All quantities are SI (metres, seconds). The paper works in units of
 * X_ref = H = 1000 m and t_ref = 1000 s (Sec. 6); callers convert.
 */
#ifndef LD_ORACLE_H
#define LD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_SE = 0, ORACLE_GL = 1, ORACLE_BAOAB = 2 };
enum { ORACLE_PROFILE_HOMOGENEOUS = 0, ORACLE_PROFILE_NEUTRAL_BL = 1 };
enum { ORACLE_RELEASE_FIXED_W = 0, ORACLE_RELEASE_GAUSSIAN_W = 1, ORACLE_RELEASE_WELL_MIXED = 2 };
enum {
    ORACLE_QOI_MEAN_Z = 0,    /* phi = X_T                                   (Sec. 2) */
    ORACLE_QOI_P_ABOVE = 1,   /* phi = 1 - theta(X_T - a), smoothed if r > 0  (Sec. 5) */
    ORACLE_QOI_P_BOX = 2,     /* phi = theta(X_T - b) - theta(X_T - a)        (Eqs. 34, 37) */
    ORACLE_QOI_VELOCITY = 3,  /* phi = U_T                                   (Sec. 2: phi(U_t, X_t)) */
    ORACLE_QOI_VELOCITY_SQ = 4/* phi = U_T^2 */
};
enum { ORACLE_COUPLING_REFLECTED = 0, ORACLE_COUPLING_NAIVE = 1 };

typedef struct {
    int32_t profile_kind;   /* ORACLE_PROFILE_* */
    int32_t integrator;     /* ORACLE_SE / ORACLE_GL / ORACLE_BAOAB */
    double H;               /* boundary-layer depth [m] */
    double sigma_u;         /* homogeneous profile: constant sigma_U [m/s] */
    double tau;             /* homogeneous profile: constant tau [s] */
    double kappa_sigma;     /* neutral profile, Eq. (5) */
    double kappa_tau;
    double u_star;          /* friction velocity [m/s] */
    double eps_reg;         /* regularisation height of Eq. (7) [m] */
    int32_t release_kind;   /* ORACLE_RELEASE_* */
    int32_t coupling;       /* ORACLE_COUPLING_*: NAIVE sets every S to 1 (negative control) */
    double z0;              /* release height [m] */
    double w0;              /* release velocity [m/s] (FIXED_W only) */
    int32_t qoi_kind;       /* ORACLE_QOI_* */
    int32_t r;              /* 0: raw indicator; 1..8: smoothing degree of Eq. (35) */
    double qa, qb;          /* z* (P_ABOVE) or [a, b] (P_BOX) [m] */
    double delta;           /* smoothing width of Eq. (37) [m] */
    double T;               /* final time [s] */
    int32_t M0;             /* timesteps on level 0 */
    uint32_t stream_id;     /* independent random stream, 24 bits */
    uint64_t seed;          /* Philox key */
    double x_adapt;         /* > 0 (symplectic Euler only): adaptive, non-nested timesteps
                               below this reference height (Sec. 7); 0: uniform steps */
} oracle_problem;

/* Adaptive timesteps (Sec. 7): a path at X takes h_n = min(h, lambda(X_adapt) / lambda(X) h)
   from its base step h (h_l on the fine path, 2 h_l on the coarse path), rounded down to a
   whole tick of h_l / 2^ORACLE_TICK_BITS (at least one) and cut at T. Time is counted in
   ticks, so coinciding fine and coarse time points coincide exactly. */
#define ORACLE_TICK_BITS 20

/* Compensated (Neumaier) sums of Y, Y^2, P_f, P_f^2 over the finite samples. */
typedef struct {
    double s[4];
    double c[4];
    uint64_t n;             /* finite samples summed */
    uint64_t n_nonfinite;   /* samples whose result was not finite; excluded from s, c */
} oracle_sums;

/* ---- generator ---------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Two N(0,1) draws of Philox block `block` for (level, sample): out[0] (cos branch),
   out[1] (sin branch). */
void oracle_normals(const oracle_problem* p, int32_t level, uint64_t sample,
                    uint32_t block, double out[2]);

/* ---- model ----------------------------------------------------------------------- */
/* Regularised sigma_U(x) and tau(x), Eqs. (5) and (7). */
void oracle_profile(const oracle_problem* p, double x, double* sigma_u, double* tau);
/* dV/dX(x, u) of the potential defined after Eq. (3). */
double oracle_dVdX(const oracle_problem* p, double x, double u);
/* Coefficients c[0..r+1] of p_r(s) = sum c_k s^k (Eq. 35 and its moment conditions). */
int oracle_smoothing_poly(int32_t r, double* coef);
double oracle_qoi(const oracle_problem* p, double x, double u);

/* One step of size h of the problem's integrator. state = {X, U, S}. If noise_is_tilde
   is 0, xi is the physical noise and *tilde receives S*xi; otherwise xi is an
   extended-variable noise and the physical noise is S*xi (Eqs. 30-32). *lam_o receives
   lambda at the point where the noise enters (the O-step point for GL and BAOAB).
   Returns 0, or -1 if the state became non-finite. */
int oracle_step(const oracle_problem* p, double h, double state[3], double xi,
                int32_t noise_is_tilde, double* tilde, double* lam_o);

/* ---- one coupled sample and level reductions ---------------------------------- */
/* P_f and P_c (P_c = 0 on level 0) of sample `sample` on `level`; returns 1 when the
   sample is non-finite. */
int oracle_sample(const oracle_problem* p, int32_t level, uint64_t sample,
                  double* pf, double* pc);
/* Per-sample dump: out[2*k] = P_f, out[2*k+1] = P_c of sample begin+k. */
void oracle_level_samples(const oracle_problem* p, int32_t level, uint64_t begin,
                          uint64_t n, double* out);
/* Terminal states: out[4*k..4*k+3] = X_f, U_f, X_c, U_c of sample begin+k. */
void oracle_level_states(const oracle_problem* p, int32_t level, uint64_t begin,
                         uint64_t n, double* out);
void oracle_level_sums(const oracle_problem* p, int32_t level, uint64_t begin,
                       uint64_t n, oracle_sums* out);
double oracle_sums_value(const oracle_sums* s, int32_t k);

/* ---- MLMC driver ---------------------------------------------------------------- */
#define ORACLE_MAX_LEVELS 32

typedef struct {
    int32_t L_min, L_max;
    int32_t fixed_L;        /* >= 0: levels 0..fixed_L, no bias test */
    int32_t fixed_N;        /* nonzero: one batch of N_init samples per level */
    uint64_t N_init;
    int32_t eps_is_relative;
    int32_t max_iter;
    double alpha;           /* weak order used by the bias test; <= 0: fit it */
} oracle_opts;

/* One decision of the adaptive algorithm; see oracle.c. */
typedef struct {
    int32_t L;
    uint64_t n[ORACLE_MAX_LEVELS];      /* finite samples so far */
    double sum1[ORACLE_MAX_LEVELS];     /* sum of Y */
    double sum2[ORACLE_MAX_LEVELS];     /* sum of Y^2 */
    int32_t M0;
    double eps;
    int32_t eps_is_relative;
    int32_t L_max;
    int32_t fixed_L;
    int32_t fixed_N;
    uint64_t N_init;
    double alpha;                       /* weak order; <= 0: least-squares fit */
} oracle_plan_in;

typedef struct {
    int32_t status;                     /* 0 more samples, 1 converged, 2 stopped at L_max */
    int32_t L;                          /* finest level after this decision */
    uint64_t dn[ORACLE_MAX_LEVELS];     /* extra samples to draw per level */
    double Yhat[ORACLE_MAX_LEVELS];
    double V[ORACLE_MAX_LEVELS];
    double estimate, eps_abs, alpha, bias_est, stat_var;
} oracle_plan_out;

void oracle_plan(const oracle_plan_in* in, oracle_plan_out* out);

typedef struct {
    double estimate, eps_abs, bias_est, stat_var, rmse_est, alpha;
    int32_t L, iterations, status;      /* status as oracle_plan_out.status */
    int32_t pad;
    uint64_t N[ORACLE_MAX_LEVELS];      /* samples drawn per level */
    uint64_t n_nonfinite;
    double Yhat[ORACLE_MAX_LEVELS], V[ORACLE_MAX_LEVELS];
    double fine_steps;                  /* sum_l N_l M_l */
    double integrator_steps;            /* sum_l N_l (M_l + M_l / 2) */
} oracle_result;

int oracle_estimate(double eps, const oracle_problem* p, const oracle_opts* opts,
                    oracle_result* out);

/* ---- vector QoI: binned concentration (Sec. 6.4) --------------------------------- */
#define ORACLE_MAX_BINS 64
enum { ORACLE_MLMC = 0, ORACLE_STMC = 1 };

/* Per-bin sums for the vector QoI of Sec. 6.4. Bin i is [a0 + i w, a0 + (i+1) w],
   i < n_bins; P_i is the box indicator of Eq. (34) (r = 0) or its smoothing by Eq. (37)
   (r > 0), with the problem's r and delta (its qoi_kind is ignored); Y_i = P_i(X_f) -
   P_i(X_c) (Eq. 16; P_i(X_c) = 0 on level 0). out[i] for i < n_bins. A sample whose
   paths are not finite is excluded from every bin and counted in each. */
void oracle_pdf_level_sums(const oracle_problem* p, int32_t level, uint64_t begin,
                           uint64_t n, double a0, double width, int32_t n_bins,
                           oracle_sums* out);

/* One decision of the adaptive algorithm for the vector QoI: the sample rule uses
   max_i Var[Y_{l,i}] in place of Var[Y_l] (Sec. 6.4); the bias test takes, over the bins,
   the largest of the scalar bias estimates; eps is absolute. */
typedef struct {
    int32_t L, n_bins;
    uint64_t n[ORACLE_MAX_LEVELS];
    double sum1[ORACLE_MAX_LEVELS][ORACLE_MAX_BINS];   /* sum of Y_{l,i} */
    double sum2[ORACLE_MAX_LEVELS][ORACLE_MAX_BINS];   /* sum of Y_{l,i}^2 */
    int32_t M0;
    int32_t L_max;
    double eps;
    int32_t fixed_L;
    int32_t pad;
    uint64_t N_init;
    double alpha;                                      /* <= 0: fit on max_i |Yhat_{l,i}| */
} oracle_pdf_plan_in;

typedef struct {
    int32_t status, L;                                 /* as oracle_plan_out */
    uint64_t dn[ORACLE_MAX_LEVELS];
    double V[ORACLE_MAX_LEVELS];                       /* max_i Var[Y_{l,i}] */
    double estimate[ORACLE_MAX_BINS];                  /* sum_l Yhat_{l,i} */
    double bias_est, stat_var, alpha;                  /* maxima over the bins */
} oracle_pdf_plan_out;

void oracle_pdf_plan(const oracle_pdf_plan_in* in, oracle_pdf_plan_out* out);

typedef struct {
    double estimate[ORACLE_MAX_BINS];
    double bias_est, stat_var, rmse_est;
    int32_t L, iterations, status, estimator;
    uint64_t N[ORACLE_MAX_LEVELS];
    uint64_t n_nonfinite;
    double V[ORACLE_MAX_LEVELS];
    double fine_steps;
} oracle_pdf_result;

/* Binned-concentration estimate to absolute RMSE eps per bin. ORACLE_MLMC: the adaptive
   driver with oracle_pdf_plan. ORACLE_STMC: standard Monte Carlo (Sec. 3.2) with the
   single fine path of step T / (M0 2^L), L = opts->fixed_L (>= 0): N_init samples,
   then N = ceil(2 max_i Var[P_i] / eps^2) with the same 1 % top-up rule. */
int oracle_estimate_pdf(double eps, const oracle_problem* p, const oracle_opts* opts,
                        double a0, double width, int32_t n_bins, int32_t estimator,
                        oracle_pdf_result* out);

int oracle_num_threads(void);
/* Sets the OpenMP threads of later calls (n >= 1); results do not depend on it. */
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
