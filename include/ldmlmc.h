/*
 * ldmlmc.h -- C ABI of the MI355X (gfx950) multilevel Monte Carlo library for
 * Lagrangian atmospheric dispersion.
 *
 * Method: G. Katsiolides, E. H. Mueller, R. Scheichl, T. Shardlow, M. B. Giles,
 * D. J. Thomson, "Multilevel Monte Carlo and improved timestepping methods in
 * atmospheric dispersion modelling", arXiv:1612.07717. Section and equation numbers
 * below are the paper's.
 *
 * The library estimates E[phi(X_T)] for the one-dimensional vertical Langevin model of
 * Sec. 2 (Eq. 4, profiles Eq. 5, cut-off Eq. 7, elastic reflection at 0 and H, Eq. 6)
 * with the multilevel Monte Carlo estimator of Sec. 3.3 (Eqs. 14-17). Each level
 * couples a fine path of M_l = M_0 2^l steps with a coarse path of M_l / 2 steps
 * driven by the combined fine increments (Eqs. 18-19), with the reflection sign
 * factors of Sec. 4 (Eqs. 31-32). Integrators: symplectic Euler (Eq. 8), geometric
 * Langevin (Eq. 9) and BAOAB (Eq. 10).
 *
 * Conventions
 *  - SI units throughout (metres, seconds, m/s).
 *  - Every function returns an int status: LD_OK (0), a positive warning with a valid
 *    result, or a negative error. Nothing throws across the ABI; nothing exits.
 *  - Pointers named d_* are DEVICE pointers (hipMalloc or a torch CUDA tensor's
 *    data_ptr on the current device); all others are host pointers. The caller owns
 *    every buffer; the library keeps no pointer after a call returns.
 *  - hip_stream is a hipStream_t (NULL = the default stream). Level-sum calls only
 *    enqueue work on it and return; mlmc_estimate blocks until done.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by `seed`, counter =
 *    (block, sample_lo, sample_hi, level | stream_id << 8), Box-Muller normals. A
 *    sample's result depends only on (problem, integrator, precision, level, sample
 *    index), never on launch shape or batching.
 *  - Level sums are FP64 compensated (Neumaier) sums in both precisions; the
 *    precision selects the arithmetic of the particle paths only.
 */
#ifndef LDMLMC_H
#define LDMLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LDMLMC_ABI_VERSION 1
#define LD_MAX_LEVELS 32

/* ---- status codes ------------------------------------------------------------- */
#define LD_OK 0
#define LD_WARN_NOT_CONVERGED 1  /* mlmc_estimate stopped at L_max or max_iter; result filled */
#define LD_EINVAL (-1)           /* invalid argument (bad parameter, null pointer, size)    */
#define LD_EUNSTABLE (-2)        /* symplectic Euler with lambda_max * h >= 2 (Sec. 3.1; with
                                    adaptive steps lambda(x_adapt) * h >= 2, Sec. 7)         */
#define LD_ENOMEM (-3)           /* workspace smaller than the *_workspace() size           */
#define LD_EDEVICE (-4)          /* HIP runtime error; ld_last_error() has the message       */
#define LD_ENONFINITE (-5)       /* some samples were non-finite (excluded from the sums)    */
#define LD_ENODEVICE (-6)        /* no usable gfx950 device                                 */

/* In C++ the typed enums below have int as their fixed underlying type, so that every
   int a C caller passes is a value of the type; the library rejects unknown values with
   LD_EINVAL. The C ABI is the same either way (an int argument). */
#ifdef __cplusplus
#define LD_ENUM_BASE : int
#else
#define LD_ENUM_BASE
#endif

typedef enum LD_ENUM_BASE { LD_SE = 0, LD_GL = 1, LD_BAOAB = 2 } ld_integrator;   /* Eqs. 8, 9, 10 */
typedef enum LD_ENUM_BASE { LD_FP64 = 0, LD_FP32 = 1 } ld_precision;              /* path arithmetic */

enum { LD_PROFILE_HOMOGENEOUS = 0, LD_PROFILE_NEUTRAL_BL = 1 };
enum { LD_RELEASE_FIXED_W = 0, LD_RELEASE_GAUSSIAN_W = 1, LD_RELEASE_WELL_MIXED = 2 };
enum {
    LD_QOI_MEAN_Z = 0,      /* phi = X_T (Sec. 2)                                         */
    LD_QOI_P_ABOVE = 1,     /* phi = 1(X_T > a); r > 0: 1 - g_r((X_T - a)/delta) (Sec. 5)  */
    LD_QOI_P_BOX = 2,       /* phi = 1_(a,b](X_T) (Eq. 34); r > 0: Eq. 37                   */
    LD_QOI_VELOCITY = 3,    /* phi = U_T                                                  */
    LD_QOI_VELOCITY_SQ = 4  /* phi = U_T^2                                                */
};

/* Turbulence profile. NEUTRAL_BL: sigma_U = kappa_sigma u_* (1 - X/H)^(3/4),
   tau = kappa_tau X / sigma_U (Eq. 5), frozen below eps_reg and above H - eps_reg
   (Eq. 7). HOMOGENEOUS: constant sigma_u and tau. Valid: 1e-6 <= H <= 1e30 (a height
   in metres; the bounds keep H a normal number in both path precisions); NEUTRAL_BL needs
   kappa_sigma, kappa_tau, u_star > 0 and 1e-6 H <= eps_reg < H/2 (a band the FP32 path
   arithmetic resolves); HOMOGENEOUS needs
   sigma_u > 0 and tau > 0. */
typedef struct {
    int32_t kind;
    int32_t reserved;
    double H;
    double sigma_u, tau;
    double kappa_sigma, kappa_tau, u_star, eps_reg;
} ld_profile;

/* Quantity of interest. r = 0 selects the raw indicator; 1 <= r <= 8 the smoothed one
   with polynomial p_r of Eq. (35) and width delta > 0 (Sec. 5). */
typedef struct {
    int32_t kind;
    int32_t r;
    double a, b, delta;
} ld_qoi;

/* Initial condition, shared by the fine and the coarse path. FIXED_W: X_0 = z0,
   U_0 = w0. GAUSSIAN_W: X_0 = z0, U_0 ~ N(0, sigma_U(z0)^2). WELL_MIXED: X_0 ~ U(0, H),
   U_0 ~ N(0, sigma_U(X_0)^2) (the invariant law of Sec. 2). 0 <= z0 <= H. */
typedef struct {
    int32_t kind;
    int32_t reserved;
    double z0, w0;
} ld_release;

/* One estimation problem. T > 0, M0 >= 1, stream_id < 2^24.
   x_adapt (symplectic Euler only; 0 = uniform steps): adaptive, non-nested timesteps
   below this reference height, 0 < x_adapt <= H (Sec. 7). A path at X steps
   h_n = min(h, lambda(x_adapt) / lambda(X) h) from its base step (h_l fine, 2 h_l coarse),
   rounded down to a whole tick of h_l / 2^20 (at least one) and cut at T; the fine and
   coarse paths draw from the merged time grid (the adaptive Euler increment of Sec. 7).
   The stability condition becomes lambda(x_adapt) h < 2. */
typedef struct {
    ld_profile profile;
    ld_release release;
    ld_qoi qoi;
    double T;
    int32_t M0;
    uint32_t stream_id;
    uint64_t seed;
    double x_adapt;
} ld_problem;

/* Compensated sums over the finite samples of one level: index 0 Y_l, 1 Y_l^2,
   2 P_l, 3 P_l^2 (Y_l = P_l - P_{l-1}, Eq. 16; Y_0 = P_0). value_k = s[k] + c[k].
   Samples with a non-finite result are counted in n_nonfinite and excluded. */
typedef struct {
    double s[4];
    double c[4];
    uint64_t n;
    uint64_t n_nonfinite;
} ld_level_sums;

typedef struct {
    int32_t level;
    int32_t reserved;
    uint64_t sample_begin;
    uint64_t n_samples;
} ld_level_range;

/* ---- level sums ----------------------------------------------------------------- */

/* Bytes of device workspace mlmc_level_sums needs for n_samples samples. */
size_t mlmc_level_sums_workspace(uint64_t n_samples);

/* Y_l and P_l sums of samples [sample_begin, sample_begin + n_samples) of `level`
   (0 <= level < LD_MAX_LEVELS, M0 * 2^level <= 2^31), Sec. 3.3, Eq. (16).
   d_out: one ld_level_sums in device memory, overwritten. d_workspace: at least
   mlmc_level_sums_workspace(n_samples) bytes of device memory, contents undefined on
   return. n_samples = 0 writes zero sums. Returns LD_EUNSTABLE for symplectic Euler
   when lambda_max * h >= 2 for a step the level uses (Sec. 3.1). Asynchronous. */
int mlmc_level_sums(const ld_problem* problem, ld_integrator integrator,
                    ld_precision precision, int32_t level, uint64_t sample_begin,
                    uint64_t n_samples, ld_level_sums* d_out, void* d_workspace,
                    size_t workspace_bytes, void* hip_stream);

/* mlmc_level_sums without a workspace, for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).
   Same arguments, kernels and results (bit for bit) as mlmc_level_sums; the block
   partials go to a device array the library owns instead: 32768 partials of 80 bytes
   (2.5 MiB) per device, kept until the process ends, enough for any range (no launch of
   one range uses more blocks). The call allocates nothing: no hipMalloc, hipFree or
   allocating library routine; its first call on a device looks up the array's address
   there. Calls on one device share that array, so calls that overlap on one device
   (on different streams, or from several threads) race and give undefined results;
   calls on one stream are ordered and safe. Nothing in the array needs clearing: every
   launch writes each partial it reads. LD_ENOMEM if a range ever needed more partials
   than the array holds; other errors as mlmc_level_sums. Asynchronous. */
int mlmc_level_sums_noalloc(const ld_problem* problem, ld_integrator integrator,
                            ld_precision precision, int32_t level, uint64_t sample_begin,
                            uint64_t n_samples, ld_level_sums* d_out, void* hip_stream);

/* Several (level, sample range) pairs of one problem in one launch; the most expensive
   levels are dispatched first. d_out: n_ranges ld_level_sums in device memory, in the
   order of `ranges`. 1 <= n_ranges <= LD_MAX_LEVELS. */
size_t mlmc_level_sums_batch_workspace(const ld_level_range* ranges, int32_t n_ranges);
int mlmc_level_sums_batch(const ld_problem* problem, ld_integrator integrator,
                          ld_precision precision, const ld_level_range* ranges,
                          int32_t n_ranges, ld_level_sums* d_out, void* d_workspace,
                          size_t workspace_bytes, void* hip_stream);

/* Per-sample results of the same kernels (a checking hook): d_pf_pc[2k] = P_l and
   d_pf_pc[2k+1] = P_{l-1} (0 on level 0) of sample sample_begin + k, as FP64.
   d_pf_pc holds 2 * n_samples doubles; d_workspace as for mlmc_level_sums. */
int mlmc_level_samples(const ld_problem* problem, ld_integrator integrator,
                       ld_precision precision, int32_t level, uint64_t sample_begin,
                       uint64_t n_samples, double* d_pf_pc, void* d_workspace,
                       size_t workspace_bytes, void* hip_stream);

/* ---- the MLMC driver -------------------------------------------------------------- */

/* One decision of the adaptive MLMC algorithm (host only, no device use). The MSE of
   Eq. (17) is split evenly between bias and variance (Sec. 3.2, Sec. 6); with the
   cost per sample C_l = M_l (condition (iv) of the theorem in Sec. 3.3) the optimal
   N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_k sqrt(V_k C_k)). Levels needing more than 1%
   more samples get them; otherwise the bias is estimated as
   max(|Yhat_L|, |Yhat_{L-1}| 2^-alpha) / (2^alpha - 1) and a level is added (with
   V_{L+1} = V_L / 4, condition (iii)) while it exceeds eps / sqrt(2). alpha <= 0 fits
   the weak order to log2 |Yhat_l|, clamped to [0.5, 2]; the paper's integrators are
   first order (Sec. 3.1), the default alpha = 1. */
typedef struct {
    int32_t L;                          /* current finest level */
    int32_t M0;
    uint64_t n[LD_MAX_LEVELS];          /* finite samples so far per level */
    double sum1[LD_MAX_LEVELS];         /* sum of Y_l */
    double sum2[LD_MAX_LEVELS];         /* sum of Y_l^2 */
    double eps;                         /* RMSE target, absolute or relative */
    double alpha;
    int32_t eps_is_relative;            /* eps_abs = eps * |sum_l Yhat_l| */
    int32_t L_max;
    int32_t fixed_L;                    /* >= 0: never add levels */
    int32_t fixed_N;                    /* nonzero: no adaptation at all */
    uint64_t N_init;                    /* minimum first batch of a new level */
} ld_plan_in;

typedef struct {
    int32_t status;                     /* 0 more samples, 1 converged, 2 stopped at L_max */
    int32_t L;                          /* finest level after this decision */
    uint64_t dn[LD_MAX_LEVELS];         /* extra samples per level */
    double Yhat[LD_MAX_LEVELS], V[LD_MAX_LEVELS];
    double estimate, eps_abs, alpha, bias_est, stat_var;
} ld_plan_out;

int mlmc_plan(const ld_plan_in* in, ld_plan_out* out);

typedef struct {
    ld_release release;
    double T;
    int32_t M0;
    int32_t L_min;           /* first levels 0..L_min (default 2) */
    int32_t L_max;           /* default 20 */
    int32_t fixed_L;         /* >= 0: levels 0..fixed_L, no bias test (default -1) */
    int32_t fixed_N;         /* nonzero: N_init samples on every level, one batch */
    int32_t eps_is_relative;
    uint64_t N_init;         /* first batch per level (default 10000) */
    double alpha;            /* weak order for the bias test (default 1) */
    ld_precision precision;  /* path arithmetic (default LD_FP64) */
    uint32_t stream_id;
    uint64_t seed;
    int32_t max_iter;        /* default 100 */
    int32_t early_topup;     /* nonzero (and L_min or fixed_L >= 5): the first batch of the
                                short levels 0..L0-5 runs on a second stream beside the long
                                levels', and the samples the variance rule asks of the short
                                levels alone are drawn at once, before the long levels end
                                (default 0). Same draws, other sample counts N_l than the
                                plain schedule; the plain MLMC estimate of what is drawn */
    double x_adapt;          /* symplectic Euler: adaptive steps below this height (0 = off) */
    double max_fine_steps;   /* cost budget: stop (LD_WARN_NOT_CONVERGED) rather than draw
                                a batch that would take sum_l N_l M_l above this; the
                                first batch always runs. 0 = no budget (default) */
    void* d_workspace;       /* NULL: allocated and freed inside the call (about 80 MiB, ~0.3 ms
                                per call: pass one for repeated calls) */
    size_t workspace_bytes;
    void* hip_stream;
} ld_estimate_opts;

typedef struct {
    double estimate;         /* sum_l Yhat_l (Eq. 15) */
    double eps_abs;
    double bias_est;
    double stat_var;         /* sum_l V_l / N_l */
    double rmse_est;         /* sqrt(bias_est^2 + stat_var) */
    double alpha;
    int32_t L, iterations, status, reserved;
    uint64_t N[LD_MAX_LEVELS];
    uint64_t n_nonfinite;
    double Yhat[LD_MAX_LEVELS], V[LD_MAX_LEVELS];
    double fine_steps;       /* sum_l N_l M_l: coupled particle-steps */
    double integrator_steps; /* sum_l N_l (M_l + M_l/2) (M_0 on level 0) */
    double wall_seconds;
    double device_seconds;   /* time inside the level-sum kernels (HIP events), summed over
                                streams where batches run side by side */
    int32_t launches;
    int32_t reserved2;
} ld_estimate_result;

void mlmc_estimate_default_opts(ld_estimate_opts* opts);
/* Bytes of workspace mlmc_estimate may need when d_workspace is given. */
size_t mlmc_estimate_workspace(void);

/* Adaptive MLMC estimate of E[phi(X_T)] to RMSE eps (Sec. 3.3, Sec. 6). Blocks until
   done. opts NULL = defaults (which release at z0 = 0 with w0 = 0: pass opts). out is
   filled also on LD_WARN_NOT_CONVERGED and LD_ENONFINITE. */
int mlmc_estimate(double eps, const ld_qoi* qoi, ld_integrator integrator,
                  const ld_profile* profile, const ld_estimate_opts* opts,
                  ld_estimate_result* out);

/* ---- vector QoI: the binned concentration of Sec. 6.4 --------------------------- */

#define LD_MAX_BINS 64

/* Equidistant bins [a0 + i width, a0 + (i+1) width], 0 <= i < n_bins, 1 <= n_bins <=
   LD_MAX_BINS, width > 0. P_i is the box indicator of Eq. (34) (qoi.r = 0) or its
   smoothing by Eq. (37) (qoi.r in 1..8, width qoi.delta > 0), taken from the problem's
   qoi (its kind, a and b are ignored). The paper's p.d.f. uses 20 bins over [0, H]
   with r = 4 and delta = H/10. */
typedef struct {
    double a0, width;
    int32_t n_bins;
    int32_t reserved;
} ld_bins;

/* Bytes of device workspace mlmc_pdf_level_sums needs for n_samples samples. */
size_t mlmc_pdf_level_sums_workspace(uint64_t n_samples, int32_t n_bins);

/* Per-bin sums of Y_i = P_i(X_l) - P_i(X_{l-1}) (Eq. 16 per component; P_i(X_{-1}) = 0),
   Y_i^2, P_i(X_l) and P_i(X_l)^2 over samples [sample_begin, sample_begin + n_samples)
   of `level`: d_out receives n_bins ld_level_sums (device memory, overwritten). The
   sample paths are those of mlmc_level_sums; a sample whose path ran away is counted
   as non-finite in every bin. Asynchronous on hip_stream. */
int mlmc_pdf_level_sums(const ld_problem* problem, ld_integrator integrator,
                        ld_precision precision, int32_t level, uint64_t sample_begin,
                        uint64_t n_samples, const ld_bins* bins, ld_level_sums* d_out,
                        void* d_workspace, size_t workspace_bytes, void* hip_stream);

/* One decision of the adaptive algorithm for the vector QoI (host only). The sample
   rule is mlmc_plan's with max_i Var[Y_{l,i}] in place of Var[Y_l] (Sec. 6.4); the bias
   test takes the largest per-bin bias estimate; eps is an absolute RMSE per bin. */
typedef struct {
    int32_t L, n_bins;
    uint64_t n[LD_MAX_LEVELS];                      /* finite samples per level */
    double sum1[LD_MAX_LEVELS][LD_MAX_BINS];        /* sum of Y_{l,i} */
    double sum2[LD_MAX_LEVELS][LD_MAX_BINS];        /* sum of Y_{l,i}^2 */
    int32_t M0, L_max;
    double eps;
    int32_t fixed_L, reserved;
    uint64_t N_init;
    double alpha;                                   /* <= 0: fit on max_i |Yhat_{l,i}| */
} ld_pdf_plan_in;

typedef struct {
    int32_t status, L;                              /* as ld_plan_out */
    uint64_t dn[LD_MAX_LEVELS];
    double V[LD_MAX_LEVELS];                        /* max_i Var[Y_{l,i}] */
    double estimate[LD_MAX_BINS];                   /* sum_l Yhat_{l,i} */
    double bias_est, stat_var, alpha;               /* maxima over the bins */
} ld_pdf_plan_out;

int mlmc_plan_pdf(const ld_pdf_plan_in* in, ld_pdf_plan_out* out);

typedef enum LD_ENUM_BASE { LD_MLMC = 0, LD_STMC = 1 } ld_estimator;

typedef struct {
    double estimate[LD_MAX_BINS];   /* E[P_i(X_T)] per bin */
    double bias_est, stat_var, rmse_est;
    int32_t L, iterations, status, estimator;
    uint64_t N[LD_MAX_LEVELS];      /* samples per level (StMC: N[0] on level L) */
    uint64_t n_nonfinite;
    double V[LD_MAX_LEVELS];        /* max_i Var[Y_{l,i}] (StMC: max_i Var[P_i]) */
    double fine_steps;              /* coupled (StMC: single) particle-steps drawn */
    double wall_seconds;
    double device_seconds;          /* path and bins kernels (HIP events) */
} ld_pdf_result;

/* Binned-concentration estimate to absolute RMSE eps per bin. LD_MLMC: the adaptive
   driver of mlmc_estimate with mlmc_plan_pdf's decisions (opts.eps_is_relative must
   be 0). LD_STMC: standard Monte Carlo (Sec. 3.2) on the single fine path of step
   T / (M0 2^L), L = opts.fixed_L (>= 0): opts.N_init samples, then
   N = ceil(2 max_i Var[P_i] / eps^2), topped up while that exceeds the samples drawn
   by more than 1 %. Blocks until done. opts.d_workspace: a caller-owned DEVICE buffer
   of at least mlmc_estimate_pdf_workspace(bins->n_bins) bytes (opts.workspace_bytes;
   LD_ENOMEM if smaller), used on opts.hip_stream; NULL: the call allocates and frees
   its own. */
int mlmc_estimate_pdf(double eps, const ld_bins* bins, const ld_qoi* qoi,
                      ld_integrator integrator, const ld_profile* profile,
                      const ld_estimate_opts* opts, ld_estimator estimator,
                      ld_pdf_result* out);

/* Bytes of the device workspace mlmc_estimate_pdf uses for n_bins bins (0 if n_bins is
   outside 1..LD_MAX_BINS). */
size_t mlmc_estimate_pdf_workspace(int32_t n_bins);

/* ---- many estimators at once: the engine ---------------------------------------- */

/* The engine runs many independent MLMC estimates (queries) together. Each iteration
   gathers every active query's planned (level, sample range) pairs, cuts them into
   tiles (one block's work: 256 lanes x spl samples, or 64 samples in wave-specialised
   blocks for long paths), and runs all tiles of all queries in one persistent kernel
   per turbulence profile that takes tiles from a queue; the longest paths go first.
   The tile partials are reduced per range in a fixed order and added to running sums
   that stay in device memory (one ld_level_sums per query slot and level). After each
   iteration every query's planner (mlmc_plan) decides its next samples. A query's
   tiles and sums depend only on the query itself, so its result is bitwise the same
   run alone or mixed with others. Queries are admitted while slots and the HBM budget
   allow (LD_EBUSY otherwise), and leave when converged: continuous batching. */

#define LD_PENDING 2             /* ld_engine_result: the query is still running        */
#define LD_EBUSY (-7)            /* ld_engine_submit: no free slot within the HBM budget */

typedef struct ld_engine ld_engine;   /* opaque */

typedef struct {
    ld_precision precision;       /* path arithmetic of all queries */
    int32_t max_queries;          /* query slots (default 256) */
    size_t hbm_budget_bytes;      /* device memory the engine may use (default 1 GiB) */
    int32_t blocks_per_cu;        /* persistent grid = blocks_per_cu x CUs (default 8) */
    uint64_t target_tiles;        /* STREAM ranges are cut into at most this many tiles
                                     before lanes take several samples (default 32768) */
    uint64_t pipe_max_samples;    /* wave-specialised tiles for ranges up to this size
                                     (default 131072; 0 disables them) */
    uint32_t pipe_min_steps;      /* ... whose paths have at least this many steps (256) */
    int32_t use_graph;            /* capture an iteration's launches in a hipGraph (default 0:
                                     direct launches, whose persistent kernels get no more
                                     blocks than their queues have tiles) */
    void* hip_stream;             /* stream of all engine work (NULL = default) */
} ld_engine_opts;

/* One estimation request: mlmc_estimate's arguments. */
typedef struct {
    ld_problem problem;
    ld_integrator integrator;
    int32_t eps_is_relative;
    double eps;
    int32_t L_min, L_max, fixed_L, max_iter;
    uint64_t N_init;
    double alpha;
    double max_fine_steps;        /* cost budget as in ld_estimate_opts (0 = none) */
} ld_query;

void ld_engine_default_opts(ld_engine_opts* opts);
/* Allocates the engine's device buffers (within hbm_budget_bytes) on the current
   device. LD_EINVAL for bad options, LD_ENOMEM if the budget cannot hold one query. */
int ld_engine_create(const ld_engine_opts* opts, ld_engine** out);
void ld_engine_destroy(ld_engine* engine);
/* Admits a query (validated as mlmc_estimate would). *handle identifies it until
   ld_engine_release. LD_EBUSY: no free slot now; retry after queries finish. */
int ld_engine_submit(ld_engine* engine, const ld_query* query, int64_t* handle);
/* One MLMC iteration of every active query (blocks until its results are back).
   *n_active receives the number of queries still running afterwards. */
int ld_engine_step(ld_engine* engine, int32_t* n_active);
/* LD_PENDING while running; otherwise the query's final status (as mlmc_estimate) with
   out filled. wall_seconds = time from submission to completion. */
int ld_engine_result(ld_engine* engine, int64_t handle, ld_estimate_result* out);
/* Frees a finished query's slot. */
int ld_engine_release(ld_engine* engine, int64_t handle);
/* Device seconds of all iterations so far (HIP events), and their count. */
int ld_engine_stats(ld_engine* engine, double* device_seconds, int64_t* iterations,
                    double* fine_steps);

/* Runs n queries to completion on a live engine: submits them in order as slots free
   up, steps until every one has finished, fills out[0..n-1] and releases their handles;
   queries already admitted by the caller run along (their results stay for
   ld_engine_result). The queries are validated first (LD_EINVAL / LD_EUNSTABLE, nothing
   submitted). Returns the worst status of the n queries (an error, else a warning, else
   LD_OK); after an error the engine may still hold some of them. */
int ld_engine_run(ld_engine* engine, const ld_query* queries, int32_t n, ld_estimate_result* out);
/* Runs n queries to completion on one engine (submitting as slots free up) and fills
   out[0..n-1]. Returns the worst status. */
int mlmc_estimate_batch(const ld_query* queries, int32_t n, const ld_engine_opts* opts,
                        ld_estimate_result* out);

/* Autotuner: times the batch `queries` on engines with each candidate persistent grid
   (blocks_per_cu in {2, 4, 6, 8, 12, 16}) and tile policy (target_tiles in
   {4096, 8192, 16384, 32768, 65536}, wave-specialised tiles on/off, graph capture
   on/off), keeps the
   fastest, and writes it to *best (other fields from base). Each candidate gets one
   engine, created outside its timings; reps timings per candidate, the median counts. */
int ld_engine_autotune(const ld_query* queries, int32_t n, const ld_engine_opts* base,
                       int32_t reps, ld_engine_opts* best, double* best_seconds);

/* ---- serving: a request loop over the engine -------------------------------------- */

/* A server owns one engine and a worker thread. Clients submit queries from any
   thread; submission only validates and enqueues (it never waits for the device).
   The worker admits queued queries in arrival order whenever the engine has a free
   slot within its HBM budget, runs one engine iteration over all admitted queries,
   hands finished results to their tickets and frees their slots; queries that arrive
   while an iteration runs join at the next one (continuous batching). Each query's
   per-level running sums, and with them its next Philox sample index per level
   (n + n_nonfinite), stay in device memory until it finishes. Because a query's
   tiles and merges depend on the query alone, its result does not depend on the
   traffic it shared the device with.

   Policy LD_SERVE_FIFO is the plain comparison point: the worker takes one query at a
   time, in arrival order, through mlmc_estimate (no batching). */

enum { LD_SERVE_BATCH = 0, LD_SERVE_FIFO = 1 };

typedef struct ld_server ld_server;   /* opaque */

typedef struct {
    ld_engine_opts engine;        /* engine of LD_SERVE_BATCH; for LD_SERVE_FIFO only
                                     engine.precision is used */
    int32_t policy;               /* LD_SERVE_BATCH (default) or LD_SERVE_FIFO */
    int32_t max_queued;           /* submissions beyond this many waiting queries get
                                     LD_EBUSY (0 = no limit) */
} ld_server_opts;

/* Clock of the request times: seconds on a monotonic clock (steady, any origin). */
typedef struct {
    double t_submit;              /* ld_server_submit accepted the query */
    double t_admit;               /* the query got a slot (FIFO: its estimate started) */
    double t_done;                /* its result was ready */
} ld_request_times;

typedef struct {
    int64_t submitted, completed, queued, running;
    int64_t iterations;           /* engine iterations (FIFO: estimates) */
    int32_t max_running, max_queued;
    double busy_seconds;          /* worker wall time inside iterations / estimates */
    double device_seconds;        /* time inside the path kernels (HIP events) */
    double fine_steps;            /* coupled particle-steps of all finished work */
} ld_server_stats;

void ld_server_default_opts(ld_server_opts* opts);
/* Creates the engine (LD_SERVE_BATCH) or a workspace and stream (LD_SERVE_FIFO) on the
   current device and starts the worker thread. */
int ld_server_create(const ld_server_opts* opts, ld_server** out);
/* Stops the worker after its current iteration and frees everything; queries not yet
   collected are dropped. No other call on this server may run concurrently. */
void ld_server_destroy(ld_server* server);
/* Thread-safe. Validates the query (LD_EINVAL / LD_EUNSTABLE as mlmc_estimate) and
   enqueues it; *ticket identifies it for ld_server_wait. LD_EBUSY if max_queued
   queries are waiting; a stored error status if the worker has failed. */
int ld_server_submit(ld_server* server, const ld_query* query, int64_t* ticket);
/* Thread-safe. Waits up to timeout_s seconds (< 0: no limit, 0: poll) for the ticket's
   result. Returns LD_PENDING on timeout; otherwise the query's final status (as
   mlmc_estimate) with out (and times, if not NULL) filled, after which the ticket is
   gone. LD_EINVAL for an unknown ticket. */
int ld_server_wait(ld_server* server, int64_t ticket, double timeout_s, ld_estimate_result* out,
                   ld_request_times* times);
/* Thread-safe snapshot of the counters. */
int ld_server_stats_get(ld_server* server, ld_server_stats* out);
/* The clock of ld_request_times, for clients that time arrivals. */
double ld_server_clock(void);

/* ---- errors --------------------------------------------------------------------- */
const char* ld_strerror(int status);
/* Message of the last error on the calling thread ("" if none). */
const char* ld_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
