// host_common.hpp -- host-side helpers shared by the C ABI translation units.
#pragma once

#include <string>

#include "ld_internal.hpp"

namespace ldm {

// Blocks targeted per (level, range): enough to fill 256 CUs several times over so the
// tail of a launch is short, while each lane gets more samples as n grows. Adaptive
// steps use one resident round of blocks (5 per CU in FP32, 3 in FP64, as their register
// use allows) with as many samples per wave as that leaves: their paths differ in length,
// and a wave's tail is shorter relative to a longer chunk.
constexpr uint64_t kTargetBlocks = 32768;
constexpr uint64_t kAdaptiveTargetBlocksFp32 = 1280;
constexpr uint64_t kAdaptiveTargetBlocksFp64 = 768;

void set_error(const std::string& msg);
int fail(int status, const std::string& msg);

// Validates a problem; returns LD_OK or LD_EINVAL (message set).
int validate_problem(const ld_problem* p);
// True if drawing dn more samples (levels 0..L) on top of `drawn` would take the
// coupled fine steps sum_l N_l M0 2^l above max_fine_steps (> 0); false without a budget.
bool exceeds_budget(double max_fine_steps, int32_t M0, const uint64_t* drawn, const uint64_t* dn,
                    int32_t L);
// The decision step shared by mlmc_plan and mlmc_plan_pdf (driver.cpp): fills dn and
// *L_out from each level's variance Vl[0..in->L] (uses in->n, L, M0, L_max, fixed_L,
// N_init), returns the status (0 more samples, 1 converged, 2 stopped at L_max).
int decide(const ld_plan_in* in, const double* Vl, double bias, double eps_abs, uint64_t* dn,
           int32_t* L_out);
// Least-squares weak order from |Yhat_l|, l = 1..L, clamped to [0.5, 2] (1 if unfit).
double fit_alpha(const double* Yhat, int32_t L);
// Validates an engine query as mlmc_estimate validates its arguments (engine.cpp).
int validate_query(const ld_query* q);
// Symplectic Euler is stable only for lambda h < 2 (Sec. 3.1); returns LD_EUNSTABLE if
// a step of `level` violates it, else LD_OK.
int check_stability(const ld_problem* p, ld_integrator integ, int32_t level);
// Regularised sigma_U(x) of the profile (Eqs. 5, 7).
double sigma_u_at(const ld_profile& prof, double x);
// lambda_max over [0, H].
double lambda_max(const ld_profile& prof);
// lambda = 1/tau at x (regularised, Eqs. 5, 7).
double lambda_at(const ld_profile& prof, double x);

// Fills the kernel-side problem (FP64 parameters, smoothing coefficients).
int make_kproblem(const ld_problem* p, ld_integrator integ, KProblem* kp);

// Smoothing polynomial p_r of Eq. (35): coef[0..r+1], r in 1..8 (smoothing.cpp).
int smoothing_coefficients(int r, double* coef);

// Launch plan of one (level, range): samples per lane and block count.
void plan_item(uint64_t n_samples, uint32_t* spl, uint32_t* n_blocks, uint64_t target_blocks = kTargetBlocks);
// Upper bound of the blocks any level's range of n_samples uses (either block mode).
uint32_t max_blocks(uint64_t n_samples);

// Builds the items of a batch (most expensive level first), returns total blocks.
int build_batch(const ld_problem* p, ld_integrator integ, ld_precision prec,
                const ld_level_range* ranges, int32_t n_ranges, KArgs* args,
                uint32_t* total_blocks);

// Runs a batch: K1 + merge; d_out gets one ld_level_sums per range.
int run_batch(const ld_problem* p, ld_integrator integ, ld_precision prec,
              const ld_level_range* ranges, int32_t n_ranges, ld_level_sums* d_out,
              void* d_workspace, size_t workspace_bytes, double* d_dump, void* stream);

}  // namespace ldm
