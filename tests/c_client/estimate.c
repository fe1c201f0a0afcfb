/* A C client of libldmlmc: one adaptive MLMC estimate through the C ABI alone (no
 * Python, no PyTorch). Neutral boundary layer (kappa_sigma = 1.3, kappa_tau = 0.5,
 * u_* = 0.2 m/s, H = 1 km, eps_reg = 10 m), release at 500 m with U_0 ~ N(0, sigma_U^2),
 * T = 1000 s, M_0 = 40, E[Z(T)] to a relative RMSE given on the command line, BAOAB,
 * FP64 paths. Prints status, L, the estimate and N_l.
 *
 *   estimate <eps_rel> [fp32]
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ldmlmc.h"

int main(int argc, char** argv) {
    const double eps = argc > 1 ? atof(argv[1]) : 1e-2;
    ld_profile prof;
    memset(&prof, 0, sizeof prof);
    prof.kind = LD_PROFILE_NEUTRAL_BL;
    prof.H = 1000.0;
    prof.kappa_sigma = 1.3;
    prof.kappa_tau = 0.5;
    prof.u_star = 0.2;
    prof.eps_reg = 10.0;
    ld_qoi qoi;
    memset(&qoi, 0, sizeof qoi);
    qoi.kind = LD_QOI_MEAN_Z;
    ld_estimate_opts o;
    mlmc_estimate_default_opts(&o);
    o.release.kind = LD_RELEASE_GAUSSIAN_W;
    o.release.z0 = 500.0;
    o.T = 1000.0;
    o.M0 = 40;
    o.eps_is_relative = 1;
    o.N_init = 2000;
    o.L_max = 10;
    o.seed = 42;
    o.precision = (argc > 2 && strcmp(argv[2], "fp32") == 0) ? LD_FP32 : LD_FP64;
    ld_estimate_result r;
    const int rc = mlmc_estimate(eps, &qoi, LD_BAOAB, &prof, &o, &r);
    if (rc < 0) {
        fprintf(stderr, "mlmc_estimate: %s (%s)\n", ld_strerror(rc), ld_last_error());
        return 1;
    }
    printf("status %d L %d estimate %.17g rmse %.6g\nN", rc, r.L, r.estimate, r.rmse_est);
    for (int l = 0; l <= r.L; ++l) printf(" %llu", (unsigned long long)r.N[l]);
    printf("\n");
    return 0;
}
