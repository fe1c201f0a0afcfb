"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, factor or index, a
transposed operand) in a copy of oracle/oracle.c, builds it into a temporary library
on the CPU and runs the fast pin tests against it; every planted mistake must make
at least one pin fail. The oracle itself is never modified.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("drift drops the U^2 term", "return -0.5 * (d + u * u * d / (su * su));", "return -0.5 * d;"),
    ("drift sign", "- oracle_dVdX(p, x, u) * h + sigma", "+ oracle_dVdX(p, x, u) * h + sigma"),
    ("SE without damping", "(1.0 - lambda * h) * u", "u"),
    ("sigma without the factor 2", "*sigma = sqrt(2.0 * su * su / tau);", "*sigma = sqrt(su * su / tau);"),
    ("profile exponent", "pow(1.0 - xr / p->H, 0.75)", "pow(1.0 - xr / p->H, 0.5)"),
    ("no lower cut-off", "if (x < p->eps_reg) xr = p->eps_reg;", "if (x < 0.0) xr = 1e-9;"),
    ("tau without kappa_tau", "*tau = p->kappa_tau * xr / su;", "*tau = xr / su;"),
    ("GL O-step decay exp(-2 lambda h)",
     "double ustar = exp(-lambda * h) * u +", "double ustar = exp(-2.0 * lambda * h) * u +"),
    ("O-step amplitude without 1/(2 lambda)",
     "sqrt(-expm1(-2.0 * lambda * h) / (2.0 * lambda)) * noise;  /* O */\n    double u1",
     "sqrt(-expm1(-2.0 * lambda * h)) * noise;  /* O */\n    double u1"),
    ("BAOAB second A full step", "double x1 = xh + ustar * (h / 2.0);", "double x1 = xh + ustar * h;"),
    ("BAOAB O-step at X_n", "coefficients(p, xh, &lambda, &sigma);", "coefficients(p, x, &lambda, &sigma);"),
    ("BAOAB last B at X_{n+1/2}", "double u1 = ustar - oracle_dVdX(p, x1, ustar) * (h / 2.0);",
     "double u1 = ustar - oracle_dVdX(p, xh, ustar) * (h / 2.0);"),
    ("BAOAB noise sign before the mid fold",
     "    double noise = enter_noise(p, s, xi, noise_is_tilde, tilde);\n    double ustar = exp(-lambda * h) * uh",
     "    double noise = enter_noise(p, st[2], xi, noise_is_tilde, tilde);\n    double ustar = exp(-lambda * h) * uh"),
    ("fold keeps U", "        *u = -*u;\n        *s = -*s;", "        *s = -*s;"),
    ("fold keeps S", "        *u = -*u;\n        *s = -*s;", "        *u = -*u;"),
    ("top wall reflects to H - X", "*x = 2.0 * H - *x;", "*x = H - *x;"),
    ("SE coupling divides by 2", "xi_c = (tilde_a + tilde_b) / sqrt(2.0);", "xi_c = (tilde_a + tilde_b) / 2.0;"),
    ("GL coupling weight exp(-2 lambda h)", "double w = exp(-lam_a * h);", "double w = exp(-2.0 * lam_a * h);"),
    ("GL coupling normalisation", "sqrt(exp(-2.0 * lam_a * h) + 1.0)", "sqrt(exp(-lam_a * h) + 1.0)"),
    ("GL coupling operands transposed", "(w * tilde_a + tilde_b)", "(w * tilde_b + tilde_a)"),
    ("coarse step uses h", "oracle_step(p, 2.0 * h, coarse", "oracle_step(p, h, coarse"),
    ("coarse noise without S_c", "double physical = noise_is_tilde ? s * xi : xi;",
     "double physical = xi;"),
    ("h_l off by one step", "double h = p->T / (double)M;               /* h_l = T / M_l */",
     "double h = p->T / (double)(M + 1);"),
    ("Y_l = P_l + P_{l-1}", "double y = pf - pc;", "double y = pf + pc;"),
    ("Philox multipliers swapped",
     "uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;\n        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;",
     "uint64_t prod0 = (uint64_t)0xCD9E8D57u * (uint64_t)x0;\n        uint64_t prod1 = (uint64_t)0xD2511F53u * (uint64_t)x2;"),
    ("Philox nine rounds", "for (int round = 0; round < 10; ++round) {", "for (int round = 0; round < 9; ++round) {"),
    ("Philox key bumped before round 0", "if (round > 0) {", "if (round >= 0) {"),
    ("Philox output pairs swapped", "out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;",
     "out[0] = x2; out[1] = x3; out[2] = x0; out[3] = x1;"),
    ("Philox high halves not crossed", "uint32_t y0 = hi1 ^ x1 ^ k0;", "uint32_t y0 = hi0 ^ x1 ^ k0;"),
    ("uniform u from the low word first", "double u = uniform_open(r[1], r[0]);",
     "double u = uniform_open(r[0], r[1]);"),
    ("counter without the level", "((uint32_t)level & 0xFFu) | (p->stream_id << 8)};",
     "(p->stream_id << 8)};"),
    ("Box-Muller radius", "sqrt(-2.0 * log(u))", "sqrt(-log(u))"),
    ("Box-Muller pair both cosines", "out[1] = rho * sin(theta);", "out[1] = rho * cos(theta);"),
    ("Box-Muller angle pi v", "double theta = 2.0 * ORACLE_PI * v;", "double theta = ORACLE_PI * v;"),
    ("level-0 reuses one normal", "bad |= oracle_step(p, h, fine, z[k % 2], 0, &tilde_a, &lam_a);",
     "bad |= oracle_step(p, h, fine, z[0], 0, &tilde_a, &lam_a);"),
    ("Neumaier compensation sign", "*c += (*s - t) + x;", "*c += (*s - t) - x;"),
    ("variance rule factor 1", "double target = ceil(2.0 * total", "double target = ceil(1.0 * total"),
    ("smoothing moment sign", "a[2 + j][n] = ((j % 2 == 0) ? 1.0L : -1.0L)", "a[2 + j][n] = (1.0L)"),
    ("box indicator reversed", "return theta(x - p->qb) - theta(x - p->qa);",
     "return theta(x - p->qa) - theta(x - p->qb);"),
    ("adaptive coarse increment without S^(f)", "wc += (naive ? 1.0 : fine[2]) * dW;",
     "wc += dW;"),
    ("adaptive step ratio inverted", "double ratio = lam_adapt / lambda;",
     "double ratio = lambda / lam_adapt;"),
    ("adaptive coarse base step h", "ec = adaptive_end(p, lam_adapt, coarse[0], tc, 2 * tick_base",
     "ec = adaptive_end(p, lam_adapt, coarse[0], tc, tick_base"),
    ("adaptive increment without the square root", "z[j % 2] * sqrt((double)(next - tau) * tick)",
     "z[j % 2] * ((double)(next - tau) * tick)"),
    ("Gaussian release uses sigma_U(0)", "oracle_profile(p, p->z0, &su, &tau);\n            oracle_normals",
     "oracle_profile(p, 0.0, &su, &tau);\n            oracle_normals"),
]

# Fast files first: a run stops at its first failing pin.
PIN_FILES = ["test_oracle_rng.py", "test_oracle_philox_independent.py", "test_oracle_model.py",
             "test_oracle_closed_forms.py", "test_oracle_adaptive.py",
             "test_oracle_smoothing_sums_driver.py", "test_oracle_paper_values.py",
             "test_oracle_coupling.py"]


def _run_mutant(args):
    name, old, new, tmp = args
    import oracle
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    mutated = src.replace(old, new, 1)
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    csrc = os.path.join(tmp, f"{tag}.c")
    lib = os.path.join(tmp, f"{tag}.so")
    with open(csrc, "w") as f:
        f.write(mutated)
    oracle.build(src=csrc, out=lib)
    env = dict(os.environ, LD_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not slow and not gpu",
           "-p", "no:cacheprovider"] + [os.path.join(ROOT, "tests", f) for f in PIN_FILES]
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    return name, r.returncode, r.stdout[-400:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=max(2, min(8, os.cpu_count() or 2))) as pool:
            results = list(pool.map(_run_mutant, [(n, o, w, tmp) for n, o, w in MUTANTS]))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    assert not survivors, "mistakes no pin caught: " + "; ".join(n for n, _ in survivors)
    # a failure must be a test failure (exit 1), not a crash of the harness
    assert all(rc == 1 for _, rc, _ in results), [(n, rc, out) for n, rc, out in results if rc != 1]
