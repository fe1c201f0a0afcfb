"""Python binding of libldmlmc (include/ldmlmc.h): argument marshalling only.

Every step of the method runs in the HIP library; this module converts workload dicts
(see workloads.py) to the C structs, takes device memory and the current stream from
PyTorch, and converts results back. If the library has not been built the import
still works but every call raises; there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# A run that checks the host code under sanitizers points this at its own build.
LIB_PATH = os.environ.get("LDMLMC_LIB", os.path.join(HERE, "libldmlmc.so"))
MAX_LEVELS = 32

LD_OK, LD_WARN_NOT_CONVERGED = 0, 1
LD_EINVAL, LD_EUNSTABLE, LD_ENOMEM, LD_EDEVICE, LD_ENONFINITE, LD_ENODEVICE = -1, -2, -3, -4, -5, -6

INTEGRATORS = {"SE": 0, "GL": 1, "BAOAB": 2}
PRECISIONS = {"fp64": 0, "fp32": 1}
PROFILES = {"homogeneous": 0, "neutral": 1}
RELEASES = {"fixed": 0, "gaussian": 1, "well_mixed": 2}
QOIS = {"mean_z": 0, "p_above": 1, "p_box": 2, "velocity": 3, "velocity_sq": 4}

EXPORTED = ["mlmc_level_sums_workspace", "mlmc_level_sums", "mlmc_level_sums_noalloc",
            "mlmc_level_sums_batch_workspace",
            "mlmc_level_sums_batch", "mlmc_level_samples", "mlmc_plan",
            "mlmc_estimate_default_opts", "mlmc_estimate_workspace", "mlmc_estimate",
            "ld_engine_default_opts", "ld_engine_create", "ld_engine_destroy", "ld_engine_submit",
            "ld_engine_step", "ld_engine_result", "ld_engine_release", "ld_engine_stats",
            "ld_engine_run",
            "mlmc_pdf_level_sums_workspace", "mlmc_pdf_level_sums", "mlmc_plan_pdf",
            "mlmc_estimate_pdf", "mlmc_estimate_pdf_workspace",
            "mlmc_estimate_batch", "ld_engine_autotune",
            "ld_server_default_opts", "ld_server_create", "ld_server_destroy", "ld_server_submit",
            "ld_server_wait", "ld_server_stats_get", "ld_server_clock",
            "ld_strerror", "ld_last_error"]
SERVE_POLICIES = {"batch": 0, "fifo": 1}
LD_PENDING, LD_EBUSY = 2, -7


class LdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ldmlmc status {status}: {message}")
        self.status = status


class Profile(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("H", C.c_double),
                ("sigma_u", C.c_double), ("tau", C.c_double), ("kappa_sigma", C.c_double),
                ("kappa_tau", C.c_double), ("u_star", C.c_double), ("eps_reg", C.c_double)]


class Qoi(C.Structure):
    _fields_ = [("kind", C.c_int32), ("r", C.c_int32), ("a", C.c_double), ("b", C.c_double),
                ("delta", C.c_double)]


class Release(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("z0", C.c_double),
                ("w0", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("profile", Profile), ("release", Release), ("qoi", Qoi), ("T", C.c_double),
                ("M0", C.c_int32), ("stream_id", C.c_uint32), ("seed", C.c_uint64),
                ("x_adapt", C.c_double)]


class LevelSums(C.Structure):
    _fields_ = [("s", C.c_double * 4), ("c", C.c_double * 4), ("n", C.c_uint64),
                ("n_nonfinite", C.c_uint64)]


class LevelRange(C.Structure):
    _fields_ = [("level", C.c_int32), ("reserved", C.c_int32), ("sample_begin", C.c_uint64),
                ("n_samples", C.c_uint64)]


class PlanIn(C.Structure):
    _fields_ = [("L", C.c_int32), ("M0", C.c_int32), ("n", C.c_uint64 * MAX_LEVELS),
                ("sum1", C.c_double * MAX_LEVELS), ("sum2", C.c_double * MAX_LEVELS),
                ("eps", C.c_double), ("alpha", C.c_double), ("eps_is_relative", C.c_int32),
                ("L_max", C.c_int32), ("fixed_L", C.c_int32), ("fixed_N", C.c_int32),
                ("N_init", C.c_uint64)]


class PlanOut(C.Structure):
    _fields_ = [("status", C.c_int32), ("L", C.c_int32), ("dn", C.c_uint64 * MAX_LEVELS),
                ("Yhat", C.c_double * MAX_LEVELS), ("V", C.c_double * MAX_LEVELS),
                ("estimate", C.c_double), ("eps_abs", C.c_double), ("alpha", C.c_double),
                ("bias_est", C.c_double), ("stat_var", C.c_double)]


class EstimateOpts(C.Structure):
    _fields_ = [("release", Release), ("T", C.c_double), ("M0", C.c_int32),
                ("L_min", C.c_int32), ("L_max", C.c_int32), ("fixed_L", C.c_int32),
                ("fixed_N", C.c_int32), ("eps_is_relative", C.c_int32), ("N_init", C.c_uint64),
                ("alpha", C.c_double), ("precision", C.c_int32), ("stream_id", C.c_uint32),
                ("seed", C.c_uint64), ("max_iter", C.c_int32), ("early_topup", C.c_int32),
                ("x_adapt", C.c_double), ("max_fine_steps", C.c_double),
                ("d_workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("hip_stream", C.c_void_p)]


class EstimateResult(C.Structure):
    _fields_ = [("estimate", C.c_double), ("eps_abs", C.c_double), ("bias_est", C.c_double),
                ("stat_var", C.c_double), ("rmse_est", C.c_double), ("alpha", C.c_double),
                ("L", C.c_int32), ("iterations", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32), ("N", C.c_uint64 * MAX_LEVELS),
                ("n_nonfinite", C.c_uint64), ("Yhat", C.c_double * MAX_LEVELS),
                ("V", C.c_double * MAX_LEVELS), ("fine_steps", C.c_double),
                ("integrator_steps", C.c_double), ("wall_seconds", C.c_double),
                ("device_seconds", C.c_double), ("launches", C.c_int32),
                ("reserved2", C.c_int32)]


class EngineOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_queries", C.c_int32),
                ("hbm_budget_bytes", C.c_size_t), ("blocks_per_cu", C.c_int32),
                ("target_tiles", C.c_uint64), ("pipe_max_samples", C.c_uint64),
                ("pipe_min_steps", C.c_uint32), ("use_graph", C.c_int32),
                ("hip_stream", C.c_void_p)]


class Query(C.Structure):
    _fields_ = [("problem", Problem), ("integrator", C.c_int32), ("eps_is_relative", C.c_int32),
                ("eps", C.c_double), ("L_min", C.c_int32), ("L_max", C.c_int32),
                ("fixed_L", C.c_int32), ("max_iter", C.c_int32), ("N_init", C.c_uint64),
                ("alpha", C.c_double), ("max_fine_steps", C.c_double)]


MAX_BINS = 64
ESTIMATORS = {"mlmc": 0, "stmc": 1}


class Bins(C.Structure):
    _fields_ = [("a0", C.c_double), ("width", C.c_double), ("n_bins", C.c_int32),
                ("reserved", C.c_int32)]


class PdfPlanIn(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_bins", C.c_int32), ("n", C.c_uint64 * MAX_LEVELS),
                ("sum1", (C.c_double * MAX_BINS) * MAX_LEVELS),
                ("sum2", (C.c_double * MAX_BINS) * MAX_LEVELS),
                ("M0", C.c_int32), ("L_max", C.c_int32), ("eps", C.c_double),
                ("fixed_L", C.c_int32), ("reserved", C.c_int32), ("N_init", C.c_uint64),
                ("alpha", C.c_double)]


class PdfPlanOut(C.Structure):
    _fields_ = [("status", C.c_int32), ("L", C.c_int32), ("dn", C.c_uint64 * MAX_LEVELS),
                ("V", C.c_double * MAX_LEVELS), ("estimate", C.c_double * MAX_BINS),
                ("bias_est", C.c_double), ("stat_var", C.c_double), ("alpha", C.c_double)]


class PdfResult(C.Structure):
    _fields_ = [("estimate", C.c_double * MAX_BINS), ("bias_est", C.c_double),
                ("stat_var", C.c_double), ("rmse_est", C.c_double), ("L", C.c_int32),
                ("iterations", C.c_int32), ("status", C.c_int32), ("estimator", C.c_int32),
                ("N", C.c_uint64 * MAX_LEVELS), ("n_nonfinite", C.c_uint64),
                ("V", C.c_double * MAX_LEVELS), ("fine_steps", C.c_double),
                ("wall_seconds", C.c_double), ("device_seconds", C.c_double)]


class ServerOpts(C.Structure):
    _fields_ = [("engine", EngineOpts), ("policy", C.c_int32), ("max_queued", C.c_int32)]


class RequestTimes(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("queued", C.c_int64),
                ("running", C.c_int64), ("iterations", C.c_int64), ("max_running", C.c_int32),
                ("max_queued", C.c_int32), ("busy_seconds", C.c_double),
                ("device_seconds", C.c_double), ("fine_steps", C.c_double)]


_lib = None


def load():
    """Load libldmlmc.so. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1612_07717_amd.build`")
    # PyTorch ships its own HIP runtime beside the system one this library links. One
    # process can use both only if PyTorch's brings the device up first (the other order
    # leaves PyTorch without a GPU), so it is initialised here, before the library can
    # make its first HIP call; without a GPU this does nothing.
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P, V = C.POINTER, C.c_void_p
    lib.mlmc_level_sums_workspace.argtypes = [C.c_uint64]
    lib.mlmc_level_sums_workspace.restype = C.c_size_t
    lib.mlmc_level_sums.argtypes = [P(Problem), C.c_int, C.c_int, C.c_int32, C.c_uint64,
                                    C.c_uint64, V, V, C.c_size_t, V]
    lib.mlmc_level_sums_noalloc.argtypes = [P(Problem), C.c_int, C.c_int, C.c_int32, C.c_uint64,
                                            C.c_uint64, V, V]
    lib.mlmc_level_sums_batch_workspace.argtypes = [P(LevelRange), C.c_int32]
    lib.mlmc_level_sums_batch_workspace.restype = C.c_size_t
    lib.mlmc_level_sums_batch.argtypes = [P(Problem), C.c_int, C.c_int, P(LevelRange),
                                          C.c_int32, V, V, C.c_size_t, V]
    lib.mlmc_level_samples.argtypes = [P(Problem), C.c_int, C.c_int, C.c_int32, C.c_uint64,
                                       C.c_uint64, V, V, C.c_size_t, V]
    lib.mlmc_plan.argtypes = [P(PlanIn), P(PlanOut)]
    lib.mlmc_estimate_default_opts.argtypes = [P(EstimateOpts)]
    lib.mlmc_estimate_default_opts.restype = None
    lib.mlmc_estimate_workspace.restype = C.c_size_t
    lib.mlmc_estimate.argtypes = [C.c_double, P(Qoi), C.c_int, P(Profile), P(EstimateOpts),
                                  P(EstimateResult)]
    lib.ld_strerror.argtypes = [C.c_int]
    lib.ld_strerror.restype = C.c_char_p
    lib.ld_last_error.restype = C.c_char_p
    lib.ld_engine_default_opts.argtypes = [P(EngineOpts)]
    lib.ld_engine_default_opts.restype = None
    lib.ld_engine_create.argtypes = [P(EngineOpts), P(C.c_void_p)]
    lib.ld_engine_destroy.argtypes = [C.c_void_p]
    lib.ld_engine_destroy.restype = None
    lib.ld_engine_submit.argtypes = [C.c_void_p, P(Query), P(C.c_int64)]
    lib.ld_engine_step.argtypes = [C.c_void_p, P(C.c_int32)]
    lib.ld_engine_result.argtypes = [C.c_void_p, C.c_int64, P(EstimateResult)]
    lib.ld_engine_release.argtypes = [C.c_void_p, C.c_int64]
    lib.ld_engine_stats.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int64), P(C.c_double)]
    lib.mlmc_estimate_batch.argtypes = [P(Query), C.c_int32, P(EngineOpts), P(EstimateResult)]
    lib.ld_engine_run.argtypes = [C.c_void_p, P(Query), C.c_int32, P(EstimateResult)]
    lib.ld_engine_autotune.argtypes = [P(Query), C.c_int32, P(EngineOpts), C.c_int32,
                                       P(EngineOpts), P(C.c_double)]
    lib.mlmc_pdf_level_sums_workspace.argtypes = [C.c_uint64, C.c_int32]
    lib.mlmc_pdf_level_sums_workspace.restype = C.c_size_t
    lib.mlmc_pdf_level_sums.argtypes = [P(Problem), C.c_int, C.c_int, C.c_int32, C.c_uint64,
                                        C.c_uint64, P(Bins), V, V, C.c_size_t, V]
    lib.mlmc_plan_pdf.argtypes = [P(PdfPlanIn), P(PdfPlanOut)]
    lib.mlmc_estimate_pdf.argtypes = [C.c_double, P(Bins), P(Qoi), C.c_int, P(Profile),
                                      P(EstimateOpts), C.c_int, P(PdfResult)]
    lib.mlmc_estimate_pdf_workspace.argtypes = [C.c_int32]
    lib.mlmc_estimate_pdf_workspace.restype = C.c_size_t
    lib.ld_server_default_opts.argtypes = [P(ServerOpts)]
    lib.ld_server_default_opts.restype = None
    lib.ld_server_create.argtypes = [P(ServerOpts), P(C.c_void_p)]
    lib.ld_server_destroy.argtypes = [C.c_void_p]
    lib.ld_server_destroy.restype = None
    lib.ld_server_submit.argtypes = [C.c_void_p, P(Query), P(C.c_int64)]
    lib.ld_server_wait.argtypes = [C.c_void_p, C.c_int64, C.c_double, P(EstimateResult),
                                   P(RequestTimes)]
    lib.ld_server_stats_get.argtypes = [C.c_void_p, P(ServerStats)]
    lib.ld_server_clock.restype = C.c_double
    _lib = lib
    return lib


def _check(rc: int, ok=(LD_OK,)) -> int:
    if rc not in ok:
        lib = load()
        raise LdError(rc, f"{lib.ld_strerror(rc).decode()}: {lib.ld_last_error().decode()}")
    return rc


# ----------------------------------------------------------------------------- structs
def make_profile(cfg: dict) -> Profile:
    return Profile(kind=PROFILES[cfg["profile"]], H=cfg["H"], sigma_u=cfg["sigma_u"],
                   tau=cfg["tau"], kappa_sigma=cfg["kappa_sigma"], kappa_tau=cfg["kappa_tau"],
                   u_star=cfg["u_star"], eps_reg=cfg["eps_reg"])


def make_qoi(cfg: dict) -> Qoi:
    return Qoi(kind=QOIS[cfg["qoi"]], r=int(cfg["r"]), a=cfg["qa"], b=cfg["qb"],
               delta=cfg["delta"])


def make_release(cfg: dict) -> Release:
    return Release(kind=RELEASES[cfg["release"]], z0=cfg["z0"], w0=cfg["w0"])


def make_problem(cfg: dict) -> Problem:
    if cfg.get("coupling", "reflected") != "reflected":
        raise ValueError("the library implements the reflection-aware coupling only")
    return Problem(profile=make_profile(cfg), release=make_release(cfg), qoi=make_qoi(cfg),
                   T=cfg["T"], M0=int(cfg["M0"]), stream_id=int(cfg["stream_id"]),
                   seed=int(cfg["seed"]), x_adapt=float(cfg.get("x_adapt", 0.0)))


def sums_to_dict(s: LevelSums) -> dict:
    v = [s.s[k] + s.c[k] for k in range(4)]
    return {"sum_y": v[0], "sum_y2": v[1], "sum_pf": v[2], "sum_pf2": v[3],
            "s": list(s.s), "c": list(s.c), "n": int(s.n), "n_nonfinite": int(s.n_nonfinite)}


# ------------------------------------------------------------------------- device calls
def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible to PyTorch")
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def level_sums_workspace(n: int) -> int:
    return int(load().mlmc_level_sums_workspace(int(n)))


def level_sums_async(cfg, level, begin, n, out, workspace, precision="fp64", stream=None):
    """Enqueue mlmc_level_sums into torch tensors: `out` >= 80 bytes, `workspace` >=
    level_sums_workspace(n) bytes (both CUDA tensors). Does not synchronise."""
    lib = load()
    p = make_problem(cfg)
    _check(lib.mlmc_level_sums(C.byref(p), INTEGRATORS[cfg["integrator"]], PRECISIONS[precision],
                               int(level), int(begin), int(n), C.c_void_p(out.data_ptr()),
                               C.c_void_p(workspace.data_ptr()),
                               workspace.numel() * workspace.element_size(), _stream_handle(stream)))


def _sums_from_tensor(t) -> dict:
    raw = t.detach().cpu().contiguous().view(-1).numpy().view(np.uint8)[: C.sizeof(LevelSums)]
    return sums_to_dict(LevelSums.from_buffer_copy(raw.tobytes()))


def level_sums(cfg, level, begin, n, precision="fp64", stream=None) -> dict:
    torch = _torch()
    out = torch.zeros(C.sizeof(LevelSums), dtype=torch.uint8, device="cuda")
    ws = torch.empty(max(level_sums_workspace(n), 1), dtype=torch.uint8, device="cuda")
    level_sums_async(cfg, level, begin, n, out, ws, precision, stream)
    torch.cuda.synchronize()
    return _sums_from_tensor(out)


def level_sums_noalloc_async(cfg, level, begin, n, out, precision="fp64", stream=None):
    """Enqueue mlmc_level_sums_noalloc into the CUDA tensor `out` (>= 80 bytes): no
    workspace, the library's own partials array. Does not synchronise."""
    lib = load()
    p = make_problem(cfg)
    _check(lib.mlmc_level_sums_noalloc(C.byref(p), INTEGRATORS[cfg["integrator"]], PRECISIONS[precision],
                                       int(level), int(begin), int(n), C.c_void_p(out.data_ptr()),
                                       _stream_handle(stream)))


def level_sums_noalloc(cfg, level, begin, n, precision="fp64", stream=None) -> dict:
    torch = _torch()
    out = torch.zeros(C.sizeof(LevelSums), dtype=torch.uint8, device="cuda")
    level_sums_noalloc_async(cfg, level, begin, n, out, precision, stream)
    torch.cuda.synchronize()
    return _sums_from_tensor(out)


def level_sums_batch(cfg, ranges, precision="fp64", stream=None) -> list:
    """ranges: list of (level, begin, n). Returns one sums dict per range."""
    torch = _torch()
    lib = load()
    arr = (LevelRange * len(ranges))(*[LevelRange(level=l, sample_begin=b, n_samples=n)
                                       for l, b, n in ranges])
    need = int(lib.mlmc_level_sums_batch_workspace(arr, len(ranges)))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    out = torch.zeros(C.sizeof(LevelSums) * len(ranges), dtype=torch.uint8, device="cuda")
    p = make_problem(cfg)
    _check(lib.mlmc_level_sums_batch(C.byref(p), INTEGRATORS[cfg["integrator"]],
                                     PRECISIONS[precision], arr, len(ranges),
                                     C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()),
                                     ws.numel(), _stream_handle(stream)))
    torch.cuda.synchronize()
    raw = out.cpu().numpy().tobytes()
    size = C.sizeof(LevelSums)
    return [sums_to_dict(LevelSums.from_buffer_copy(raw[i * size:(i + 1) * size]))
            for i in range(len(ranges))]


def level_samples(cfg, level, begin, n, precision="fp64", stream=None) -> np.ndarray:
    """Per-sample (P_l, P_{l-1}) in FP64, shape (n, 2)."""
    torch = _torch()
    lib = load()
    out = torch.empty((max(n, 1), 2), dtype=torch.float64, device="cuda")
    ws = torch.empty(max(level_sums_workspace(n), 1), dtype=torch.uint8, device="cuda")
    p = make_problem(cfg)
    _check(lib.mlmc_level_samples(C.byref(p), INTEGRATORS[cfg["integrator"]],
                                  PRECISIONS[precision], int(level), int(begin), int(n),
                                  C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream_handle(stream)))
    torch.cuda.synchronize()
    return out[:n].cpu().numpy()


def estimate_opts(cfg, *, precision="fp64", L_min=2, L_max=20, fixed_L=-1, fixed_N=False,
                  N_init=10000, eps_is_relative=False, alpha=1.0, max_iter=100,
                  max_fine_steps=0.0, early_topup=False, workspace=None, stream=None) -> EstimateOpts:
    o = EstimateOpts()
    load().mlmc_estimate_default_opts(C.byref(o))
    o.release = make_release(cfg)
    o.T = cfg["T"]
    o.M0 = int(cfg["M0"])
    o.L_min, o.L_max, o.fixed_L, o.fixed_N = L_min, L_max, fixed_L, int(bool(fixed_N))
    o.eps_is_relative = int(bool(eps_is_relative))
    o.N_init = int(N_init)
    o.alpha = float(alpha)
    o.precision = PRECISIONS[precision]
    o.stream_id = int(cfg["stream_id"])
    o.seed = int(cfg["seed"])
    o.max_iter = int(max_iter)
    o.max_fine_steps = float(max_fine_steps)
    o.early_topup = int(bool(early_topup))
    o.x_adapt = float(cfg.get("x_adapt", 0.0))
    if workspace is not None:
        o.d_workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if stream is not None or workspace is not None:
        o.hip_stream = _stream_handle(stream).value
    return o


def estimate_workspace_bytes() -> int:
    return int(load().mlmc_estimate_workspace())


def estimate(eps, cfg, **kw) -> dict:
    """mlmc_estimate(eps, qoi, integrator, profile) with options from cfg and kw. Without
    a workspace, one comes from PyTorch's caching allocator on the current stream, so
    repeated calls do not each allocate and free it on the device (mlmc_estimate returns
    only after its work on that stream is done)."""
    lib = load()
    if kw.get("workspace") is None:
        import torch
        if torch.cuda.is_available():   # else the library reports the missing device itself
            kw["workspace"] = torch.empty(estimate_workspace_bytes(), dtype=torch.uint8, device="cuda")
    o = estimate_opts(cfg, **kw)
    r = EstimateResult()
    q, prof = make_qoi(cfg), make_profile(cfg)
    rc = lib.mlmc_estimate(float(eps), C.byref(q), INTEGRATORS[cfg["integrator"]],
                           C.byref(prof), C.byref(o), C.byref(r))
    _check(rc, ok=(LD_OK, LD_WARN_NOT_CONVERGED, LD_ENONFINITE))
    L = r.L
    return {"rc": rc, "estimate": r.estimate, "eps_abs": r.eps_abs, "bias_est": r.bias_est,
            "stat_var": r.stat_var, "rmse_est": r.rmse_est, "alpha": r.alpha, "L": L,
            "iterations": r.iterations, "status": r.status,
            "N": [int(r.N[l]) for l in range(L + 1)], "n_nonfinite": int(r.n_nonfinite),
            "Yhat": list(r.Yhat[: L + 1]), "V": list(r.V[: L + 1]),
            "fine_steps": r.fine_steps, "integrator_steps": r.integrator_steps,
            "wall_seconds": r.wall_seconds, "device_seconds": r.device_seconds,
            "launches": r.launches}


# --------------------------------------------------------------------------- host only
def plan(d: dict) -> dict:
    """mlmc_plan: one decision of the adaptive algorithm (host only, no GPU)."""
    pin = PlanIn()
    pin.L = d["L"]
    pin.M0 = d["M0"]
    for l, v in enumerate(d["n"]):
        pin.n[l] = int(v)
    for l, v in enumerate(d["sum1"]):
        pin.sum1[l] = float(v)
    for l, v in enumerate(d["sum2"]):
        pin.sum2[l] = float(v)
    pin.eps = d["eps"]
    pin.alpha = d.get("alpha", 1.0)
    pin.eps_is_relative = int(d.get("eps_is_relative", 0))
    pin.L_max = d.get("L_max", 20)
    pin.fixed_L = d.get("fixed_L", -1)
    pin.fixed_N = int(d.get("fixed_N", 0))
    pin.N_init = d.get("N_init", 10000)
    out = PlanOut()
    _check(load().mlmc_plan(C.byref(pin), C.byref(out)))
    Lp = out.L
    return {"status": out.status, "L": Lp, "dn": [int(out.dn[l]) for l in range(Lp + 1)],
            "Yhat": list(out.Yhat[: d["L"] + 1]), "V": list(out.V[: d["L"] + 1]),
            "estimate": out.estimate, "eps_abs": out.eps_abs, "alpha": out.alpha,
            "bias_est": out.bias_est, "stat_var": out.stat_var}


# ------------------------------------------------------------------------- the engine
def _result_dict(r: EstimateResult, rc: int) -> dict:
    L = r.L
    return {"rc": rc, "estimate": r.estimate, "eps_abs": r.eps_abs, "bias_est": r.bias_est,
            "stat_var": r.stat_var, "rmse_est": r.rmse_est, "alpha": r.alpha, "L": L,
            "iterations": r.iterations, "status": r.status,
            "N": [int(r.N[l]) for l in range(L + 1)], "n_nonfinite": int(r.n_nonfinite),
            "Yhat": list(r.Yhat[: L + 1]), "V": list(r.V[: L + 1]),
            "fine_steps": r.fine_steps, "integrator_steps": r.integrator_steps,
            "wall_seconds": r.wall_seconds, "device_seconds": r.device_seconds,
            "launches": r.launches}


def make_query(cfg: dict, eps: float, *, eps_is_relative=True, L_min=2, L_max=20, fixed_L=-1,
               N_init=10000, alpha=1.0, max_iter=100, max_fine_steps=0.0) -> Query:
    return Query(problem=make_problem(cfg), integrator=INTEGRATORS[cfg["integrator"]],
                 eps_is_relative=int(bool(eps_is_relative)), eps=float(eps), L_min=L_min,
                 L_max=L_max, fixed_L=fixed_L, max_iter=max_iter, N_init=int(N_init),
                 alpha=float(alpha), max_fine_steps=float(max_fine_steps))


def engine_opts(*, precision="fp32", max_queries=256, hbm_budget_bytes=1 << 30, blocks_per_cu=8,
                target_tiles=32768, pipe_max_samples=64 * 2048, pipe_min_steps=256,
                use_graph=False, stream=None) -> EngineOpts:
    o = EngineOpts()
    load().ld_engine_default_opts(C.byref(o))
    o.precision = PRECISIONS[precision]
    o.max_queries = int(max_queries)
    o.hbm_budget_bytes = int(hbm_budget_bytes)
    o.blocks_per_cu = int(blocks_per_cu)
    o.target_tiles = int(target_tiles)
    o.pipe_max_samples = int(pipe_max_samples)
    o.pipe_min_steps = int(pipe_min_steps)
    o.use_graph = int(bool(use_graph))
    if stream is not None:
        o.hip_stream = _stream_handle(stream).value
    return o


class Engine:
    """ld_engine: submit queries, step MLMC iterations of all of them, read results."""

    def __init__(self, opts: EngineOpts | None = None, **kw):
        _torch()
        self._lib = load()
        self._opts = opts if opts is not None else engine_opts(**kw)
        h = C.c_void_p()
        _check(self._lib.ld_engine_create(C.byref(self._opts), C.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            self._lib.ld_engine_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, query: Query):
        """Handle of the admitted query, or None if no slot is free (LD_EBUSY)."""
        h = C.c_int64()
        rc = self._lib.ld_engine_submit(self._h, C.byref(query), C.byref(h))
        if rc == LD_EBUSY:
            return None
        _check(rc)
        return int(h.value)

    def step(self) -> int:
        n = C.c_int32()
        _check(self._lib.ld_engine_step(self._h, C.byref(n)))
        return int(n.value)

    def result(self, handle: int):
        """Result dict once finished, None while pending."""
        r = EstimateResult()
        rc = self._lib.ld_engine_result(self._h, int(handle), C.byref(r))
        if rc == LD_PENDING:
            return None
        _check(rc, ok=(LD_OK, LD_WARN_NOT_CONVERGED, LD_ENONFINITE))
        return _result_dict(r, rc)

    def release(self, handle: int):
        _check(self._lib.ld_engine_release(self._h, int(handle)))

    def run(self, queries: list) -> list:
        """ld_engine_run: the queries to completion on this engine (submitted as slots free
        up), their result dicts in order."""
        arr = (Query * len(queries))(*queries)
        res = (EstimateResult * len(queries))()
        rc = self._lib.ld_engine_run(self._h, arr, len(queries), res)
        _check(rc, ok=(LD_OK, LD_WARN_NOT_CONVERGED, LD_ENONFINITE))
        return [_result_dict(r, r.status) for r in res]

    def stats(self) -> dict:
        d, it, fs = C.c_double(), C.c_int64(), C.c_double()
        _check(self._lib.ld_engine_stats(self._h, C.byref(d), C.byref(it), C.byref(fs)))
        return {"device_seconds": d.value, "iterations": int(it.value), "fine_steps": fs.value}


def estimate_batch(queries: list, opts: EngineOpts | None = None, **kw) -> list:
    """mlmc_estimate_batch: all queries to completion on one engine."""
    _torch()
    lib = load()
    o = opts if opts is not None else engine_opts(**kw)
    arr = (Query * len(queries))(*queries)
    res = (EstimateResult * len(queries))()
    rc = lib.mlmc_estimate_batch(arr, len(queries), C.byref(o), res)
    _check(rc, ok=(LD_OK, LD_WARN_NOT_CONVERGED, LD_ENONFINITE))
    return [_result_dict(r, r.status) for r in res]


def autotune(queries: list, base: EngineOpts | None = None, reps: int = 2, **kw):
    """ld_engine_autotune: the fastest engine options for this batch, and its time."""
    _torch()
    lib = load()
    b = base if base is not None else engine_opts(**kw)
    arr = (Query * len(queries))(*queries)
    best = EngineOpts()
    t = C.c_double()
    _check(lib.ld_engine_autotune(arr, len(queries), C.byref(b), int(reps), C.byref(best), C.byref(t)))
    return best, t.value


def opts_dict(o: EngineOpts) -> dict:
    return {"precision": "fp32" if o.precision == 1 else "fp64", "max_queries": o.max_queries,
            "hbm_budget_bytes": o.hbm_budget_bytes, "blocks_per_cu": o.blocks_per_cu,
            "target_tiles": o.target_tiles, "pipe_max_samples": o.pipe_max_samples,
            "pipe_min_steps": o.pipe_min_steps, "use_graph": bool(o.use_graph)}


def make_bins(a0: float, width: float, n_bins: int) -> Bins:
    return Bins(a0=float(a0), width=float(width), n_bins=int(n_bins), reserved=0)


def pdf_level_sums(cfg, level, begin, n, a0, width, n_bins, precision="fp64", stream=None) -> list:
    """mlmc_pdf_level_sums: per-bin sums of the binned concentration (Sec. 6.4)."""
    torch = _torch()
    lib = load()
    ws = torch.empty(max(1, lib.mlmc_pdf_level_sums_workspace(n, n_bins)), dtype=torch.uint8, device="cuda")
    out = torch.zeros(n_bins * C.sizeof(LevelSums), dtype=torch.uint8, device="cuda")
    b = make_bins(a0, width, n_bins)
    _check(lib.mlmc_pdf_level_sums(C.byref(make_problem(cfg)), INTEGRATORS[cfg["integrator"]],
                                   PRECISIONS[precision], level, begin, n, C.byref(b),
                                   C.c_void_p(out.data_ptr()), C.c_void_p(ws.data_ptr()),
                                   ws.numel(), _stream_handle(stream)))
    torch.cuda.synchronize()
    raw = out.cpu().numpy().tobytes()
    sz = C.sizeof(LevelSums)
    return [sums_to_dict(LevelSums.from_buffer_copy(raw[i * sz:(i + 1) * sz])) for i in range(n_bins)]


def pdf_plan(d: dict) -> dict:
    """mlmc_plan_pdf (host only)."""
    pin = PdfPlanIn()
    pin.L, pin.n_bins = d["L"], d["n_bins"]
    for l in range(d["L"] + 1):
        pin.n[l] = int(d["n"][l])
        for i in range(d["n_bins"]):
            pin.sum1[l][i] = d["sum1"][l][i]
            pin.sum2[l][i] = d["sum2"][l][i]
    pin.M0, pin.eps, pin.L_max = d["M0"], d["eps"], d.get("L_max", 20)
    pin.fixed_L, pin.N_init, pin.alpha = d.get("fixed_L", -1), d.get("N_init", 10000), d.get("alpha", 1.0)
    out = PdfPlanOut()
    _check(load().mlmc_plan_pdf(C.byref(pin), C.byref(out)))
    L = out.L
    return {"status": out.status, "L": L, "dn": [int(out.dn[l]) for l in range(L + 1)],
            "V": list(out.V[: d["L"] + 1]), "estimate": list(out.estimate[: d["n_bins"]]),
            "bias_est": out.bias_est, "stat_var": out.stat_var, "alpha": out.alpha}


def estimate_pdf(eps, cfg, a0, width, n_bins, *, estimator="mlmc", stream=None, **kw) -> dict:
    """mlmc_estimate_pdf: binned concentration to absolute RMSE eps per bin. Without a
    workspace, one comes from PyTorch's caching allocator on the current stream."""
    torch = _torch()
    lib = load()
    kw.setdefault("eps_is_relative", False)
    if kw.get("workspace") is None:
        kw["workspace"] = torch.empty(int(lib.mlmc_estimate_pdf_workspace(int(n_bins))),
                                      dtype=torch.uint8, device="cuda")
    o = estimate_opts(cfg, stream=stream, **kw)
    r = PdfResult()
    b = make_bins(a0, width, n_bins)
    q, prof = make_qoi(cfg), make_profile(cfg)
    rc = lib.mlmc_estimate_pdf(float(eps), C.byref(b), C.byref(q), INTEGRATORS[cfg["integrator"]],
                               C.byref(prof), C.byref(o), ESTIMATORS[estimator], C.byref(r))
    _check(rc, ok=(LD_OK, LD_WARN_NOT_CONVERGED, LD_ENONFINITE))
    L = r.L
    nl = 1 if estimator == "stmc" else L + 1
    return {"rc": rc, "estimate": list(r.estimate[:n_bins]), "bias_est": r.bias_est,
            "stat_var": r.stat_var, "rmse_est": r.rmse_est, "L": L, "iterations": r.iterations,
            "status": r.status, "N": [int(r.N[l]) for l in range(nl)],
            "n_nonfinite": int(r.n_nonfinite), "V": list(r.V[:nl]), "fine_steps": r.fine_steps,
            "wall_seconds": r.wall_seconds, "device_seconds": r.device_seconds}


class Server:
    """ld_server: a worker thread that serves queries with continuous batching
    (policy "batch") or one at a time through mlmc_estimate (policy "fifo").
    submit() only enqueues; wait() blocks until a query's result is ready."""

    def __init__(self, policy="batch", max_queued=0, opts: EngineOpts | None = None, **kw):
        _torch()
        self._lib = load()
        so = ServerOpts()
        self._lib.ld_server_default_opts(C.byref(so))
        so.engine = opts if opts is not None else engine_opts(**kw)
        so.policy = SERVE_POLICIES[policy]
        so.max_queued = int(max_queued)
        h = C.c_void_p()
        _check(self._lib.ld_server_create(C.byref(so), C.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            self._lib.ld_server_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, query: Query):
        """Ticket of the enqueued query, or None if the admission queue is full."""
        t = C.c_int64()
        rc = self._lib.ld_server_submit(self._h, C.byref(query), C.byref(t))
        if rc == LD_EBUSY:
            return None
        _check(rc)
        return int(t.value)

    def wait(self, ticket: int, timeout: float | None = None):
        """(result dict, times dict) once finished; None if timeout (seconds) passed."""
        r, tm = EstimateResult(), RequestTimes()
        rc = self._lib.ld_server_wait(self._h, int(ticket), -1.0 if timeout is None else float(timeout),
                                      C.byref(r), C.byref(tm))
        if rc == LD_PENDING:
            return None
        _check(rc, ok=(LD_OK, LD_WARN_NOT_CONVERGED, LD_ENONFINITE))
        return _result_dict(r, rc), {"t_submit": tm.t_submit, "t_admit": tm.t_admit,
                                     "t_done": tm.t_done}

    def stats(self) -> dict:
        st = ServerStats()
        _check(self._lib.ld_server_stats_get(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}


def clock() -> float:
    """ld_server_clock: the monotonic clock of the request times."""
    return float(load().ld_server_clock())
