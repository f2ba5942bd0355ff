"""ctypes binding of libbamg.so (argument marshalling only).

Every array argument is a torch tensor on the GPU; the library receives raw
device pointers and the current HIP stream. Nothing here computes any part of
the solve: if the shared library is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbamg.so")

BA_OK, BA_NOT_CONVERGED = 0, 1
PC_BLOCK_JACOBI, PC_MULTIGRID, PC_CLUSTER_JACOBI = 0, 1, 2
FP64, MIXED = 0, 1
OP_AUTO, OP_IMPLICIT, OP_EXPLICIT = 0, 1, 2
STOP_RESIDUAL, STOP_NASH_SOFER = 0, 1
LOSS_SQUARED, LOSS_HUBER = 0, 1
PROLONG_TENTATIVE, PROLONG_SMOOTHED = 0, 1
TERM_MAX_ITERS, TERM_FUNCTION, TERM_PARAMETER, TERM_RADIUS = 0, 1, 2, 3
USE_STEP, USE_BACKWARD, USE_LM = 0, 1, 2
BA_ERR_WORKSPACE = -6

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class BAError(RuntimeError):
    def __init__(self, status, name, detail):
        super().__init__(f"{name}: {detail}")
        self.status = status
        self.name = name


class NotConverged(RuntimeWarning):
    pass


class _Opts(ctypes.Structure):
    _fields_ = [("precond", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lam", ctypes.c_double), ("rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("inner_rtol", ctypes.c_double),
                ("agg_cap", ctypes.c_int32), ("cheb_degree", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("coarse_max_nodes", ctypes.c_int32),
                ("max_levels", ctypes.c_int32),
                ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
                ("min_coarsen_ratio", ctypes.c_double),
                ("level0_op", ctypes.c_int32), ("freeze_damping_in_grad", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("stop_rule", ctypes.c_int32), ("prolongator", ctypes.c_int32),
                ("forcing", ctypes.c_double), ("loss", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("loss_scale", ctypes.c_double), ("smooth_omega", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("nodes", ctypes.c_int32 * 16),
                ("rel_res", ctypes.c_double), ("t_jacobian_ms", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("fallback_fp64", ctypes.c_int32), ("reserved_stats", ctypes.c_int32),
                ("agg_min", ctypes.c_int32 * 16), ("agg_max", ctypes.c_int32 * 16),
                ("agg_mean", ctypes.c_double * 16)]


class _LMOpts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("radius0", ctypes.c_double), ("min_relative_decrease", ctypes.c_double),
                ("function_tol", ctypes.c_double), ("parameter_tol", ctypes.c_double),
                ("min_radius", ctypes.c_double), ("max_radius", ctypes.c_double),
                ("reserved", ctypes.c_double * 2)]


class _LMIter(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_double), ("cost_candidate", ctypes.c_double),
                ("model_decrease", ctypes.c_double), ("rho", ctypes.c_double),
                ("radius", ctypes.c_double), ("step_norm", ctypes.c_double),
                ("accepted", ctypes.c_int32), ("pcg_iters", ctypes.c_int32), ("t_ms", ctypes.c_double)]


class _LMSummary(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("termination", ctypes.c_int32), ("pcg_iters", ctypes.c_int32),
                ("cost0", ctypes.c_double), ("cost", ctypes.c_double), ("t_ms", ctypes.c_double)]


@dataclasses.dataclass
class LMOptions:
    """Mirror of ba_lm_opts (defaults as in ba_lm_opts_default)."""
    max_iters: int = 100
    radius0: float = 1e4
    min_relative_decrease: float = 1e-3
    function_tol: float = 1e-6
    parameter_tol: float = 1e-8
    min_radius: float = 1e-32
    max_radius: float = 1e16

    def to_c(self) -> _LMOpts:
        o = _LMOpts()
        o.max_iters, o.radius0 = self.max_iters, self.radius0
        o.min_relative_decrease, o.function_tol = self.min_relative_decrease, self.function_tol
        o.parameter_tol, o.min_radius, o.max_radius = self.parameter_tol, self.min_radius, self.max_radius
        return o


@dataclasses.dataclass
class Options:
    """Mirror of ba_opts (defaults as in ba_opts_default)."""
    precond: str = "mg"              # "mg" | "bj" | "cj" (visibility-based block Jacobi)
    precision: str = "fp64"          # "fp64" | "mixed"
    lam: float = 1e-4
    rtol: float = 1e-6
    max_iter: int = 2000
    max_refine: int = 10
    inner_rtol: float = 1e-3
    agg_cap: int = 20
    cheb_degree: int = 2
    lanczos_steps: int = 5
    coarse_max_nodes: int = 128
    max_levels: int = 12
    cheb_lo: float = 0.3
    cheb_hi: float = 1.1
    min_coarsen_ratio: float = 0.9
    level0_op: str = "auto"          # "auto" | "implicit" | "explicit"
    freeze_damping_in_grad: bool = False
    check_every: int = 4
    deterministic: bool = False
    stop_rule: str = "residual"      # "residual" | "nash_sofer"
    forcing: float = 0.1
    loss: str = "squared"            # "squared" | "huber"
    loss_scale: float = 1.0
    graph: bool = False              # replay PCG iterations from a captured HIP graph
    prolongator: str = "tentative"   # "tentative" | "smoothed" (fixed when the plan is built)
    smooth_omega: float = 4.0 / 3.0

    def to_c(self) -> _Opts:
        o = _Opts()
        o.precond = {"bj": PC_BLOCK_JACOBI, "mg": PC_MULTIGRID, "cj": PC_CLUSTER_JACOBI}[self.precond]
        o.precision = {"fp64": FP64, "mixed": MIXED}[self.precision]
        o.lam, o.rtol, o.max_iter = self.lam, self.rtol, self.max_iter
        o.max_refine, o.inner_rtol = self.max_refine, self.inner_rtol
        o.agg_cap, o.cheb_degree, o.lanczos_steps = self.agg_cap, self.cheb_degree, self.lanczos_steps
        o.coarse_max_nodes, o.max_levels = self.coarse_max_nodes, self.max_levels
        o.cheb_lo, o.cheb_hi, o.min_coarsen_ratio = self.cheb_lo, self.cheb_hi, self.min_coarsen_ratio
        o.level0_op = {"auto": OP_AUTO, "implicit": OP_IMPLICIT, "explicit": OP_EXPLICIT}[self.level0_op]
        o.freeze_damping_in_grad = int(self.freeze_damping_in_grad)
        o.check_every = self.check_every
        o.deterministic = int(self.deterministic)
        o.stop_rule = {"residual": STOP_RESIDUAL, "nash_sofer": STOP_NASH_SOFER}[self.stop_rule]
        o.forcing = self.forcing
        o.loss = {"squared": LOSS_SQUARED, "huber": LOSS_HUBER}[self.loss]
        o.loss_scale = self.loss_scale
        o.graph = int(self.graph)
        o.prolongator = {"tentative": PROLONG_TENTATIVE, "smoothed": PROLONG_SMOOTHED}[self.prolongator]
        o.smooth_omega = self.smooth_omega
        return o


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(or python paper_2007_01941_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    SZ = ctypes.c_size_t
    sig = {
        "ba_opts_default": [P],
        "ba_plan_create": [I32, I32, I64, P, P, P, P, P, P, P, P],
        "ba_plan_destroy": [P],
        "ba_plan_bytes": [P],
        "ba_workspace_bytes": [P, P, I32],
        "ba_lm_step": [P, P, P, P, P, P, P, SZ, P, P, P, P],
        "ba_lm_step_backward": [P, P, P, P, P, P, P, P, P, P, P, SZ, P, P, P, P, P],
        "ba_eval_jacobian": [P, P, P, P, P, SZ, P, P, P, P],
        "ba_step_prepare": [P, P, P, P, P, P, P, SZ, P, P],
        "ba_step_solve": [P, P, P, P, P, P],
        "ba_schur_apply": [P, I32, P, P, P],
        "ba_schur_offdiag_apply": [P, I32, P, P, P],
        "ba_precond_apply": [P, P, I32, P, P, P],
        "ba_step_blocks": [P, P, P, P, P],
        "ba_mg_levels": [P, P, P],
        "ba_mg_aggregates": [P, I32, P],
        "ba_mg_covisibility": [P, I32, P, P, P, P],
        "ba_mg_level_data": [P, I32, I32, P, P],
        "ba_selftest_tile_mma": [P, P, P, I32, P],
        "ba_lm_opts_default": [P],
        "ba_cost": [P, P, P, P, P, P, SZ, P, P, P],
        "ba_cost_noalloc": [P, P, P, P, P, P, P, P],
        "ba_lm_solve": [P, P, P, P, P, P, P, SZ, P, P, P],
        "ba_status_str": [I32],
        "ba_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int32
    lib.ba_plan_destroy.restype = None
    lib.ba_plan_bytes.restype = ctypes.c_size_t
    lib.ba_workspace_bytes.restype = ctypes.c_size_t
    lib.ba_status_str.restype = ctypes.c_char_p
    lib.ba_last_error.restype = ctypes.c_char_p
    return lib


LIB = _load()

# The C ABI's exported symbols, as declared in include/*.h.
EXPORTED = ["ba_opts_default", "ba_plan_create", "ba_plan_destroy", "ba_plan_bytes", "ba_workspace_bytes",
            "ba_lm_step",
            "ba_lm_step_backward", "ba_eval_jacobian", "ba_step_prepare", "ba_step_solve",
            "ba_schur_apply", "ba_schur_offdiag_apply", "ba_precond_apply", "ba_step_blocks", "ba_mg_levels",
            "ba_mg_aggregates", "ba_mg_covisibility", "ba_mg_level_data", "ba_selftest_tile_mma",
            "ba_lm_opts_default", "ba_cost", "ba_cost_noalloc", "ba_lm_solve", "ba_status_str", "ba_last_error"]


def check(status: int, allow_not_converged=True):
    if status == BA_OK:
        return status
    if status == BA_NOT_CONVERGED and allow_not_converged:
        return status
    name = LIB.ba_status_str(status).decode()
    detail = LIB.ba_last_error().decode()
    raise BAError(status, name, detail)
