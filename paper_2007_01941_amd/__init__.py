"""Multigrid bundle adjustment on AMD Instinct MI355X.

One Levenberg-Marquardt linear solve (Konolige and Brown, "Multigrid for
Bundle Adjustment"): residual and Jacobian, PCG on the implicitly applied
Schur complement, preconditioned by block Jacobi or an unsmoothed-aggregation
multigrid V-cycle; FP64 or mixed FP32/FP64; with an adjoint for gradients.
All of it runs in hand-written HIP kernels in libbamg.so; this package only
marshals torch tensors (device memory and the current stream) to its C ABI.
"""
from __future__ import annotations

import ctypes
import dataclasses
import warnings

import torch

from . import _lib
from ._lib import BAError, LMOptions, NotConverged, Options

__all__ = ["Plan", "Options", "LMOptions", "LMIteration", "LMSummary", "Stats", "lm_step", "LMStep",
           "BAError", "NotConverged"]


@dataclasses.dataclass
class Stats:
    iters: int
    refine_steps: int
    levels: int
    nodes: list
    rel_res: float
    t_jacobian_ms: float
    t_setup_ms: float
    t_solve_ms: float
    converged: bool = True
    fallback_fp64: bool = False
    agg_sizes: list = dataclasses.field(default_factory=list)   # (min, mean, max) per aggregated level


def _stats(st: _lib._Stats, status) -> Stats:
    nl = max(st.levels, 0)
    return Stats(st.iters, st.refine_steps, st.levels, list(st.nodes[:nl]),
                 st.rel_res, st.t_jacobian_ms, st.t_setup_ms, st.t_solve_ms,
                 status == _lib.BA_OK, bool(st.fallback_fp64),
                 [(st.agg_min[l], st.agg_mean[l], st.agg_max[l]) for l in range(max(nl - 1, 0))])


@dataclasses.dataclass
class LMIteration:
    cost: float
    cost_candidate: float
    model_decrease: float
    rho: float
    radius: float
    step_norm: float
    accepted: bool
    pcg_iters: int
    t_ms: float


@dataclasses.dataclass
class LMSummary:
    iters: int
    accepted: int
    termination: str
    pcg_iters: int
    cost0: float
    cost: float
    t_ms: float
    history: list


_TERM = {_lib.TERM_MAX_ITERS: "max_iters", _lib.TERM_FUNCTION: "function_tol",
         _lib.TERM_PARAMETER: "parameter_tol", _lib.TERM_RADIUS: "min_radius"}


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensors passed to the bamg library must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the bamg library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, shape, name):
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class _TorchMemory:
    """Device memory the library asks for through its allocation callbacks,
    handed out as torch uint8 tensors and kept alive until released."""

    def __init__(self, device):
        self.device = device
        self.live = {}
        self.alloc_cb = _lib.ALLOC_FN(self._alloc)
        self.free_cb = _lib.FREE_FN(self._free)

    def _alloc(self, nbytes, ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:        # out of memory: the library reports the NULL
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, ctx):
        self.live.pop(ptr, None)

    @property
    def bytes(self):
        return sum(t.numel() for t in self.live.values())


class Plan:
    """Integer structure of one visibility graph (observation layout, tiles and
    the multigrid hierarchy pattern), reusable across LM steps. All device
    memory is torch's: the plan's persistent arrays come through the
    library's allocation callbacks, and each step runs in a workspace tensor
    of ba_workspace_bytes() bytes that this object keeps (and grows)."""

    def __init__(self, n_cam, n_pt, obs_cam, obs_pt, opts: Options | None = None):
        self.opts = opts or Options()
        self.n_cam, self.n_pt = int(n_cam), int(n_pt)
        obs_cam = obs_cam.to(torch.int32).contiguous()
        obs_pt = obs_pt.to(torch.int32).contiguous()
        self.n_obs = int(obs_cam.numel())
        self._mem = _TorchMemory(obs_cam.device)
        self._ws = None
        self._h = ctypes.c_void_p()
        o = self.opts.to_c()
        _lib.check(_lib.LIB.ba_plan_create(self.n_cam, self.n_pt, self.n_obs, _ptr(obs_cam),
                                           _ptr(obs_pt), ctypes.byref(o), self._mem.alloc_cb,
                                           self._mem.free_cb, None, _stream(), ctypes.byref(self._h)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None and _lib.LIB is not None:
            _lib.LIB.ba_plan_destroy(h)
            self._h = None

    def workspace_bytes(self, opts: Options | None = None, uses: int = _lib.USE_STEP) -> int:
        o = self._opts(opts)
        n = int(_lib.LIB.ba_workspace_bytes(self._h, ctypes.byref(o), uses))
        if n == 0:
            raise _lib.BAError(-1, "BA_ERR_ARG", _lib.LIB.ba_last_error().decode())
        return n

    def _workspace(self, o, uses):
        """(pointer, bytes) of a workspace tensor large enough for the options."""
        need = int(_lib.LIB.ba_workspace_bytes(self._h, ctypes.byref(o), uses))
        if need == 0:
            raise _lib.BAError(-1, "BA_ERR_ARG", _lib.LIB.ba_last_error().decode())
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self._mem.device)
        return ctypes.c_void_p(self._ws.data_ptr()), ctypes.c_size_t(self._ws.numel())

    @property
    def device_bytes(self) -> int:
        """Device bytes of the plan's persistent arrays plus its workspace."""
        return int(_lib.LIB.ba_plan_bytes(self._h)) + (self._ws.numel() if self._ws is not None else 0)

    def _opts(self, opts):
        # the prolongator is fixed when the plan is built: steps take the plan's
        o = opts or self.opts
        if o.prolongator != self.opts.prolongator:
            o = dataclasses.replace(o, prolongator=self.opts.prolongator)
        return o.to_c()

    # ---- full step
    def lm_step(self, cams, pts, uv, D=None, opts: Options | None = None):
        """(delta_cam [n_cam, 9], delta_pt [n_pt, 3], Stats)."""
        self._check_inputs(cams, pts, uv)
        dc = torch.empty((self.n_cam, 9), dtype=torch.float64, device=cams.device)
        dp = torch.empty((self.n_pt, 3), dtype=torch.float64, device=cams.device)
        st = _lib._Stats()
        o = self._opts(opts)
        ws, wsb = self._workspace(o, _lib.USE_STEP)
        status = _lib.check(_lib.LIB.ba_lm_step(self._h, ctypes.byref(o), _ptr(cams), _ptr(pts), _ptr(uv),
                                                _ptr(D), ws, wsb, _ptr(dc), _ptr(dp), ctypes.byref(st),
                                                _stream()))
        if status == _lib.BA_NOT_CONVERGED:
            warnings.warn("PCG did not reach rtol within max_iter", NotConverged)
        return dc, dp, _stats(st, status)

    def backward(self, cams, pts, uv, delta_cam, delta_pt, gd_cam, gd_pt, opts=None, D=None):
        """Gradients (g_cams, g_pts, g_uv) of L(delta) given dL/d delta. D: the
        explicit damping diagonal of the forward step, if it had one."""
        self._check_inputs(cams, pts, uv)
        g_c = torch.empty_like(cams)
        g_p = torch.empty_like(pts)
        g_u = torch.empty_like(uv)
        st = _lib._Stats()
        o = self._opts(opts)
        if D is not None:
            D = _f64(D, (9 * self.n_cam + 3 * self.n_pt,), "D")
        ws, wsb = self._workspace(o, _lib.USE_BACKWARD)
        status = _lib.check(_lib.LIB.ba_lm_step_backward(
            self._h, ctypes.byref(o), _ptr(cams), _ptr(pts), _ptr(uv), _ptr(D) if D is not None else None,
            _ptr(delta_cam.contiguous()), _ptr(delta_pt.contiguous()), _ptr(gd_cam.contiguous()),
            _ptr(gd_pt.contiguous()), ws, wsb, _ptr(g_c), _ptr(g_p), _ptr(g_u), ctypes.byref(st), _stream()))
        if status == _lib.BA_NOT_CONVERGED:
            warnings.warn("adjoint PCG did not reach rtol within max_iter", NotConverged)
        return g_c, g_p, g_u, _stats(st, status)

    # ---- the Levenberg-Marquardt loop
    def cost(self, cams, pts, uv, opts: Options | None = None):
        """(1/2 sum rho(|f_o|^2) with the loss of opts, number of observations
        with the point at or behind the camera or a non-finite residual)."""
        self._check_inputs(cams, pts, uv)
        c = ctypes.c_double()
        bad = ctypes.c_int64()
        o = self._opts(opts)
        ws, wsb = self._workspace(o, _lib.USE_LM)
        _lib.check(_lib.LIB.ba_cost(self._h, ctypes.byref(o), _ptr(cams), _ptr(pts), _ptr(uv), ws, wsb,
                                    ctypes.byref(c), ctypes.byref(bad), _stream()))
        return c.value, bad.value

    def cost_noalloc(self, cams, pts, uv, opts: Options | None = None):
        """As cost(), through ba_cost_noalloc: no workspace, no allocation
        (a static device scratch array shared by all calls on the GPU)."""
        self._check_inputs(cams, pts, uv)
        c = ctypes.c_double()
        bad = ctypes.c_int64()
        o = self._opts(opts)
        _lib.check(_lib.LIB.ba_cost_noalloc(self._h, ctypes.byref(o), _ptr(cams), _ptr(pts), _ptr(uv),
                                            ctypes.byref(c), ctypes.byref(bad), _stream()))
        return c.value, bad.value

    def lm_solve(self, cams, pts, uv, opts: Options | None = None, lm_opts: LMOptions | None = None):
        """Levenberg-Marquardt from (cams, pts), which are updated in place.
        Returns an LMSummary with the per-iteration history."""
        self._check_inputs(cams, pts, uv)
        lo = (lm_opts or LMOptions()).to_c()
        o = self._opts(opts)
        hist = (_lib._LMIter * max(lo.max_iters, 1))()
        sm = _lib._LMSummary()
        ws, wsb = self._workspace(o, _lib.USE_LM)
        _lib.check(_lib.LIB.ba_lm_solve(self._h, ctypes.byref(o), ctypes.byref(lo), _ptr(cams), _ptr(pts),
                                        _ptr(uv), ws, wsb, hist, ctypes.byref(sm), _stream()),
                   allow_not_converged=False)
        h = [LMIteration(r.cost, r.cost_candidate, r.model_decrease, r.rho, r.radius, r.step_norm,
                         bool(r.accepted), r.pcg_iters, r.t_ms) for r in hist[: sm.iters]]
        return LMSummary(sm.iters, sm.accepted, _TERM[sm.termination], sm.pcg_iters, sm.cost0, sm.cost,
                         sm.t_ms, h)

    # ---- stages
    def eval_jacobian(self, cams, pts, uv):
        self._check_inputs(cams, pts, uv)
        dev = cams.device
        f = torch.empty((self.n_obs, 2), dtype=torch.float64, device=dev)
        F = torch.empty((self.n_obs, 2, 9), dtype=torch.float64, device=dev)
        E = torch.empty((self.n_obs, 2, 3), dtype=torch.float64, device=dev)
        ws, wsb = self._workspace(self._opts(None), _lib.USE_STEP)
        _lib.check(_lib.LIB.ba_eval_jacobian(self._h, _ptr(cams), _ptr(pts), _ptr(uv), ws, wsb, _ptr(f), _ptr(F),
                                             _ptr(E), _stream()))
        return f, F, E

    def prepare(self, cams, pts, uv, D=None, opts=None):
        self._check_inputs(cams, pts, uv)
        st = _lib._Stats()
        o = self._opts(opts)
        ws, wsb = self._workspace(o, _lib.USE_STEP)
        _lib.check(_lib.LIB.ba_step_prepare(self._h, ctypes.byref(o), _ptr(cams), _ptr(pts), _ptr(uv),
                                            _ptr(D), ws, wsb, ctypes.byref(st), _stream()))
        return _stats(st, 0)

    def solve(self, opts=None, device="cuda"):
        dc = torch.empty((self.n_cam, 9), dtype=torch.float64, device=device)
        dp = torch.empty((self.n_pt, 3), dtype=torch.float64, device=device)
        st = _lib._Stats()
        o = self._opts(opts)
        status = _lib.check(_lib.LIB.ba_step_solve(self._h, ctypes.byref(o), _ptr(dc), _ptr(dp),
                                                   ctypes.byref(st), _stream()))
        return dc, dp, _stats(st, status)

    def schur_apply(self, x, precision="fp64"):
        x = x.contiguous()
        y = torch.empty_like(x)
        _lib.check(_lib.LIB.ba_schur_apply(self._h, _lib.FP64 if precision == "fp64" else _lib.MIXED,
                                           _ptr(x), _ptr(y), _stream()))
        return y

    def schur_offdiag_apply(self, x, y, precision="fp64"):
        """y -= W C^-1 W^T x in place (the point-elimination term of S)."""
        x = x.contiguous()
        assert y.is_contiguous() and y.dtype == torch.float64 and y.shape == x.shape
        _lib.check(_lib.LIB.ba_schur_offdiag_apply(self._h, _lib.FP64 if precision == "fp64" else _lib.MIXED,
                                                   _ptr(x), _ptr(y), _stream()))
        return y

    def precond_apply(self, r, opts=None, precision="fp64"):
        r = r.contiguous()
        z = torch.empty_like(r)
        o = self._opts(opts)
        _lib.check(_lib.LIB.ba_precond_apply(self._h, ctypes.byref(o),
                                             _lib.FP64 if precision == "fp64" else _lib.MIXED,
                                             _ptr(r), _ptr(z), _stream()))
        return z

    def step_blocks(self, device="cuda"):
        b = torch.empty((self.n_cam, 9), dtype=torch.float64, device=device)
        Cinv = torch.empty((self.n_pt, 3, 3), dtype=torch.float64, device=device)
        Scc = torch.empty((self.n_cam, 9, 9), dtype=torch.float64, device=device)
        _lib.check(_lib.LIB.ba_step_blocks(self._h, _ptr(b), _ptr(Cinv), _ptr(Scc), _stream()))
        return b, Cinv, Scc

    # ---- hierarchy
    def mg_levels(self):
        n = ctypes.c_int32()
        nodes = (ctypes.c_int32 * 16)()
        _lib.check(_lib.LIB.ba_mg_levels(self._h, ctypes.byref(n), nodes))
        return list(nodes[: n.value])

    def mg_aggregates(self, level, device="cuda"):
        n = self.mg_levels()[level]
        agg = torch.empty(n, dtype=torch.int32, device=device)
        _lib.check(_lib.LIB.ba_mg_aggregates(self._h, level, _ptr(agg)))
        return agg

    def mg_covisibility(self, level, device="cuda"):
        nnz = ctypes.c_int64()
        _lib.check(_lib.LIB.ba_mg_covisibility(self._h, level, ctypes.byref(nnz), None, None, None))
        n = self.mg_levels()[level]
        rp = torch.empty(n + 1, dtype=torch.int64, device=device)
        col = torch.empty(nnz.value, dtype=torch.int32, device=device)
        val = torch.empty(nnz.value, dtype=torch.int64, device=device)
        _lib.check(_lib.LIB.ba_mg_covisibility(self._h, level, ctypes.byref(nnz), _ptr(rp), _ptr(col),
                                               _ptr(val)))
        return rp, col, val

    def mg_level_data(self, level, what, device="cuda"):
        nodes = self.mg_levels()
        n = nodes[level]
        bs = 9 if level == 0 else 16
        nv = n * bs
        nc = nodes[level + 1] * 16 if level + 1 < len(nodes) else 0
        shapes = {"operator": (nv, nv), "P": (n, bs, 16), "K": (n, bs, 16), "Dinv": (n, bs, bs),
                  "lmax": (1,), "coarse_inverse": (nv, nv), "P_smoothed": (nv, nc)}
        codes = {"operator": 0, "P": 1, "K": 2, "Dinv": 3, "lmax": 4, "coarse_inverse": 5, "P_smoothed": 6}
        out = torch.empty(shapes[what], dtype=torch.float64, device=device)
        _lib.check(_lib.LIB.ba_mg_level_data(self._h, level, codes[what], _ptr(out), _stream()))
        return out

    def _check_inputs(self, cams, pts, uv):
        _f64(cams, (self.n_cam, 9), "cams")
        _f64(pts, (self.n_pt, 3), "pts")
        _f64(uv, (self.n_obs, 2), "uv")


def lm_step(cams, pts, uv, obs_cam, obs_pt, opts: Options | None = None, D=None):
    """One LM step from scratch (plan + step): (delta_cam, delta_pt, Stats)."""
    plan = Plan(cams.shape[0], pts.shape[0], obs_cam, obs_pt, opts)
    return plan.lm_step(cams, pts, uv, D=D, opts=opts)


class LMStep(torch.autograd.Function):
    """delta = LMStep.apply(cams, pts, uv, plan, opts, D): differentiable LM
    step; backward runs the adjoint solve with the same Schur system and
    preconditioner. D (optional) is an explicit damping diagonal, held
    constant (no gradient flows to it)."""

    @staticmethod
    def forward(ctx, cams, pts, uv, plan: Plan, opts: Options | None = None, D=None):
        dc, dp, st = plan.lm_step(cams.detach(), pts.detach(), uv.detach(), opts=opts,
                                  D=None if D is None else D.detach())
        ctx.plan, ctx.opts = plan, opts
        ctx.D = None if D is None else D.detach()
        ctx.save_for_backward(cams, pts, uv, dc, dp)
        return dc, dp

    @staticmethod
    def backward(ctx, gdc, gdp):
        cams, pts, uv, dc, dp = ctx.saved_tensors
        if gdc is None:
            gdc = torch.zeros_like(dc)
        if gdp is None:
            gdp = torch.zeros_like(dp)
        g_c, g_p, g_u, _ = ctx.plan.backward(cams.detach(), pts.detach(), uv.detach(), dc, dp,
                                             gdc.contiguous(), gdp.contiguous(), ctx.opts, D=ctx.D)
        return g_c, g_p, g_u, None, None, None
