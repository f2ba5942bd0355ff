"""Oracle: one Levenberg-Marquardt linear solve, end to end (Section 2.1).

Test infrastructure only. Composes the other oracle modules: residual and
Jacobian, damped normal blocks, the Schur system, its solve (direct, or PCG with
point-block-Jacobi or with the multigrid V-cycle) and back-substitution.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import aggregation as agglib
from . import cluster as cl
from . import multigrid as mg
from .camera import jacobian_blocks, residuals
from .normal import Normal, cholesky_solve, solve_full
from .nullspace import camera_nullspace
from .robust import weights as robust_weights


@dataclasses.dataclass
class StepResult:
    delta_c: np.ndarray
    delta_p: np.ndarray
    iters: int = 0
    rel_res: float = 0.0
    converged: bool = True
    levels: list = None
    normal: Normal = None
    b: np.ndarray = None


def normal_for(cams, pts, obs_cam, obs_pt, uv, lam=1e-4, D=None, loss=None, loss_scale=1.0):
    """Normal blocks of the step; with loss="huber" every observation's residual
    and Jacobian rows are weighted by sqrt(rho'(|f_o|^2)) (oracle.robust)."""
    F, E = jacobian_blocks(cams, pts, obs_cam, obs_pt)
    f = residuals(cams, pts, obs_cam, obs_pt, uv)
    w = robust_weights(f, loss, loss_scale)
    F, E, f = F * w[:, None, None], E * w[:, None, None], f * w[:, None]
    return Normal(F, E, f, obs_cam, obs_pt, cams.shape[0], pts.shape[0], lam=lam, D=D)


def lm_step(cams, pts, obs_cam, obs_pt, uv, lam=1e-4, method="mg", rtol=1e-8,
            max_iter=10000, opts: mg.MGOptions = mg.MGOptions(), D=None, forcing=None, loss=None,
            loss_scale=1.0):
    """method: 'full' (sparse LU of J^T J + D), 'schur' (dense Cholesky of S),
    'bj' (PCG, point-block-Jacobi), 'mg' (PCG, multigrid V-cycle), 'cj' (PCG,
    visibility-based block Jacobi over camera clusters, oracle.cluster).
    forcing: Nash-Sofer tolerance tau for the PCG methods (None: residual rule only).
    loss: None (squared) or "huber" with scale loss_scale (oracle.robust)."""
    nrm = normal_for(cams, pts, obs_cam, obs_pt, uv, lam, D, loss, loss_scale)
    n_cam = cams.shape[0]
    if method == "full":
        dc, dp = solve_full(nrm)
        return StepResult(dc, dp, normal=nrm, b=nrm.rhs())
    b = nrm.rhs()
    if method == "schur":
        xc = cholesky_solve(nrm.S_dense(), b)
        dp = nrm.recover_points(xc, -nrm.g_p.ravel())
        return StepResult(xc.reshape(n_cam, 9), dp, normal=nrm, b=b)
    if method == "bj":
        Binv = np.linalg.inv(nrm.block_jacobi_blocks())
        M = lambda r: mg.apply_blocks(Binv, r)
        levels = None
    elif method == "mg":
        levels = hierarchy_for(nrm, cams, obs_cam, obs_pt, opts)
        M = lambda r: mg.vcycle(levels, r, opts)
    elif method == "cj":
        W0 = agglib.covisibility(obs_cam, obs_pt, n_cam, nrm.n_pt)
        agg, n_agg = cl.clusters(W0, opts)
        blocks = cl.cluster_inverses(nrm.S_sparse(), agg, n_agg)
        M = lambda r: cl.apply(blocks, r)
        levels = None
    else:
        raise ValueError(method)
    res = mg.pcg(nrm.S_apply, M, b, rtol, max_iter, forcing)
    dp = nrm.recover_points(res.x, -nrm.g_p.ravel())
    return StepResult(res.x.reshape(n_cam, 9), dp, res.iters, res.rel_res, res.converged,
                      levels, nrm, b)


def hierarchy_for(nrm: Normal, cams, obs_cam, obs_pt, opts: mg.MGOptions = mg.MGOptions()):
    W0 = agglib.covisibility(obs_cam, obs_pt, cams.shape[0], nrm.n_pt)
    K0 = camera_nullspace(cams)
    return mg.build_hierarchy(nrm.S_sparse(), K0, W0, opts)


def error_triple(delta_c, ref_c, nrm: Normal, b):
    """||d - d*|| / ||d*||, ||d - d*||_S / ||d*||_S, ||b - S d|| / ||b|| (camera part)."""
    e = (delta_c - ref_c).ravel()
    r = ref_c.ravel()
    Se = nrm.S_apply(e)
    Sr = nrm.S_apply(r)
    res = b - nrm.S_apply(delta_c.ravel())
    return (float(np.linalg.norm(e) / np.linalg.norm(r)),
            float(np.sqrt(max(e @ Se, 0.0)) / np.sqrt(r @ Sr)),
            float(np.linalg.norm(res) / np.linalg.norm(b)))
