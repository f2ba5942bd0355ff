"""Oracle: gradient of a loss of one LM step with respect to its inputs.

Test infrastructure only. Not in the paper; it differentiates the step of
Section 2.1. With f = pi(x) - u, H = J^T J + lam diag(J^T J), g = J^T f and the
step H delta = -g, an upstream gradient gbar = dL/d delta gives, with
mu = H^-1 gbar (H is symmetric):
    dL/du_o = J_o mu_o,
    dL/dx   = -J^T (J mu) - sum_o scatter_o( sum_r Hess(pi_{o,r}) w_{o,r} ),
    w_{o,r} = (f_{o,r} + (J_o delta_o)_r) mu_o + (J_o mu_o)_r delta_o
              + 2 lam (mu_o * delta_o * J_o[r,:])          [last term: d D/dx]
where mu_o, delta_o are the 12-vectors (camera, point) of observation o and
Hess(pi_{o,r}) is the 12x12 Hessian of the r-th projected coordinate. Here the
Hessian-vector products are central differences of the analytic Jacobian.
"""
from __future__ import annotations

import numpy as np

from .camera import jacobian_blocks, residuals
from .normal import Normal, ScaledLU


def _obs_vectors(v_c, v_p, obs_cam, obs_pt):
    return np.concatenate([v_c[obs_cam], v_p[obs_pt]], axis=1)   # [n, 12]


def hessian_vector(cams, pts, obs_cam, obs_pt, wdir, h=1e-5):
    """For every observation o and row r, (Hess pi_{o,r}) wdir[o, r] as a 12-vector,
    by central differences of the analytic Jacobian. wdir: [n, 2, 12]."""
    n = obs_cam.shape[0]
    cam = cams[obs_cam]
    pt = pts[obs_pt]
    ident = np.arange(n)
    out = np.zeros((n, 2, 12))
    for r in range(2):
        w = wdir[:, r, :]
        scale = np.maximum(np.linalg.norm(w, axis=1), 1e-300)
        hh = h / scale
        Fp, Ep = jacobian_blocks(cam + hh[:, None] * w[:, :9], pt + hh[:, None] * w[:, 9:],
                                 ident, ident)
        Fm, Em = jacobian_blocks(cam - hh[:, None] * w[:, :9], pt - hh[:, None] * w[:, 9:],
                                 ident, ident)
        Jp = np.concatenate([Fp[:, r, :], Ep[:, r, :]], axis=1)
        Jm = np.concatenate([Fm[:, r, :], Em[:, r, :]], axis=1)
        out[:, r, :] = (Jp - Jm) / (2.0 * hh[:, None])
    out[np.linalg.norm(wdir, axis=2) == 0.0] = 0.0
    return out


def step_and_gradient(cams, pts, obs_cam, obs_pt, uv, gbar_fn, lam=1e-4,
                      freeze_damping=False):
    """Exact step (sparse LU) and the gradient of L(delta) w.r.t. (cams, pts, uv).
    gbar_fn(delta_c, delta_p) -> (dL/d delta_c, dL/d delta_p)."""
    n_cam, n_pt = cams.shape[0], pts.shape[0]
    F, E = jacobian_blocks(cams, pts, obs_cam, obs_pt)
    f = residuals(cams, pts, obs_cam, obs_pt, uv)
    nrm = Normal(F, E, f, obs_cam, obs_pt, n_cam, n_pt, lam=lam)
    lu = ScaledLU(nrm.H_sparse())
    g = np.concatenate([nrm.g_c.ravel(), nrm.g_p.ravel()])
    d = lu.solve(-g)
    dc, dp = d[:9 * n_cam].reshape(n_cam, 9), d[9 * n_cam:].reshape(n_pt, 3)
    gc, gp = gbar_fn(dc, dp)
    mu = lu.solve(np.concatenate([gc.ravel(), gp.ravel()]))
    mc, mp = mu[:9 * n_cam].reshape(n_cam, 9), mu[9 * n_cam:].reshape(n_pt, 3)
    Jo = np.concatenate([F, E], axis=2)                       # [n, 2, 12]
    mu_o = _obs_vectors(mc, mp, obs_cam, obs_pt)
    de_o = _obs_vectors(dc, dp, obs_cam, obs_pt)
    Jmu = np.einsum("nrk,nk->nr", Jo, mu_o)
    Jde = np.einsum("nrk,nk->nr", Jo, de_o)
    g_uv = Jmu.copy()
    # first-order term: -J^T (J mu)
    first = -np.einsum("nrk,nr->nk", Jo, Jmu)
    wdir = (f + Jde)[:, :, None] * mu_o[:, None, :] + Jmu[:, :, None] * de_o[:, None, :]
    if not freeze_damping:
        wdir = wdir + 2.0 * lam * (mu_o * de_o)[:, None, :] * Jo
    hv = hessian_vector(cams, pts, obs_cam, obs_pt, wdir)
    tot = first - hv.sum(axis=1)                              # [n, 12]
    g_c = np.zeros((n_cam, 9))
    g_p = np.zeros((n_pt, 3))
    np.add.at(g_c, obs_cam, tot[:, :9])
    np.add.at(g_p, obs_pt, tot[:, 9:])
    return (dc, dp), (g_c, g_p, g_uv), (mc, mp)


def loss_sq(dc, dp):
    """L = ||delta_c||^2 + ||delta_p||^2 and its gradient 2 delta."""
    return float(np.sum(dc * dc) + np.sum(dp * dp))


def gbar_sq(dc, dp):
    return 2.0 * dc, 2.0 * dp
