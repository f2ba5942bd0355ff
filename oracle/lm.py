"""Oracle: the Levenberg-Marquardt outer loop around the linear solve
(Section 2.1; the solver settings of Section 5).

Test infrastructure only. The paper runs Ceres' trust-region
Levenberg-Marquardt with an initial trust-region radius of 1e4 and a constant
forcing sequence tau for the Nash-Sofer stop rule of the inner PCG; it does not
write the outer loop out. Readings taken here:

  * damping D = diag(J^T J) / radius (Marquardt's scaling; lambda = 1/radius,
    so the initial radius 1e4 gives the lambda = 1e-4 of a single step);
  * step quality rho = (cost(x) - cost(x + delta)) / (m(0) - m(delta)) with the
    Gauss-Newton model m(delta) = 1/2 |f + J delta|^2 and cost = 1/2 |f|^2;
  * the radius update of Madsen, Nielsen and Tingleff, "Methods for non-linear
    least squares problems" (2004), Section 3.2, written for radius = 1/mu:
    a step with rho > 1e-3 is accepted, radius /= max(1/3, 1 - (2 rho - 1)^3)
    (capped at max_radius) and nu = 2; otherwise radius /= nu, nu *= 2;
  * parameters are updated additively (all 9 camera parameters, including the
    angle-axis rotation, and the 3 point coordinates);
  * a candidate with a point at or behind an observing camera, or a non-finite
    cost, counts as a rejected step;
  * with the Huber loss (oracle.robust) the cost is 1/2 sum rho(|f_o|^2) and the
    model is that of the reweighted step, 1/2 |f~ + J~ delta|^2;
  * a step whose damped system is not numerically positive definite (PCG or
    a factorization breaks down) is a failed step, handled like a rejection;
  * stopping: max_iters iterations; |delta| <= parameter_tol (|x| +
    parameter_tol) before the candidate is evaluated; an accepted step whose
    cost decrease is <= function_tol times the previous cost; radius below
    min_radius.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import multigrid as mg
from .camera import project
from .normal import assemble_J
from .robust import objective as robust_objective
from .step import lm_step

TERM_MAX_ITERS, TERM_FUNCTION, TERM_PARAMETER, TERM_RADIUS = 0, 1, 2, 3


@dataclasses.dataclass
class LMOptions:
    max_iters: int = 100
    radius0: float = 1e4
    min_relative_decrease: float = 1e-3
    function_tol: float = 1e-6
    parameter_tol: float = 1e-8
    min_radius: float = 1e-32
    max_radius: float = 1e16


@dataclasses.dataclass
class Iteration:
    cost: float             # cost at the start of the iteration
    cost_candidate: float   # cost at x + delta (inf if the candidate is invalid)
    model_decrease: float   # m(0) - m(delta)
    rho: float
    radius: float           # radius of this step (lambda = 1 / radius)
    step_norm: float
    accepted: bool
    pcg_iters: int


@dataclasses.dataclass
class LMResult:
    cams: np.ndarray
    pts: np.ndarray
    cost0: float
    cost: float
    termination: int
    history: list


def cost_and_valid(cams, pts, obs_cam, obs_pt, uv, loss=None, loss_scale=1.0):
    """1/2 sum rho(|pi_o - u_o|^2) (rho(s) = s for the squared loss) and whether
    every point is in front of its observers."""
    pi, xc = project(cams, pts, obs_cam, obs_pt)
    f = pi - uv
    valid = bool(np.all(xc[:, 2] < 0.0))
    c = robust_objective(f, loss, loss_scale)
    return c, valid and np.isfinite(c)


def model_decrease(nrm, delta_c, delta_p):
    """m(0) - m(delta) = 1/2 |f|^2 - 1/2 |f + J delta|^2 with J assembled explicitly."""
    J = assemble_J(nrm.F, nrm.E, nrm.obs_cam, nrm.obs_pt, nrm.n_cam, nrm.n_pt)
    Jd = J @ np.concatenate([delta_c.ravel(), delta_p.ravel()])
    f = nrm.f.ravel()
    return 0.5 * float(f @ f) - 0.5 * float((f + Jd) @ (f + Jd))


def radius_update(radius, nu, rho, accepted, o: LMOptions):
    """Next (radius, nu) after a step of quality rho."""
    if accepted:
        return min(o.max_radius, radius / max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)), 2.0
    return radius / nu, 2.0 * nu


def solve(cams, pts, obs_cam, obs_pt, uv, o: LMOptions = LMOptions(), method="bj", rtol=1e-8,
          forcing=None, max_pcg=10000, mg_opts: mg.MGOptions = mg.MGOptions(), loss=None,
          loss_scale=1.0) -> LMResult:
    cams = np.array(cams, dtype=np.float64)
    pts = np.array(pts, dtype=np.float64)
    cost, valid = cost_and_valid(cams, pts, obs_cam, obs_pt, uv, loss, loss_scale)
    if not valid:
        raise ValueError("initial parameters put a point at or behind an observing camera")
    cost0 = cost
    radius, nu = o.radius0, 2.0
    hist = []
    term = TERM_MAX_ITERS
    for _ in range(o.max_iters):
        try:
            st = lm_step(cams, pts, obs_cam, obs_pt, uv, lam=1.0 / radius, method=method, rtol=rtol,
                         max_iter=max_pcg, opts=mg_opts, forcing=forcing, loss=loss, loss_scale=loss_scale)
        except np.linalg.LinAlgError:
            hist.append(Iteration(cost, np.inf, 0.0, -np.inf, radius, 0.0, False, 0))
            radius, nu = radius_update(radius, nu, -np.inf, False, o)
            if radius < o.min_radius:
                term = TERM_RADIUS
                break
            continue
        dc, dp = st.delta_c, st.delta_p
        step_norm = float(np.sqrt(np.sum(dc * dc) + np.sum(dp * dp)))
        x_norm = float(np.sqrt(np.sum(cams * cams) + np.sum(pts * pts)))
        if step_norm <= o.parameter_tol * (x_norm + o.parameter_tol):
            term = TERM_PARAMETER
            break
        md = model_decrease(st.normal, dc, dp)
        cams_new, pts_new = cams + dc, pts + dp
        cost_new, valid = cost_and_valid(cams_new, pts_new, obs_cam, obs_pt, uv, loss, loss_scale)
        if not valid:
            cost_new = np.inf
        rho = (cost - cost_new) / md if (md > 0.0 and valid) else -np.inf
        accepted = bool(rho > o.min_relative_decrease)
        hist.append(Iteration(cost, cost_new, md, rho, radius, step_norm, accepted, st.iters))
        radius, nu = radius_update(radius, nu, rho, accepted, o)
        if accepted:
            decrease = cost - cost_new
            cams, pts = cams_new, pts_new
            if decrease <= o.function_tol * cost:
                cost = cost_new
                term = TERM_FUNCTION
                break
            cost = cost_new
        elif radius < o.min_radius:
            term = TERM_RADIUS
            break
    return LMResult(cams, pts, cost0, cost, term, hist)
