"""Pins for the oracle's gradient of one LM step (differentiation form)."""
import numpy as np
import pytest

from oracle import adjoint, step
from tests._fixtures import scene


def _loss(sc, cams, pts, uv, lam=1e-4):
    r = step.lm_step(cams, pts, sc.obs_cam, sc.obs_pt, uv, method="full", lam=lam)
    return adjoint.loss_sq(r.delta_c, r.delta_p)


@pytest.fixture(scope="module")
def ring20_grad():
    sc = scene("ring20")
    _, grads, _ = adjoint.step_and_gradient(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv,
                                            adjoint.gbar_sq)
    return sc, grads


def test_directional_derivatives_match_finite_differences(ring20_grad):
    sc, (gc, gp, guv) = ring20_grad
    gnorm = np.sqrt((gc ** 2).sum() + (gp ** 2).sum() + (guv ** 2).sum())
    rng = np.random.default_rng(11)

    def central(h, vc, vp, vu):
        return (_loss(sc, sc.cams + h * vc, sc.pts + h * vp, sc.uv + h * vu)
                - _loss(sc, sc.cams - h * vc, sc.pts - h * vp, sc.uv - h * vu)) / (2 * h)

    for _ in range(16):
        vc = rng.normal(size=sc.cams.shape)
        vp = rng.normal(size=sc.pts.shape)
        vu = rng.normal(size=sc.uv.shape)
        s = np.sqrt((vc ** 2).sum() + (vp ** 2).sum() + (vu ** 2).sum())
        vc, vp, vu = vc / s, vp / s, vu / s
        # Richardson extrapolation of central differences: O(h^4) truncation
        h = 2e-4
        fd = (4.0 * central(h / 2, vc, vp, vu) - central(h, vc, vp, vu)) / 3.0
        an = (gc * vc).sum() + (gp * vp).sum() + (guv * vu).sum()
        # finite-difference noise scales with the overall sensitivity |grad L|
        # (unit directions), not with this particular directional derivative
        assert abs(fd - an) <= 1e-6 * gnorm + 1e-6 * abs(an)


def test_observation_gradient_closed_form(ring20_grad):
    # delta is affine in u, so L is quadratic in u and central differences
    # along u are exact up to rounding
    sc, (_, _, guv) = ring20_grad
    rng = np.random.default_rng(5)
    for _ in range(4):
        vu = rng.normal(size=sc.uv.shape)
        h = 1e-3
        fd = (_loss(sc, sc.cams, sc.pts, sc.uv + h * vu)
              - _loss(sc, sc.cams, sc.pts, sc.uv - h * vu)) / (2 * h)
        assert abs(fd - (guv * vu).sum()) <= 1e-7 * abs(fd)


def test_damping_term_matters(ring20_grad):
    # with D(x) frozen the gradient differs: the d D/dx term is not negligible
    sc, (gc, _, _) = ring20_grad
    _, (gc2, _, _), _ = adjoint.step_and_gradient(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt,
                                                  sc.uv, adjoint.gbar_sq, freeze_damping=True)
    assert np.linalg.norm(gc - gc2) > 1e-4 * np.linalg.norm(gc)
