"""Pins of the oracle's Huber loss and the reweighted step (robust error
metrics, Section 5.4)."""
import os

import numpy as np

from oracle import lm, robust, step as ostep
from oracle.camera import jacobian_blocks, residuals
from scenes import tiny_scene
from tests._fixtures import GOLDEN


def test_huber_hand_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "huber_hand.txt"), comments="#", ndmin=2)
    for a, s, rho, drho in rows:
        assert abs(robust.huber(np.array([s]), a)[0] - rho) <= 1e-15 * max(1.0, rho)
        assert abs(robust.huber_derivative(np.array([s]), a)[0] - drho) <= 1e-15


def test_huber_derivative_by_finite_differences_and_continuity():
    for a in (1.0, 2.5):
        s = np.array([0.1, 0.5, 0.9, 1.5, 3.0, 40.0]) * a * a
        h = 1e-6 * s
        fd = (robust.huber(s + h, a) - robust.huber(s - h, a)) / (2 * h)
        assert np.allclose(fd, robust.huber_derivative(s, a), rtol=1e-8, atol=0)
        # value and slope continuous across s = a^2
        e = 1e-9 * a * a
        lo, hi = robust.huber(np.array([a * a - e, a * a + e]), a)
        assert abs(hi - lo) <= 3 * e
        d = robust.huber_derivative(np.array([a * a - e, a * a + e]), a)
        assert abs(d[1] - d[0]) <= 1e-8


def test_reweighted_gradient_is_the_robust_gradient():
    """J~^T f~ (weights sqrt(rho')) equals the gradient of 1/2 sum rho(|f|^2),
    checked by central differences along random directions."""
    sc = tiny_scene(8, 60, seed=3, k_min=2, k_max=4)
    rng = np.random.default_rng(0)
    uv = sc.uv.copy()
    uv[rng.random(sc.n_obs) < 0.3] += 40.0          # many observations in the linear branch
    nrm = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, loss="huber", loss_scale=2.0)
    f = residuals(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv)
    s = np.sum(f * f, axis=1)
    assert np.any(s > 4.0) and np.any(s <= 4.0)
    g = np.concatenate([nrm.g_c.ravel(), nrm.g_p.ravel()])

    def cost(x):
        c = x[: 9 * sc.n_cam].reshape(sc.n_cam, 9)
        p = x[9 * sc.n_cam:].reshape(sc.n_pt, 3)
        return robust.objective(residuals(c, p, sc.obs_cam, sc.obs_pt, uv), "huber", 2.0)

    x0 = np.concatenate([sc.cams.ravel(), sc.pts.ravel()])
    for _ in range(6):
        d = rng.normal(size=x0.shape)
        d /= np.linalg.norm(d)
        h = 1e-6
        fd = (cost(x0 + h * d) - cost(x0 - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), np.linalg.norm(g))


def test_all_inliers_give_the_squared_step():
    sc = tiny_scene(8, 60, seed=4, k_min=2, k_max=4)
    f = residuals(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
    a = 2.0 * np.sqrt(np.max(np.sum(f * f, axis=1)))
    st_h = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="full", loss="huber", loss_scale=a)
    st_s = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="full")
    assert np.array_equal(st_h.delta_c, st_s.delta_c) and np.array_equal(st_h.delta_p, st_s.delta_p)


def test_huber_lm_resists_outliers():
    """With gross outliers in the pixels, LM on the Huber objective ends closer to
    the truth (reprojection error against the noise-free pixels, which is
    gauge-free) than LM on the squared objective."""
    sc = tiny_scene(10, 150, seed=21, k_min=3, k_max=5)
    rng = np.random.default_rng(1)
    uv = sc.uv.copy()
    bad = rng.random(sc.n_obs) < 0.05
    uv[bad] += rng.normal(0.0, 60.0, (int(bad.sum()), 2))
    o = lm.LMOptions(max_iters=40)
    sq = lm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, o, method="schur")
    hb = lm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, o, method="schur", loss="huber", loss_scale=1.0)

    def clean_rms(r):
        f = residuals(r.cams, r.pts, sc.obs_cam, sc.obs_pt, sc.uv_clean)
        return float(np.sqrt(np.mean(np.sum(f * f, axis=1))))

    print(f"clean-pixel RMS: squared {clean_rms(sq):.3f}, huber {clean_rms(hb):.3f}")
    assert clean_rms(hb) < 0.5 * clean_rms(sq)
    # the Huber run's accepted costs decrease monotonically in its own objective
    prev = hb.cost0
    for it in hb.history:
        if it.accepted:
            assert it.cost_candidate < prev
            prev = it.cost_candidate
