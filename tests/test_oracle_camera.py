"""Pins for the oracle's camera model: residual and Jacobian (Sections 2.1, 6)."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import camera
from scenes import tiny_scene
from tests._fixtures import projection_cases, scene


@pytest.mark.parametrize("name", ["ring64", "ring20", "city200", "path500"])
def test_noise_free_data_gives_zero_residual(name):
    # The generator writes pixels with its own rotation-matrix forward model;
    # agreement to rounding checks the oracle's angle-axis model against it.
    sc = scene(name)
    f = camera.residuals(sc.cams_true, sc.pts_true, sc.obs_cam, sc.obs_pt, sc.uv_clean)
    assert np.abs(f).max() <= 1e-9


def test_projection_hand_cases():
    rows = projection_cases()
    cams = rows[:, 0:9]
    pts = rows[:, 9:12]
    idx = np.arange(rows.shape[0])
    pi, _ = camera.project(cams, pts, idx, idx)
    np.testing.assert_allclose(pi, rows[:, 12:14], rtol=0, atol=1e-10)


def test_rotation_matches_library():
    rng = np.random.default_rng(7)
    w = np.concatenate([rng.normal(size=(200, 3)),
                        rng.normal(size=(50, 3)) * 1e-3,
                        rng.normal(size=(50, 3)) * 1e-7,
                        np.zeros((1, 3))])
    # near pi
    v = rng.normal(size=(20, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    w = np.concatenate([w, v * (np.pi - 1e-6)])
    R = camera.rotation_matrix(w)
    Rref = Rotation.from_rotvec(w).as_matrix()
    np.testing.assert_allclose(R, Rref, rtol=0, atol=2e-15 * 8)
    np.testing.assert_allclose(R @ np.swapaxes(R, 1, 2), np.broadcast_to(np.eye(3), R.shape),
                               atol=1e-14)


def test_series_and_closed_forms_agree():
    # both branches evaluated on either side of the switch agree to rounding
    th_lo = np.array([0.2499999])
    th_hi = np.array([0.2500001])
    lo = camera.rotation_coeffs(th_lo)
    hi = camera.rotation_coeffs(th_hi)
    for a, b in zip(lo, hi):
        assert abs(a[0] - b[0]) < 1e-7 * max(1.0, abs(a[0]))
    # closed forms at 0.2 against the series branch at 0.2
    t = 0.2
    s, c = np.sin(t), np.cos(t)
    ref = [s / t, (1 - c) / t ** 2, (t * c - s) / t ** 3, (t * s - 2 * (1 - c)) / t ** 4]
    got = [v[0] for v in camera.rotation_coeffs(np.array([t]))]
    np.testing.assert_allclose(got, ref, rtol=1e-11)
    # limits at 0: a = 1, b = 1/2, a'/t = -1/3, b'/t = -1/12
    np.testing.assert_allclose([v[0] for v in camera.rotation_coeffs(np.array([0.0]))],
                               [1.0, 0.5, -1.0 / 3.0, -1.0 / 12.0], rtol=1e-15)


@pytest.mark.parametrize("name", ["ring20", "city200"])
def test_jacobian_matches_central_differences(name):
    sc = scene(name)
    sel = np.arange(min(sc.n_obs, 4000))
    oc, op = sc.obs_cam[sel], sc.obs_pt[sel]
    F, E = camera.jacobian_blocks(sc.cams, sc.pts, oc, op)
    Ff, Ef = camera.jacobian_fd(sc.cams, sc.pts, oc, op)
    # relative error per block, against the block's scale
    for A, B in ((F, Ff), (E, Ef)):
        scale = np.abs(A).max(axis=(1, 2))
        err = np.abs(A - B).max(axis=(1, 2)) / scale
        assert err.max() <= 1e-6


def test_jacobian_small_and_large_angles():
    sc = tiny_scene(6, 40, seed=5)
    cams = sc.cams.copy()
    cams[0, 0:3] = [1e-9, -2e-9, 0.0]     # series branch
    cams[1, 0:3] = [0.0, 0.0, 0.0]        # exactly zero
    cams[2, 0:3] = [0.1, 0.12, -0.05]     # series branch
    F, E = camera.jacobian_blocks(cams, sc.pts, sc.obs_cam, sc.obs_pt)
    Ff, Ef = camera.jacobian_fd(cams, sc.pts, sc.obs_cam, sc.obs_pt)
    assert np.abs(F - Ff).max() / np.abs(F).max() < 1e-7
    assert np.abs(E - Ef).max() / np.abs(E).max() < 1e-7


def test_gradient_is_J_transpose_f():
    # dObjective/dx = J^T f, checked by central differences of the objective
    sc = scene("ring20")
    F, E = camera.jacobian_blocks(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt)
    f = camera.residuals(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
    g_c = np.zeros_like(sc.cams)
    np.add.at(g_c, sc.obs_cam, np.einsum("nki,nk->ni", F, f))
    h = 1e-6
    for c, k in [(0, 0), (3, 4), (7, 6), (11, 8)]:
        cp, cm = sc.cams.copy(), sc.cams.copy()
        cp[c, k] += h
        cm[c, k] -= h
        fd = (camera.objective(cp, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
              - camera.objective(cm, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)) / (2 * h)
        assert abs(fd - g_c[c, k]) <= 1e-5 * max(1.0, abs(g_c[c, k]))
