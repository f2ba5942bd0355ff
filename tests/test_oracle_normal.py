"""Pins for the oracle's normal equations and Schur complement (Section 2.1),
and for the near-nullspace of Section 3.1."""
import numpy as np
import pytest

from oracle import camera, multigrid as mg, normal, nullspace, step
from scenes import tiny_scene
from tests._fixtures import scene


def _normal(sc, lam=1e-4, D=None):
    return step.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, lam=lam, D=D)


def test_schur_block_elimination_matches_dense_H():
    # S from the dense H by textbook block elimination, H = J^T J + D formed densely
    sc = scene("ring20")
    nrm = _normal(sc)
    J = normal.assemble_J(nrm.F, nrm.E, sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt).toarray()
    H = J.T @ J
    H += np.diag(1e-4 * np.diag(H))
    nc = 9 * sc.n_cam
    Scl = H[:nc, :nc] - H[:nc, nc:] @ np.linalg.solve(H[nc:, nc:], H[nc:, :nc])
    S = nrm.S_dense()
    assert np.abs(S - Scl).max() <= 1e-9 * np.abs(Scl).max()
    # right-hand side from the same elimination
    g = J.T @ nrm.f.ravel()
    bcl = -g[:nc] + H[:nc, nc:] @ np.linalg.solve(H[nc:, nc:], g[nc:])
    np.testing.assert_allclose(nrm.rhs(), bcl, rtol=0, atol=1e-9 * np.abs(bcl).max())


@pytest.mark.parametrize("name", ["ring20", "ring64"])
def test_schur_step_equals_full_solve(name):
    sc = scene(name)
    full = step.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="full")
    sch = step.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="schur")
    rc = np.linalg.norm(sch.delta_c - full.delta_c) / np.linalg.norm(full.delta_c)
    rp = np.linalg.norm(sch.delta_p - full.delta_p) / np.linalg.norm(full.delta_p)
    assert rc < 1e-7 and rp < 1e-7


def test_full_solve_satisfies_definition():
    sc = scene("ring20")
    nrm = _normal(sc)
    dc, dp = normal.solve_full(nrm)
    H = nrm.H_sparse()
    g = np.concatenate([nrm.g_c.ravel(), nrm.g_p.ravel()])
    res = H @ np.concatenate([dc.ravel(), dp.ravel()]) + g
    assert np.linalg.norm(res) <= 1e-10 * np.linalg.norm(g)


def test_implicit_product_equals_explicit():
    sc = tiny_scene(7, 60, seed=2)
    nrm = _normal(sc)
    S = nrm.S_dense()
    n = 9 * sc.n_cam
    cols = np.column_stack([nrm.S_apply(np.eye(n)[:, k]) for k in range(n)])
    assert np.abs(cols - S).max() <= 1e-11 * np.abs(S).max()
    assert np.abs(S - S.T).max() <= 1e-11 * np.abs(S).max()


def test_block_jacobi_blocks_are_diagonal_of_S():
    sc = tiny_scene(6, 50, seed=3)
    nrm = _normal(sc)
    S = nrm.S_dense()
    B = nrm.block_jacobi_blocks()
    for c in range(sc.n_cam):
        np.testing.assert_allclose(B[c], S[9 * c:9 * c + 9, 9 * c:9 * c + 9], rtol=1e-12,
                                   atol=1e-12 * np.abs(S).max())


def test_cholesky_solve_matches_library():
    sc = scene("ring20")
    nrm = _normal(sc)
    S = nrm.S_dense()
    b = nrm.rhs()
    x = normal.cholesky_solve(S, b)
    np.testing.assert_allclose(x, np.linalg.solve(S, b), rtol=1e-6,
                               atol=1e-8 * np.abs(x).max())


@pytest.mark.parametrize("which", ["truth", "perturbed"])
def test_gauge_nullspace_of_J(which):
    # J N = 0 for the 7 similarity modes, at any parameter values
    sc = scene("ring20")
    cams = sc.cams_true if which == "truth" else sc.cams
    pts = sc.pts_true if which == "truth" else sc.pts
    F, E = camera.jacobian_blocks(cams, pts, sc.obs_cam, sc.obs_pt)
    J = normal.assemble_J(F, E, sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    N = nullspace.full_gauge(cams, pts)
    JN = J @ N
    scale = np.abs(J).max() * np.abs(N).max()
    assert np.abs(JN).max() <= 1e-12 * scale * 10


def test_schur_gauge_nullspace_and_eigen_gap():
    sc = scene("ring20")
    D = np.zeros(9 * sc.n_cam + 3 * sc.n_pt)
    # D = 0 makes C singular only if a point had < 2 views; ring20 has 8 per point.
    nrm = _normal(sc, D=D)
    S = nrm.S_dense()
    K = nullspace.camera_nullspace(sc.cams)[:, :, 9:16].reshape(-1, 7)
    SK = S @ K
    assert np.abs(SK).max() <= 1e-8 * np.abs(S).max() * np.abs(K).max()
    # exactly 7 tiny eigenvalues after Jacobi scaling, then a clear gap
    s = 1.0 / np.sqrt(np.diag(S))
    ev = np.linalg.eigvalsh(S * s[:, None] * s[None, :])
    assert np.all(ev[:7] <= 1e-10 * ev[-1])
    assert ev[7] >= 1e-6 * ev[-1]


def test_decoupled_cameras_block_jacobi_converges_in_one_iteration():
    # cameras that share no point: S is block diagonal, block-Jacobi is exact
    rng = np.random.default_rng(0)
    base = tiny_scene(4, 40, seed=9, shuffle=False)
    keep = []
    owner = rng.integers(0, 4, base.n_pt)
    for o in range(base.n_obs):
        if base.obs_cam[o] == owner[base.obs_pt[o]]:
            keep.append(o)
    keep = np.array(keep)
    used_pts = np.unique(base.obs_pt[keep])
    remap = -np.ones(base.n_pt, dtype=np.int64)
    remap[used_pts] = np.arange(used_pts.size)
    oc = base.obs_cam[keep]
    op = remap[base.obs_pt[keep]]
    res = step.lm_step(base.cams, base.pts[used_pts], oc, op, base.uv[keep], method="bj",
                       rtol=1e-6)
    # one iteration reaches the exact solution up to the rounding of the
    # (ill-conditioned) 9x9 block inverses
    assert res.iters == 1


def test_lm_step_reduces_linearized_model():
    # the step decreases the damped quadratic model: m(d) = |f + J d|^2 + d^T D d < |f|^2
    sc = scene("ring20")
    nrm = _normal(sc)
    dc, dp = normal.solve_full(nrm)
    J = normal.assemble_J(nrm.F, nrm.E, sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    d = np.concatenate([dc.ravel(), dp.ravel()])
    Dd = np.concatenate([nrm.Dc.ravel(), nrm.Dp.ravel()])
    m = np.sum((nrm.f.ravel() + J @ d) ** 2) + d @ (Dd * d)
    assert m < np.sum(nrm.f ** 2)
