"""Pins of the oracle's Levenberg-Marquardt outer loop and of the Nash-Sofer
forcing rule (Section 2.1; solver settings of Section 5)."""
import os

import numpy as np
import pytest

from oracle import lm, multigrid as mg, step as ostep
from scenes import tiny_scene
from tests._fixtures import GOLDEN


def test_nash_sofer_hand_example():
    """The worked example in tests/golden/nash_sofer_hand.txt (hand arithmetic)."""
    A = np.diag([1.0, 2.0])
    b = np.ones(2)
    rows = np.loadtxt(os.path.join(GOLDEN, "nash_sofer_hand.txt"), comments="#", ndmin=2)
    for tau, iters, x0, x1 in rows:
        res = mg.pcg(lambda v: A @ v, lambda r: r, b, rtol=0.0, max_iter=10, forcing=tau)
        assert res.iters == int(iters)
        assert np.allclose(res.x, [x0, x1], rtol=0, atol=1e-15)


def test_nash_sofer_monotone_in_tau_and_bounded_by_residual_rule():
    """A looser forcing tolerance never takes more iterations, and never more
    than the residual rule alone; the stopped iterate's model value lies
    between Q(0) = 0 and the minimum."""
    rng = np.random.default_rng(0)
    n = 60
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(np.geomspace(1.0, 1e4, n)) @ Q.T
    b = rng.normal(size=n)
    d = 1.0 / np.diag(A)
    M = lambda r: d * r
    its = [mg.pcg(lambda v: A @ v, M, b, 1e-10, 1000, forcing=t).iters for t in (1.0, 0.3, 0.1, 1e-2, 1e-3)]
    assert all(a <= c for a, c in zip(its, its[1:]))
    assert its[-1] <= mg.pcg(lambda v: A @ v, M, b, 1e-10, 1000).iters
    assert its[0] < its[-1]
    # at the exact minimiser Q = -1/2 b^T A^-1 b (closed form); the stopped iterate
    # lies above it and below Q(0) = 0
    xs = mg.pcg(lambda v: A @ v, M, b, 1e-10, 1000, forcing=0.1).x
    q = 0.5 * xs @ A @ xs - xs @ b
    qstar = -0.5 * b @ np.linalg.solve(A, b)
    assert qstar - 1e-9 * abs(qstar) <= q < 0.0


def test_radius_update_hand_values():
    """Madsen-Nielsen-Tingleff update in radius form, values worked by hand."""
    o = lm.LMOptions()
    assert lm.radius_update(10.0, 2.0, 1.0, True, o) == (30.0, 2.0)      # max(1/3, 1 - 1) = 1/3
    assert lm.radius_update(10.0, 8.0, 0.5, True, o) == (10.0, 2.0)      # 1 - 0 = 1
    r, nu = lm.radius_update(10.0, 2.0, 0.75, True, o)                  # 1 - 1/8 = 7/8
    assert nu == 2.0 and abs(r - 80.0 / 7.0) <= 1e-12
    assert lm.radius_update(10.0, 2.0, -1.0, False, o) == (5.0, 4.0)
    assert lm.radius_update(5.0, 4.0, 0.0, False, o) == (1.25, 8.0)
    assert lm.radius_update(1e16, 2.0, 1.0, True, o) == (1e16, 2.0)     # capped


def _scene():
    return tiny_scene(10, 150, seed=21, k_min=2, k_max=5)


def test_model_decrease_closed_form():
    """For an exact step (J^T J + D) delta = -g:  m(0) - m(delta) =
    1/2 (delta^T D delta - g^T delta)  (expand m and use the step equation)."""
    sc = _scene()
    st = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, lam=3e-3, method="full")
    nrm = st.normal
    d = np.concatenate([st.delta_c.ravel(), st.delta_p.ravel()])
    D = np.concatenate([nrm.Dc.ravel(), nrm.Dp.ravel()])
    g = np.concatenate([nrm.g_c.ravel(), nrm.g_p.ravel()])
    closed = 0.5 * (d @ (D * d) - g @ d)
    got = lm.model_decrease(nrm, st.delta_c, st.delta_p)
    assert got > 0 and abs(got - closed) <= 1e-9 * closed


def test_lm_noise_free_converges_to_zero_cost():
    """With noise-free pixels the minimum cost is 0; LM from the perturbed start
    reaches it (to rounding) and stops on the function or parameter rule."""
    sc = _scene()
    res = lm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv_clean, lm.LMOptions(max_iters=50),
                   method="schur")
    assert res.cost <= 1e-16 * res.cost0
    assert res.termination in (lm.TERM_FUNCTION, lm.TERM_PARAMETER)


def test_lm_history_invariants():
    """Accepted steps lower the cost by at least min_relative_decrease of the model
    decrease; rejected steps leave the parameters (and cost) unchanged; the final
    cost does not exceed the truth's cost by more than the noise floor allows."""
    sc = _scene()
    o = lm.LMOptions(max_iters=30, radius0=1e8)
    res = lm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, o, method="bj", rtol=1e-10)
    h = res.history
    assert len(h) >= 2
    for a, b in zip(h, h[1:]):
        assert b.cost == (a.cost_candidate if a.accepted else a.cost)
    for it in h:
        if it.accepted:
            assert it.cost - it.cost_candidate > o.min_relative_decrease * it.model_decrease
    from oracle.camera import objective
    truth = objective(sc.cams_true, sc.pts_true, sc.obs_cam, sc.obs_pt, sc.uv)
    assert res.cost <= truth


def test_lm_forcing_reduces_pcg_work():
    """The Nash-Sofer rule with a loose constant forcing solves each linear system
    less accurately than the residual rule at 1e-10 (fewer PCG iterations), and
    LM still converges to the same minimum."""
    sc = _scene()
    o = lm.LMOptions(max_iters=40)
    tight = lm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, o, method="bj", rtol=1e-10)
    loose = lm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, o, method="bj", rtol=1e-10,
                     forcing=0.1)
    assert sum(i.pcg_iters for i in loose.history) < sum(i.pcg_iters for i in tight.history)
    assert abs(loose.cost - tight.cost) <= 1e-6 * tight.cost


def hard_start(sc, d=0.3, every=15):
    """Every `every`-th point moved to d metres in front of its first observer:
    the first Gauss-Newton-like steps carry those points behind a camera."""
    from oracle.camera import rotation_matrix
    R = rotation_matrix(sc.cams[:, :3])
    C = -np.einsum("nji,nj->ni", R, sc.cams[:, 3:6])
    fwd = -R[:, 2, :]
    pts = sc.pts.copy()
    for p in range(0, sc.n_pt, every):
        c = sc.obs_cam[sc.obs_pt == p][0]
        pts[p] = C[c] + d * fwd[c]
    return pts


def test_lm_rejections_shrink_radius():
    """Candidates that put a point behind a camera are rejected with infinite
    candidate cost; consecutive rejections divide the radius by 2, 4, 8, ...
    and an accepted step resets that factor to 2."""
    sc = _scene()
    pts = hard_start(sc)
    res = lm.solve(sc.cams, pts, sc.obs_cam, sc.obs_pt, sc.uv, lm.LMOptions(max_iters=12), method="bj",
                   rtol=1e-10)
    h = res.history
    assert not h[0].accepted and np.isinf(h[0].cost_candidate)
    nu = 2.0
    for a, b in zip(h, h[1:]):
        if a.accepted:
            assert a.radius / 2.0 < b.radius <= 3.0 * a.radius * (1 + 1e-15)
            nu = 2.0
        else:
            assert b.radius == a.radius / nu
            nu *= 2.0
    assert any(i.accepted for i in h) and res.cost < res.cost0


def test_lm_breakdown_is_a_failed_step():
    """With almost no damping (radius 1e12) the hard start's first damped systems
    are not numerically positive definite and PCG breaks down: the loop counts
    those as failed steps, shrinks the radius as for a rejection and goes on to
    lower the cost."""
    sc = _scene()
    pts = hard_start(sc)
    res = lm.solve(sc.cams, pts, sc.obs_cam, sc.obs_pt, sc.uv, lm.LMOptions(max_iters=25, radius0=1e12),
                   method="bj", rtol=1e-10)
    failed = [i for i, h in enumerate(res.history) if np.isinf(h.cost_candidate) and h.step_norm == 0.0]
    assert failed, "expected at least one breakdown"
    i = failed[0]
    assert res.history[i + 1].radius == res.history[i].radius / 2.0
    assert res.cost < res.cost0
