"""GPU parity of the Huber loss (robust error metrics, Section 5.4): the
reweighted normal blocks, Schur product, explicit level-0 operator, steps,
cost and LM loop against the oracle (oracle.robust)."""
import numpy as np
import pytest

from oracle import lm as olm, multigrid as omg, robust, step as ostep
from oracle.camera import residuals
from scenes import tiny_scene
from tests._fixtures import scene
from tests._gpu import dev, host, inputs, plan_for, rel
from tests.test_gpu_step import TOL_U, rhs_abs, schur_abs, schur_abs_dense

pytestmark = pytest.mark.gpu


def _outliers(sc, frac=0.05, px=50.0, seed=9):
    """The scene's pixels with a fraction moved by px-sized errors, and a Huber
    scale at the median squared residual, so that both branches of the loss
    are populated."""
    rng = np.random.default_rng(seed)
    uv = sc.uv.copy()
    bad = rng.random(sc.n_obs) < frac
    uv[bad] += rng.normal(0.0, px, (int(bad.sum()), 2))
    f = residuals(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv)
    a = float(np.sqrt(np.median(np.sum(f * f, axis=1))))
    return uv, a


# Fixed bound on the relative difference of the Huber weight rho' between the
# two sides. Above the threshold rho'(s) = a / |f|, so |d rho'| / rho' =
# |df| / |f| with df the difference of the residuals, which the two sides
# evaluate through different but equivalent rotation formulas (FP64, a few
# ulps of the pixel scale f |p| ~ 1e2..1e3 px, i.e. ~1e-13 px) and |f| > a
# (about 1 px here): ~1e-13. EPS_W leaves two orders of margin and is what
# the tolerances use; the measured difference is only checked against it, so
# a wrong GPU residual cannot widen its own tolerance.
EPS_W = 1e-11


def _weight_eps(sc, plan, uv, a):
    """Check the measured weight difference against EPS_W; return EPS_W."""
    f_g = host(plan.eval_jacobian(*inputs(sc, uv=uv))[0])
    f_o = residuals(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv)
    n = np.sqrt(np.sum(f_o * f_o, axis=1))
    eps = float(np.where(n > a, np.linalg.norm(f_g - f_o, axis=1) / n, 0.0).max())
    print(f"[gpu] measured Huber weight difference {eps:.1e} (bound {EPS_W:.0e})", flush=True)
    assert eps <= EPS_W
    return EPS_W


def _sc(name):
    if name == "wide":
        return tiny_scene(300, 60, seed=5, k_min=2)
    return scene(name)


@pytest.mark.parametrize("name", ["ring64", "city200", "wide"])
def test_huber_blocks_and_product(name):
    sc = _sc(name)
    uv, a = _outliers(sc)
    plan, opts = plan_for(sc, precond="bj", loss="huber", loss_scale=a)
    eps = _weight_eps(sc, plan, uv, a)      # before prepare: it reuses the step's buffers
    plan.prepare(*inputs(sc, uv=uv), opts=opts)
    b, Cinv, Scc = (host(t) for t in plan.step_blocks())
    nrm = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, loss="huber", loss_scale=a)
    w = robust.weights(residuals(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv), "huber", a)
    print(f"[gpu] {name} huber a={a:.3g}: {np.mean(w < 1):.2f} of observations down-weighted, "
          f"weight bound {eps:.0e}", flush=True)
    assert 0.2 < np.mean(w < 1) < 0.8
    # every weighted quantity is at most quadratic in the weights
    tol = TOL_U + 3 * eps
    assert np.all(np.abs(b - nrm.rhs().reshape(-1, 9)) <= tol * rhs_abs(nrm))
    condC = np.linalg.cond(nrm.C)
    assert np.all(np.abs(Cinv - nrm.Cinv) <= (1e-13 + 2 * eps) * condC[:, None, None]
                  * np.abs(nrm.Cinv).max(axis=(1, 2), keepdims=True))
    from oracle.normal import block_sum
    Babs = np.abs(nrm.A) + block_sum(nrm.obs_cam, np.einsum("nij,njk,nlk->nil", np.abs(nrm.Y),
                                                           np.abs(nrm.Cinv[nrm.obs_pt]), np.abs(nrm.Y)), nrm.n_cam)
    assert np.all(np.abs(Scc - nrm.block_jacobi_blocks()) <= tol * Babs)
    x = np.random.default_rng(0).normal(size=(sc.n_cam, 9))
    y = host(plan.schur_apply(dev(x)))
    assert np.all(np.abs(y - nrm.S_apply(x).reshape(-1, 9)) <= tol * schur_abs(nrm, x))
    # evaluating the Jacobian reuses the step's buffers: the step must be prepared again
    import paper_2007_01941_amd as bamg
    plan.eval_jacobian(*inputs(sc, uv=uv))
    with pytest.raises(bamg.BAError):
        plan.schur_apply(dev(x))


@pytest.mark.parametrize("name", ["ring64", "city200"])
def test_huber_explicit_level0(name):
    """The explicit level-0 S of the multigrid setup recomputes both
    observations' Jacobians of every shared point: with the loss, both carry
    their own weights."""
    sc = _sc(name)
    uv, a = _outliers(sc)
    plan, opts = plan_for(sc, precond="mg", coarse_max_nodes=16, loss="huber", loss_scale=a)
    tol = TOL_U + 3 * _weight_eps(sc, plan, uv, a)
    plan.prepare(*inputs(sc, uv=uv), opts=opts)
    nrm = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, loss="huber", loss_scale=a)
    S0 = host(plan.mg_level_data(0, "operator"))
    assert np.all(np.abs(S0 - nrm.S_dense()) <= tol * schur_abs_dense(nrm))


@pytest.mark.parametrize("pc", ["bj", "mg"])
def test_huber_step(pc):
    sc = scene("city200")
    uv, a = _outliers(sc)
    kw = dict(coarse_max_nodes=16) if pc == "mg" else {}
    plan, opts = plan_for(sc, precond=pc, rtol=1e-10, loss="huber", loss_scale=a, **kw)
    dc, dp, st = plan.lm_step(*inputs(sc, uv=uv))
    nrm = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, loss="huber", loss_scale=a)
    full = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, method="schur", loss="huber", loss_scale=a)
    r = nrm.rhs() - nrm.S_apply(host(dc).ravel())
    slack = TOL_U * np.linalg.norm(schur_abs(nrm, host(dc)) + rhs_abs(nrm))
    print(f"[gpu] city200 huber {pc}: iters {st.iters} rel_res {st.rel_res:.2e} "
          f"err_vs_direct {rel(host(dc), full.delta_c):.2e}", flush=True)
    assert st.converged
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(nrm.rhs()) + slack
    assert rel(host(dc), full.delta_c) <= 1e-6 and rel(host(dp), full.delta_p) <= 1e-6


def test_huber_cost_and_backward_rejected():
    import paper_2007_01941_amd as bamg
    sc = scene("city200")
    uv, a = _outliers(sc)
    plan, opts = plan_for(sc, precond="bj", loss="huber", loss_scale=a)
    c, bad = plan.cost(*inputs(sc, uv=uv), opts=opts)
    ref = robust.objective(residuals(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv), "huber", a)
    assert bad == 0 and abs(c - ref) <= 1e-12 * ref
    cams, pts, uvd = inputs(sc, uv=uv)
    dc, dp, _ = plan.lm_step(cams, pts, uvd, opts=opts)
    with pytest.raises(bamg.BAError):
        plan.backward(cams, pts, uvd, dc, dp, 2 * dc, 2 * dp, opts=opts)


def test_huber_lm_matches_oracle():
    """The LM loop on the Huber objective takes the oracle's decisions and ends
    at its cost. Its model underestimates the decrease (rho near 2), the radius
    grows to ~1e13 and the damping vanishes, so the parameters along the
    near-gauge directions are fixed only to about cond(S) times the inner
    rtol; they are compared at that level."""
    import paper_2007_01941_amd as bamg
    sc = tiny_scene(10, 150, seed=21, k_min=3, k_max=5)
    rng = np.random.default_rng(1)
    uv = sc.uv.copy()
    bad = rng.random(sc.n_obs) < 0.05
    uv[bad] += rng.normal(0.0, 60.0, (int(bad.sum()), 2))
    lo = bamg.LMOptions(max_iters=20)
    plan, opts = plan_for(sc, precond="bj", rtol=1e-11, max_iter=5000, loss="huber", loss_scale=1.0)
    cams, pts, uvd = inputs(sc, uv=uv)
    out = plan.lm_solve(cams, pts, uvd, opts=opts, lm_opts=lo)
    res = olm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, uv, olm.LMOptions(max_iters=20), method="bj",
                    rtol=1e-11, loss="huber", loss_scale=1.0)
    print(f"[gpu] huber lm: iters {out.iters} accepted {out.accepted} term {out.termination} "
          f"cost {out.cost:.10e} (oracle {res.cost:.10e})", flush=True)
    assert len(out.history) == len(res.history)
    for g, o in zip(out.history, res.history):
        assert g.accepted == o.accepted
        assert abs(g.cost - o.cost) <= 1e-8 * o.cost
        assert abs(g.radius - o.radius) <= 1e-8 * o.radius
    assert abs(out.cost - res.cost) <= 1e-8 * res.cost
    assert rel(host(cams), res.cams) <= 1e-6 and rel(host(pts), res.pts) <= 1e-5
