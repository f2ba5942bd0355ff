"""GPU parity of the Levenberg-Marquardt outer loop and of the Nash-Sofer
forcing rule (Section 2.1; solver settings of Section 5) against the oracle."""
import numpy as np
import pytest

from oracle import lm as olm, multigrid as omg, step as ostep
from oracle.camera import project
from scenes import tiny_scene
from tests._fixtures import scene
from tests._gpu import dev, host, inputs, plan_for, rel
from tests.test_oracle_lm import hard_start

pytestmark = pytest.mark.gpu


def _oracle_cost(sc, cams, pts):
    pi, xc = project(cams, pts, sc.obs_cam, sc.obs_pt)
    f = pi - sc.uv
    ok = xc[:, 2] < 0.0
    return 0.5 * float(np.sum(f[ok] * f[ok])), int(np.sum(~ok))


@pytest.mark.parametrize("name", ["ring64", "city200"])
def test_cost(name):
    sc = scene(name)
    plan, _ = plan_for(sc, precond="bj")
    c, bad = plan.cost(*inputs(sc))
    ref, ref_bad = _oracle_cost(sc, sc.cams, sc.pts)
    print(f"[gpu] {name} cost {c:.10e} oracle {ref:.10e}", flush=True)
    assert bad == ref_bad == 0
    assert abs(c - ref) <= 1e-12 * ref


def test_cost_counts_points_behind_cameras():
    sc = tiny_scene(10, 150, seed=21, k_min=2, k_max=5)
    pts = hard_start(sc, d=-0.5)          # these points now lie behind their first observer
    plan, _ = plan_for(sc, precond="bj")
    c, bad = plan.cost(*inputs(sc, pts=pts))
    ref, ref_bad = _oracle_cost(sc, sc.cams, pts)
    print(f"[gpu] behind: invalid {bad} (oracle {ref_bad})", flush=True)
    assert ref_bad > 0 and bad == ref_bad
    assert abs(c - ref) <= 1e-12 * ref


def _rule_values(nrm, b, iterates):
    """Nash-Sofer rule values i (Q_i - Q_{i-1}) / Q_i of PCG iterates x_1, x_2, ...
    with Q(x) = 1/2 x^T S x - x^T b evaluated by the oracle's S and b."""
    vals, q_prev = [], 0.0
    for k, x in enumerate(iterates, start=1):
        q = 0.5 * x @ nrm.S_apply(x) - x @ b
        vals.append(k * (q - q_prev) / q)
        q_prev = q
    return vals


def _gpu_iterate(plan, sc, k, **kw):
    """The GPU's own PCG iterate after exactly k iterations (residual rule out of reach)."""
    import warnings
    import paper_2007_01941_amd as bamg
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", bamg.NotConverged)
        dc, _, _ = plan.lm_step(*inputs(sc), opts=bamg.Options(rtol=1e-14, max_iter=k, **kw))
    return host(dc).ravel()


@pytest.mark.parametrize("pc", ["bj", "mg"])
@pytest.mark.parametrize("tau", [0.1, 0.01])
def test_nash_sofer_step(pc, tau):
    """The GPU's PCG stops at the first iterate where the rule holds, evaluated
    by the oracle's quadratic model on the GPU's own iterates (up to rounding at
    the threshold). With block Jacobi the iterates are unique and the step
    equals the oracle's; the multigrid iterates depend on the non-unique extra
    columns of rank-deficient aggregates, so there the GPU's stopped step is
    compared with the GPU's own iterate of the same index."""
    sc = scene("ring64")
    kw = dict(precond=pc, coarse_max_nodes=16) if pc == "mg" else dict(precond=pc)
    plan, opts = plan_for(sc, rtol=1e-12, stop_rule="nash_sofer", forcing=tau, **kw)
    dc, dp, st = plan.lm_step(*inputs(sc))
    mgo = omg.MGOptions(coarse_max_nodes=16)
    ref = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method=pc, rtol=1e-12, opts=mgo,
                        forcing=tau)
    its = [_gpu_iterate(plan, sc, k, **kw) for k in range(1, st.iters + 1)]
    vals = _rule_values(ref.normal, ref.b, its)
    print(f"[gpu] ring64 {pc} tau {tau}: iters {st.iters} (oracle {ref.iters}) rule values on the GPU "
          f"iterates {[round(float(v), 6) for v in vals]} err vs oracle {rel(host(dc), ref.delta_c):.2e}",
          flush=True)
    assert st.converged
    assert vals[-1] <= tau * (1 + 1e-6)
    assert all(v > tau * (1 - 1e-6) for v in vals[:-1])
    assert rel(host(dc).ravel(), its[-1]) <= 1e-10
    if pc == "bj":
        assert st.iters == ref.iters
        assert rel(host(dc), ref.delta_c) <= 1e-7
        assert rel(host(dp), ref.delta_p) <= 1e-7


def _compare_histories(h_gpu, res, tol):
    assert len(h_gpu) == len(res.history)
    for g, o in zip(h_gpu, res.history):
        assert g.accepted == o.accepted
        assert g.pcg_iters >= 1
        for a, b in ((g.cost, o.cost), (g.radius, o.radius), (g.step_norm, o.step_norm)):
            assert abs(a - b) <= tol * abs(b), (a, b)
        if np.isinf(o.cost_candidate):
            assert np.isinf(g.cost_candidate)
        else:
            assert abs(g.cost_candidate - o.cost_candidate) <= tol * o.cost_candidate
            assert abs(g.model_decrease - o.model_decrease) <= tol * abs(o.model_decrease)


@pytest.mark.parametrize("start", ["perturbed", "hard"])
def test_lm_solve_matches_oracle(start):
    """With tight inner solves the GPU loop takes the oracle's decisions
    (accept/reject, radius, termination) and reaches its parameters. Both inner
    solves stop at rtol 1e-11, so their steps agree to about cond(S) times
    that: 1e-8 from the perturbed start, 1e-6 from the hard start whose points
    sit 0.3 m in front of a camera."""
    import paper_2007_01941_amd as bamg
    sc = tiny_scene(10, 150, seed=21, k_min=2, k_max=5)
    pts0 = sc.pts if start == "perturbed" else hard_start(sc)
    lo = bamg.LMOptions(max_iters=12)
    plan, opts = plan_for(sc, precond="bj", rtol=1e-11, max_iter=5000)
    cams, pts, uv = inputs(sc, pts=pts0)
    out = plan.lm_solve(cams, pts, uv, opts=opts, lm_opts=lo)
    res = olm.solve(sc.cams, pts0, sc.obs_cam, sc.obs_pt, sc.uv, olm.LMOptions(max_iters=12), method="bj",
                    rtol=1e-11)
    print(f"[gpu] lm {start}: iters {out.iters} accepted {out.accepted} term {out.termination} "
          f"cost {out.cost0:.6e} -> {out.cost:.10e} (oracle {res.cost:.10e}, term {res.termination}) "
          f"decisions {[int(h.accepted) for h in out.history]}", flush=True)
    tol = 1e-8 if start == "perturbed" else 1e-6
    _compare_histories(out.history, res, tol)
    term = {"max_iters": olm.TERM_MAX_ITERS, "function_tol": olm.TERM_FUNCTION,
            "parameter_tol": olm.TERM_PARAMETER, "min_radius": olm.TERM_RADIUS}[out.termination]
    assert term == res.termination
    assert abs(out.cost - res.cost) <= tol * res.cost
    assert rel(host(cams), res.cams) <= tol and rel(host(pts), res.pts) <= tol
    # the returned parameters have the reported cost
    c, bad = plan.cost(cams, pts, uv)
    assert bad == 0 and abs(c - out.cost) <= 1e-12 * out.cost


def test_lm_solve_multigrid_nash_sofer():
    """LM with the multigrid preconditioner and a constant forcing tau = 0.1
    (the paper's setting) against the oracle's loop with the same rule: the
    same minimum, monotone accepted costs, far fewer PCG iterations than tight
    solves."""
    import paper_2007_01941_amd as bamg
    sc = scene("ring64")
    lo = bamg.LMOptions(max_iters=25)
    plan, opts = plan_for(sc, precond="mg", rtol=1e-12, coarse_max_nodes=16, stop_rule="nash_sofer",
                          forcing=0.1)
    cams, pts, uv = inputs(sc)
    out = plan.lm_solve(cams, pts, uv, opts=opts, lm_opts=lo)
    res = olm.solve(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, olm.LMOptions(max_iters=25), method="mg",
                    rtol=1e-12, forcing=0.1, mg_opts=omg.MGOptions(coarse_max_nodes=16))
    print(f"[gpu] lm ring64 mg tau 0.1: iters {out.iters} pcg {out.pcg_iters} term {out.termination} "
          f"cost {out.cost:.10e} (oracle {res.cost:.10e}, pcg {sum(h.pcg_iters for h in res.history)}) "
          f"{out.t_ms:.1f} ms", flush=True)
    assert out.termination == "function_tol" and res.termination == olm.TERM_FUNCTION
    assert [h.accepted for h in out.history] == [h.accepted for h in res.history]
    assert abs(out.cost - res.cost) <= 1e-6 * res.cost
    prev = out.cost0
    for h in out.history:
        if h.accepted:
            assert h.cost_candidate < prev
            prev = h.cost_candidate
    assert out.pcg_iters <= 10 * out.iters



def test_lm_survives_breakdowns():
    """With almost no damping (radius 1e12) from the hard start the damped
    systems can stop being numerically positive definite; the loop treats such
    a step as failed (infinite candidate cost, radius shrunk as for a
    rejection) instead of aborting, and still lowers the cost. Whether a system
    this close to singular still counts as positive definite is decided by
    rounding, so the two sides need not fail at the same iterations; but a
    failed step and a rejected one update the radius alike, so the oracle's
    loop from the same start must reject wherever the GPU failed and take the
    same accept/reject decisions and radii throughout."""
    import paper_2007_01941_amd as bamg
    sc = tiny_scene(10, 150, seed=21, k_min=2, k_max=5)
    pts0 = hard_start(sc)
    plan, opts = plan_for(sc, precond="bj", rtol=1e-10, max_iter=5000)
    cams, pts, uv = inputs(sc, pts=pts0)
    out = plan.lm_solve(cams, pts, uv, opts=opts, lm_opts=bamg.LMOptions(max_iters=25, radius0=1e12))
    failed = [i for i, h in enumerate(out.history) if np.isinf(h.cost_candidate) and h.step_norm == 0.0]
    res = olm.solve(sc.cams, pts0, sc.obs_cam, sc.obs_pt, sc.uv, olm.LMOptions(max_iters=25, radius0=1e12),
                    method="bj", rtol=1e-10, max_pcg=5000)
    failed_ref = [i for i, h in enumerate(res.history) if np.isinf(h.cost_candidate) and h.step_norm == 0.0]
    print(f"[gpu] lm breakdowns at iterations {failed} (oracle {failed_ref}); "
          f"cost {out.cost0:.3e} -> {out.cost:.3e} (oracle {res.cost:.3e})", flush=True)
    assert failed
    assert all(not res.history[i].accepted for i in failed)
    assert [h.accepted for h in out.history] == [h.accepted for h in res.history]
    for h, r in zip(out.history, res.history):
        assert abs(h.radius - r.radius) <= 1e-6 * r.radius   # rho differs by rounding
    # a failed step's PCG work is counted in the history
    assert all(h.pcg_iters >= 0 for h in out.history)
    assert out.pcg_iters == sum(h.pcg_iters for h in out.history)
    nu = 2.0
    for a, b in zip(out.history, out.history[1:]):
        if a.accepted:
            nu = 2.0
        else:
            assert b.radius == a.radius / nu
            nu *= 2.0
    assert out.cost < out.cost0
    assert abs(out.cost - res.cost) <= 1e-6 * res.cost
