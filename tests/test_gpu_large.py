"""GPU parity on the long-path scene (10,000 cameras along a 5 km path without
loop closures, 4M points, ~25M observations), the workload of the precision
form. The oracle cannot form this system in a test's time, so it checks the
GPU by outputs it can compute one by one: the Jacobian blocks of sampled
observations, and, for sampled cameras, the rows of b, S_cc and S x, which
depend only on the points those cameras see and all observations of those
points (a local sub-problem of the oracle); C^-1 and the back-substituted
delta_p for sampled points; aggregation bit for bit on every level; and the
FP64 and mixed steps by their residuals under the (sample-checked) product."""
import numpy as np
import pytest

from oracle import aggregation as agglib, camera
from oracle.multigrid import MGOptions
from oracle.normal import Normal
from tests._fixtures import scene
from tests._gpu import dev, host, inputs, plan_for, rel
from tests.test_gpu_step import TOL_U, rhs_abs, schur_abs

pytestmark = pytest.mark.gpu

BENCH = dict(rtol=1e-6, max_iter=5000)


@pytest.fixture(scope="module")
def path():
    sc = scene("path10k")
    plan, opts = plan_for(sc, precond="mg", **BENCH)
    return sc, plan, opts


def local_problem(sc, cams_sel):
    """Oracle normal equations restricted to the points seen by cams_sel and
    all observations of those points: exact for the rows of cams_sel."""
    pts_sel = np.unique(sc.obs_pt[np.isin(sc.obs_cam, cams_sel)])
    keep = np.isin(sc.obs_pt, pts_sel)
    oc, op = sc.obs_cam[keep], sc.obs_pt[keep]
    local = np.searchsorted(pts_sel, op)
    F, E = camera.jacobian_blocks(sc.cams, sc.pts, oc, op)
    f = camera.residuals(sc.cams, sc.pts, oc, op, sc.uv[keep])
    return Normal(F, E, f, oc, local, sc.n_cam, pts_sel.shape[0]), pts_sel


def test_large_jacobian_sampled(path):
    sc, plan, _ = path
    f, F, E = (host(t) for t in plan.eval_jacobian(*inputs(sc)))
    idx = np.random.default_rng(3).choice(sc.n_obs, 20000, replace=False)
    F_ref, E_ref = camera.jacobian_blocks(sc.cams, sc.pts, sc.obs_cam[idx], sc.obs_pt[idx])
    f_ref = camera.residuals(sc.cams, sc.pts, sc.obs_cam[idx], sc.obs_pt[idx], sc.uv[idx])
    assert np.abs(f[idx] - f_ref).max() <= 1e-9 * max(1.0, np.abs(f_ref).max())
    for got, ref in ((F[idx], F_ref), (E[idx], E_ref)):
        scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
        assert (np.abs(got - ref) / scale).max() <= 1e-11


def test_large_rows_sampled(path):
    sc, plan, opts = path
    plan.prepare(*inputs(sc), opts=opts)
    b, Cinv, Scc = (host(t) for t in plan.step_blocks())
    rng = np.random.default_rng(4)
    cams_sel = np.sort(rng.choice(sc.n_cam, 6, replace=False))
    sub, pts_sel = local_problem(sc, cams_sel)
    b_ref = sub.rhs().reshape(-1, 9)
    bb = rhs_abs(sub)
    assert np.all(np.abs(b[cams_sel] - b_ref[cams_sel]) <= TOL_U * bb[cams_sel])
    S_ref = sub.block_jacobi_blocks()
    from oracle.normal import block_sum
    Babs = np.abs(sub.A) + block_sum(sub.obs_cam, np.einsum("nij,njk,nlk->nil", np.abs(sub.Y),
                                                           np.abs(sub.Cinv[sub.obs_pt]), np.abs(sub.Y)),
                                     sub.n_cam)
    assert np.all(np.abs(Scc[cams_sel] - S_ref[cams_sel]) <= TOL_U * Babs[cams_sel])
    err = np.abs(Cinv[pts_sel] - sub.Cinv).max(axis=(1, 2))
    cond = np.linalg.cond(sub.C)
    assert np.all(err <= 1e-10 * cond * np.abs(sub.Cinv).max(axis=(1, 2)))
    x = rng.normal(size=(sc.n_cam, 9))
    y = host(plan.schur_apply(dev(x)))
    y_ref = sub.S_apply(x).reshape(-1, 9)
    bound = schur_abs(sub, x)
    assert np.all(np.abs(y[cams_sel] - y_ref[cams_sel]) <= TOL_U * bound[cams_sel])


def test_large_aggregation_bit_exact(path):
    sc, plan, _ = path
    W = agglib.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    nodes = plan.mg_levels()
    o = MGOptions()
    for l in range(len(nodes)):
        assert W.shape[0] == nodes[l]
        rp, col, val = (host(t) for t in plan.mg_covisibility(l))
        W.sort_indices()
        assert np.array_equal(rp, W.indptr) and np.array_equal(col, W.indices)
        assert np.array_equal(val, W.data)
        if l + 1 == len(nodes):
            break
        agg, n_agg = agglib.aggregate(W, o.agg_cap)
        assert np.array_equal(host(plan.mg_aggregates(l)), agg)
        W = agglib.coarse_covisibility(W, agg, n_agg)


def _residual(plan, b, dc):
    r = b - host(plan.schur_apply(dev(dc)))
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def test_large_steps_fp64_and_mixed(path):
    """The precision form against the all-FP64 GPU path at rtol 1e-6 (both
    by their true residual under the FP64 product), and delta_p of sampled
    points against the oracle's back-substitution."""
    sc, plan, opts = path
    import paper_2007_01941_amd as bamg
    dc64, dp64, st64 = plan.lm_step(*inputs(sc), opts=opts)
    plan.prepare(*inputs(sc), opts=opts)
    b = host(plan.step_blocks()[0])
    res64 = _residual(plan, b, host(dc64))
    mixed = bamg.Options(precond="mg", precision="mixed", **BENCH)
    dc32, dp32, st32 = plan.lm_step(*inputs(sc), opts=mixed)
    plan.prepare(*inputs(sc), opts=opts)
    res32 = _residual(plan, b, host(dc32))
    diff = rel(host(dc32), host(dc64))
    print(f"[gpu] path10k: fp64 iters {st64.iters} res {res64:.2e}; mixed iters {st32.iters} "
          f"refine {st32.refine_steps} fp64 fallback {st32.fallback_fp64} res {res32:.2e}; "
          f"|mixed - fp64| / |fp64| {diff:.2e}; levels {st64.nodes}", flush=True)
    assert st64.converged and st32.converged
    # the FP32 inner solves stay well defined on this deep hierarchy (the
    # coarse levels of the FP32 V-cycle run in FP64), so no FP64 finish
    assert not st32.fallback_fp64
    assert res64 <= 2 * BENCH["rtol"] and res32 <= 2 * BENCH["rtol"]
    # delta_p = C^-1 (-g_p - W^T delta_c) for the points of sampled cameras
    rng = np.random.default_rng(5)
    cams_sel = np.sort(rng.choice(sc.n_cam, 4, replace=False))
    sub, pts_sel = local_problem(sc, cams_sel)
    # the local problem holds every observation of its points
    dp_ref = sub.recover_points(host(dc64).ravel(), -sub.g_p.ravel())
    assert rel(host(dp64)[pts_sel], dp_ref) <= 1e-9
