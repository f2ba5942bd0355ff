"""GPU parity on the largest single-GPU scene: a 4 x 4 km city grid of 100 m
blocks, 30,000 cameras with loop closures every 500 cameras, 12M points with
heavy-tailed visibility (2-15 views), ~78M observations. At this size the
aggregation of level 0 runs in global memory (k_aggregate_global), a path no
smaller scene takes. Checked: the covisibility counts and the aggregates of
every level bit for bit against the oracle; Jacobian blocks of sampled
observations; for sampled cameras the rows of b, S_cc and S x from the
oracle's exact local sub-problem; the mixed-precision multigrid step (the
precision form this scene is measured in) by its residual under the FP64
product, against the FP64 step."""
import time

import numpy as np
import pytest

from oracle import aggregation as agglib, camera
from oracle.multigrid import MGOptions
from tests._fixtures import scene
from tests._gpu import dev, host, inputs, plan_for, rel
from tests.test_gpu_large import local_problem
from tests.test_gpu_step import TOL_U, block_jacobi_abs, rhs_abs, schur_abs

pytestmark = pytest.mark.gpu

BENCH = dict(rtol=1e-6, max_iter=5000)


@pytest.fixture(scope="module")
def city():
    t = time.time()
    print("[gpu] generating city30k ...", flush=True)
    sc = scene("city30k")
    print(f"[gpu] city30k: {sc.n_cam} cameras, {sc.n_pt} points, {sc.n_obs} observations "
          f"({time.time() - t:.0f} s)", flush=True)
    plan, opts = plan_for(sc, precond="mg", precision="mixed", **BENCH)
    return sc, plan, opts


def test_city30k_aggregation_bit_exact(city):
    sc, plan, _ = city
    W = agglib.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    nodes = plan.mg_levels()
    print(f"[gpu] city30k levels {nodes}", flush=True)
    assert nodes[0] * 2 * 4 > 150 * 1024     # level 0 aggregates in global memory
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


def test_city30k_jacobian_sampled(city):
    sc, plan, _ = city
    f, F, E = (host(t) for t in plan.eval_jacobian(*inputs(sc)))
    idx = np.random.default_rng(7).choice(sc.n_obs, 20000, replace=False)
    F_ref, E_ref = camera.jacobian_blocks(sc.cams, sc.pts, sc.obs_cam[idx], sc.obs_pt[idx])
    f_ref = camera.residuals(sc.cams, sc.pts, sc.obs_cam[idx], sc.obs_pt[idx], sc.uv[idx])
    assert np.abs(f[idx] - f_ref).max() <= 1e-9 * max(1.0, np.abs(f_ref).max())
    for got, ref in ((F[idx], F_ref), (E[idx], E_ref)):
        scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
        assert (np.abs(got - ref) / scale).max() <= 1e-11


def test_city30k_rows_sampled(city):
    sc, plan, opts = city
    plan.prepare(*inputs(sc), opts=opts)
    b, Cinv, Scc = (host(t) for t in plan.step_blocks())
    rng = np.random.default_rng(8)
    cams_sel = np.sort(rng.choice(sc.n_cam, 6, replace=False))
    sub, pts_sel = local_problem(sc, cams_sel)
    # this scene has short-baseline points (cond(C_p) up to ~1e4 among these
    # cameras' points): the bounds carry cond(C_p) (see schur_abs)
    print(f"[gpu] city30k sampled cameras {cams_sel}: {sub.n_pt} points, "
          f"max cond(C_p) {np.linalg.cond(sub.C).max():.1e}", flush=True)
    assert np.all(np.abs(b[cams_sel] - sub.rhs().reshape(-1, 9)[cams_sel])
                  <= TOL_U * rhs_abs(sub, cond=True)[cams_sel])
    err = np.abs(Cinv[pts_sel] - sub.Cinv).max(axis=(1, 2))
    assert np.all(err <= 1e-10 * np.linalg.cond(sub.C) * np.abs(sub.Cinv).max(axis=(1, 2)))
    Babs = block_jacobi_abs(sub, cond=True)
    assert np.all(np.abs(Scc[cams_sel] - sub.block_jacobi_blocks()[cams_sel]) <= TOL_U * Babs[cams_sel])
    x = rng.normal(size=(sc.n_cam, 9))
    y_ref = sub.S_apply(x).reshape(-1, 9)
    bound = schur_abs(sub, x, cond=True)
    y64 = host(plan.schur_apply(dev(x), "fp64"))
    y32 = host(plan.schur_apply(dev(x), "mixed"))
    assert np.all(np.abs(y64[cams_sel] - y_ref[cams_sel]) <= TOL_U * bound[cams_sel])
    assert np.all(np.abs(y32[cams_sel] - y_ref[cams_sel]) <= 1e-4 * bound[cams_sel])


def test_city30k_mixed_step(city):
    sc, plan, opts = city
    import paper_2007_01941_amd as bamg
    dc32, dp32, st32 = plan.lm_step(*inputs(sc), opts=opts)
    fp64 = bamg.Options(precond="mg", **BENCH)
    dc64, dp64, st64 = plan.lm_step(*inputs(sc), opts=fp64)
    plan.prepare(*inputs(sc), opts=fp64)
    b = host(plan.step_blocks()[0])

    def res(dc):
        r = b - host(plan.schur_apply(dev(dc)))
        return float(np.linalg.norm(r) / np.linalg.norm(b))

    r32, r64 = res(host(dc32)), res(host(dc64))
    print(f"[gpu] city30k: mixed iters {st32.iters} refine {st32.refine_steps} res {r32:.2e}; "
          f"fp64 iters {st64.iters} res {r64:.2e}; |mixed - fp64| / |fp64| "
          f"{rel(host(dc32), host(dc64)):.2e}", flush=True)
    assert st32.converged and st64.converged and not st32.fallback_fp64
    assert r32 <= 2 * BENCH["rtol"] and r64 <= 2 * BENCH["rtol"]
    # delta_p of the points of sampled cameras against the oracle's back-substitution
    cams_sel = np.sort(np.random.default_rng(9).choice(sc.n_cam, 4, replace=False))
    sub, pts_sel = local_problem(sc, cams_sel)
    dp_ref = sub.recover_points(host(dc64).ravel(), -sub.g_p.ravel())
    assert rel(host(dp64)[pts_sel], dp_ref) <= 1e-9
