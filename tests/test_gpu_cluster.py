"""GPU parity of the visibility-based block-Jacobi preconditioner (the
comparison preconditioner of Section 2.2; clusters = level-0 aggregates)
against the oracle (oracle.cluster)."""
import numpy as np
import pytest

from oracle import aggregation as agglib, cluster as cl, step as ostep
from oracle.multigrid import MGOptions
from tests._fixtures import scene
from tests._gpu import dev, host, inputs, plan_for, rel
from tests.test_gpu_step import TOL_U, rhs_abs, schur_abs, schur_abs_dense

pytestmark = pytest.mark.gpu


def test_cluster_apply_solves_each_cluster_block():
    """z = M^-1 r: on every cluster, S_c z_c = r_c with the oracle's S, up to
    the two sides' rounding of S (TOL_U |S| |z|) and the in-place inversion's
    error (a multiple of u cond(S_c) |S_c| |z_c|; some cluster blocks of this
    scene have cond ~ 1e10, which is also why the operators are compared
    through this residual rather than entry by entry)."""
    sc = scene("city200")
    plan, opts = plan_for(sc, precond="cj")
    plan.prepare(*inputs(sc), opts=opts)
    nrm = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
    W = agglib.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    agg, n_agg = cl.clusters(W, MGOptions())
    assert n_agg < sc.n_cam
    r = np.random.default_rng(0).normal(size=9 * sc.n_cam)
    z = host(plan.precond_apply(dev(r), opts)).ravel()
    S = nrm.S_dense()
    Sabs = schur_abs_dense(nrm)
    worst, cmax = 0.0, 1.0
    for a in range(n_agg):
        mem = np.flatnonzero(agg == a)
        idx = (9 * mem[:, None] + np.arange(9)[None, :]).ravel()
        Sc = S[np.ix_(idx, idx)]
        res = np.linalg.norm(Sc @ z[idx] - r[idx])
        cond = np.linalg.cond(Sc)
        cmax = max(cmax, cond)
        bound = (TOL_U * np.linalg.norm(Sabs[np.ix_(idx, idx)] @ np.abs(z[idx]))
                 + 1e-13 * cond * np.linalg.norm(Sc, 2) * np.linalg.norm(z[idx]))
        worst = max(worst, res / bound)
        assert res <= bound, (a, len(mem))
    # and the whole operator against the oracle's, to the same first order
    zr = cl.apply(cl.cluster_inverses(nrm.S_sparse(), agg, n_agg), r)
    print(f"[gpu] city200 clusters {n_agg} (largest {np.bincount(agg).max()}, max cond {cmax:.1e}): "
          f"worst residual / bound {worst:.2e}, |z - z_oracle| / |z_oracle| {rel(z, zr):.2e}", flush=True)
    assert rel(z, zr) <= 1e-12 * cmax


def test_cluster_step():
    sc = scene("city200")
    plan, opts = plan_for(sc, precond="cj", rtol=1e-10, max_iter=5000)
    dc, dp, st = plan.lm_step(*inputs(sc))
    ref = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="cj", rtol=1e-10)
    direct = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="schur")
    nrm = ref.normal
    r = nrm.rhs() - nrm.S_apply(host(dc).ravel())
    slack = TOL_U * np.linalg.norm(schur_abs(nrm, host(dc)) + rhs_abs(nrm))
    print(f"[gpu] city200 cj: iters {st.iters} (oracle {ref.iters}) rel_res {st.rel_res:.2e} "
          f"err_vs_direct {rel(host(dc), direct.delta_c):.2e}", flush=True)
    assert st.converged
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(nrm.rhs()) + slack
    assert abs(st.iters - ref.iters) <= 2
    assert rel(host(dc), direct.delta_c) <= 1e-6 and rel(host(dp), direct.delta_p) <= 1e-6
