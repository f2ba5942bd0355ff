"""Pins of the oracle's visibility-based block-Jacobi preconditioner (the
comparison preconditioner of Section 2.2)."""
import numpy as np

from oracle import aggregation as agglib, cluster as cl, multigrid as mg, step as ostep
from oracle.multigrid import MGOptions
from scenes import tiny_scene
from tests._fixtures import scene


def _normal(sc):
    return ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)


def test_singleton_clusters_are_point_block_jacobi():
    sc = tiny_scene(12, 200, seed=2, k_min=2, k_max=5)
    nrm = _normal(sc)
    blocks = cl.cluster_inverses(nrm.S_sparse(), np.arange(sc.n_cam), sc.n_cam)
    r = np.random.default_rng(0).normal(size=9 * sc.n_cam)
    ref = mg.apply_blocks(np.linalg.inv(nrm.block_jacobi_blocks()), r)
    assert np.allclose(cl.apply(blocks, r), ref, rtol=1e-10, atol=0)


def test_one_cluster_is_the_exact_inverse():
    """All cameras in one cluster: M = S^-1 and PCG stops after one iteration."""
    sc = tiny_scene(8, 120, seed=3, k_min=2, k_max=5)
    nrm = _normal(sc)
    blocks = cl.cluster_inverses(nrm.S_sparse(), np.zeros(sc.n_cam, dtype=int), 1)
    b = nrm.rhs()
    res = mg.pcg(nrm.S_apply, lambda r: cl.apply(blocks, r), b, 1e-10, 10)
    assert res.iters == 1


def test_cluster_blocks_are_principal_submatrices_and_spd():
    sc = tiny_scene(12, 200, seed=4, k_min=2, k_max=5)
    nrm = _normal(sc)
    S = nrm.S_dense()
    agg = np.array([0, 0, 1, 1, 1, 2, 3, 3, 3, 3, 2, 0])
    blocks = cl.cluster_inverses(nrm.S_sparse(), agg, 4)
    for mem, inv in blocks:
        assert np.array_equal(mem, np.flatnonzero(agg == agg[mem[0]]))
        # brute force: the block of S on the members, entry by entry
        blk = np.array([[S[9 * mem[i // 9] + i % 9, 9 * mem[j // 9] + j % 9] for j in range(9 * len(mem))]
                        for i in range(9 * len(mem))])
        assert np.allclose(inv @ blk, np.eye(blk.shape[0]), atol=1e-8)
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=(2, 9 * sc.n_cam))
    Mx, My = cl.apply(blocks, x), cl.apply(blocks, y)
    assert abs(x @ My - y @ Mx) <= 1e-10 * np.linalg.norm(x) * np.linalg.norm(My)
    assert x @ Mx > 0


def test_clusters_follow_the_hierarchy_rule():
    o = MGOptions()
    small = tiny_scene(12, 200, seed=4, k_min=2, k_max=5)
    W = agglib.covisibility(small.obs_cam, small.obs_pt, small.n_cam, small.n_pt)
    agg, n_agg = cl.clusters(W, o)
    assert n_agg == small.n_cam and np.array_equal(agg, np.arange(small.n_cam))
    sc = scene("city200")
    W = agglib.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    agg, n_agg = cl.clusters(W, o)
    ref, n_ref = agglib.aggregate(W, o.agg_cap)
    assert n_agg == n_ref < sc.n_cam and np.array_equal(agg, ref)


def test_cluster_jacobi_beats_point_block_jacobi_on_a_street_scene():
    sc = scene("city200")
    bj = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="bj", rtol=1e-6)
    cj = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="cj", rtol=1e-6)
    print(f"PCG iterations to 1e-6: point block Jacobi {bj.iters}, cluster block Jacobi {cj.iters}")
    assert cj.converged and cj.iters < bj.iters
