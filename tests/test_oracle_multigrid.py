"""Pins for the oracle's aggregation (Section 3.2), prolongation (3.3),
smoother (3.4), V-cycle (Algorithm 1) and PCG."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import aggregation as ag
from oracle import multigrid as mg
from oracle import nullspace, step
from scenes import tiny_scene
from tests._fixtures import case_matrix, parse_aggregation_cases, scene


# ------------------------------------------------------------------ aggregation

@pytest.mark.parametrize("case", parse_aggregation_cases(), ids=lambda c: c["name"])
def test_aggregation_hand_worked(case):
    W = sp.csr_matrix(case_matrix(case))
    agg, n_agg = ag.aggregate(W)
    assert list(agg) == case["expect"]
    assert n_agg == max(case["expect"]) + 1


def test_cap_and_leftover_rule():
    # 25-clique, equal weights: 0..19 fill aggregate 0 (cap 20); 20 pairs with 21;
    # 22..24 join it.  21-clique: node 20 finds every neighbour in a full
    # aggregate and joins its first neighbour's aggregate (leftover rule).
    for n, expect in [(25, [0] * 20 + [1] * 5), (21, [0] * 21)]:
        W = np.full((n, n), 3, dtype=np.int64)
        np.fill_diagonal(W, 10)
        agg, _ = ag.aggregate(sp.csr_matrix(W))
        assert list(agg) == expect


def test_covisibility_brute_force():
    sc = tiny_scene(9, 70, seed=4)
    W = ag.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt).toarray()
    seen = [set(sc.obs_pt[sc.obs_cam == c]) for c in range(sc.n_cam)]
    for i in range(sc.n_cam):
        for j in range(sc.n_cam):
            assert W[i, j] == len(seen[i] & seen[j])


def _random_graph(rng, n, p):
    V = (rng.random((n, 3 * n)) < p).astype(np.int64)
    return sp.csr_matrix(V @ V.T)


@pytest.mark.parametrize("seed", range(6))
def test_aggregation_invariants(seed):
    rng = np.random.default_rng(seed)
    W = _random_graph(rng, 60, 0.05)
    agg, n_agg = ag.aggregate(W, cap=5)
    assert agg.min() == 0 and agg.max() == n_agg - 1
    Wd = W.toarray()
    sizes = np.bincount(agg, minlength=n_agg)
    for a in range(n_agg):
        mem = np.nonzero(agg == a)[0]
        # connected in the strength graph
        seen, stack = {mem[0]}, [mem[0]]
        while stack:
            i = stack.pop()
            for j in mem:
                if j not in seen and Wd[i, j] > 0:
                    seen.add(j)
                    stack.append(j)
        assert len(seen) == len(mem)
        if sizes[a] > 5:
            # over the cap only through the leftover rule: such a node had all
            # its neighbours in full aggregates
            pass
        if sizes[a] == 1:
            i = mem[0]
            assert np.count_nonzero(Wd[i]) == 1      # isolated node
    # creation order: the first member of aggregate a precedes that of a+1
    firsts = [np.nonzero(agg == a)[0][0] for a in range(n_agg)]
    assert firsts == sorted(firsts)


def test_street_scene_aggregate_sizes():
    # Section 3.2 reports aggregate sizes usually between 3 and 8, mean a
    # little above 3, on street-view problems (a sanity band, not exact)
    sc = scene("city200")
    W = ag.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    agg, n_agg = ag.aggregate(W)
    sizes = np.bincount(agg)
    assert 2.0 <= sizes.mean() <= 5.0
    assert np.percentile(sizes, 90) <= 8


# ------------------------------------------------------------------ prolongation

def test_splitmix64_published_value():
    # first output of a splitmix64 generator seeded with 0
    assert mg.splitmix64(0) == 0xE220A8397B1DCDAF
    assert mg.splitmix64(0x9E3779B97F4A7C15) == 0x6E789E6AA1B965F4


def test_qr_invariants():
    rng = np.random.default_rng(1)
    for rows in (18, 27, 45, 320):
        K = rng.normal(size=(rows, 16))
        Q, R = mg.householder_qr(K)
        np.testing.assert_allclose(Q.T @ Q, np.eye(16), atol=1e-13)
        np.testing.assert_allclose(Q @ R, K, atol=1e-12 * np.abs(K).max())
        assert np.all(np.tril(R, -1) == 0) or np.abs(np.tril(R, -1)).max() < 1e-14
        assert np.all(np.diag(R) >= 0)


def test_prolongator_represents_near_nullspace():
    sc = scene("city200")
    W = ag.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    agg, n_agg = ag.aggregate(W)
    K0 = nullspace.camera_nullspace(sc.cams)
    Pb, Kc, P = mg.tentative_prolongator(K0, agg, n_agg)
    Kf = K0.reshape(-1, 16)
    np.testing.assert_allclose(P @ (P.T @ Kf), Kf, atol=1e-10 * np.abs(Kf).max())
    # P K_coarse = K: the coarse near-nullspace reproduces the fine one
    np.testing.assert_allclose(P @ Kc.reshape(-1, 16), Kf, atol=1e-10 * np.abs(Kf).max())
    PtP = (P.T @ P).toarray()
    np.testing.assert_allclose(PtP, np.eye(PtP.shape[0]), atol=1e-12)


def test_coarse_operator_inherits_gauge_nullspace():
    sc = scene("ring64")
    D = np.zeros(9 * sc.n_cam + 3 * sc.n_pt)
    nrm = step.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, D=D)
    S = nrm.S_sparse()
    W = ag.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    agg, n_agg = ag.aggregate(W)
    K0 = nullspace.camera_nullspace(sc.cams)
    Pb, Kc, P = mg.tentative_prolongator(K0, agg, n_agg)
    S1 = (P.T @ S @ P).toarray()
    G = Kc.reshape(-1, 16)[:, 9:16]
    assert np.abs(S1 @ G).max() <= 1e-8 * np.abs(S1).max() * np.abs(G).max()
    # Galerkin product in sparse form equals the dense triple product
    Sd = S.toarray()
    Pd = P.toarray()
    np.testing.assert_allclose(S1, Pd.T @ Sd @ Pd, atol=1e-10 * np.abs(S1).max())


# ------------------------------------------------------------------ smoother

def test_chebyshev_closed_form_on_diagonal():
    # for A = diag(lam), D = I: the error after m steps from x0 = 0 is
    # T_m((theta - lam)/delta) / T_m(theta/delta) times the initial error.
    lam = np.linspace(0.05, 1.0, 40)
    A = lambda v: lam * v
    Dinv = np.ones((40, 1, 1))
    b = np.ones(40)
    lmax = 1.0
    lo, hi = 0.3, 1.1
    theta, delta = 0.5 * (hi + lo) * lmax, 0.5 * (hi - lo) * lmax
    Tm = lambda m, x: np.cosh(m * np.arccosh(x)) if np.all(np.abs(x) >= 1) else \
        np.polynomial.chebyshev.chebval(x, [0] * m + [1])
    for m in (1, 2, 3, 5):
        x, r = mg.chebyshev(A, Dinv, b, np.zeros(40), lmax, m, lo, hi, r=b.copy())
        e = 1.0 / lam - x                    # exact solution 1/lam
        poly = np.polynomial.chebyshev.chebval((theta - lam) / delta, [0] * m + [1]) / \
            np.polynomial.chebyshev.chebval(theta / delta, [0] * m + [1])
        np.testing.assert_allclose(e, poly / lam, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(r, b - lam * x, atol=1e-12)


def test_lanczos_exact_with_few_distinct_eigenvalues():
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(30, 30)))
    ev = np.repeat([0.5, 1.0, 2.0, 7.0], [10, 8, 7, 5])
    A = (Q * ev) @ Q.T
    Dblk = np.eye(30)[None]
    got = mg.lanczos_lmax(lambda v: A @ v, Dblk, rng.normal(size=30), 5)
    assert abs(got - 7.0) < 1e-10


def test_lanczos_generalized_below_true_max():
    sc = scene("ring64")
    nrm = step.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
    S = nrm.S_dense()
    B = nrm.block_jacobi_blocks()
    Binv = np.linalg.inv(B)
    est = mg.lanczos_lmax(lambda v: S @ v, Binv, mg.lanczos_start(S.shape[0], 0), 5)
    Dm = np.zeros_like(S)
    for c in range(sc.n_cam):
        Dm[9 * c:9 * c + 9, 9 * c:9 * c + 9] = B[c]
    L = np.linalg.cholesky(Dm)
    Li = np.linalg.inv(L)
    true = np.linalg.eigvalsh(Li @ S @ Li.T)[-1]
    assert est <= true * (1 + 1e-12)
    assert est >= 0.5 * true


# ------------------------------------------------------------------ V-cycle, PCG

def _hier(sc, **kw):
    nrm = step.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
    return nrm, step.hierarchy_for(nrm, sc.cams, sc.obs_cam, sc.obs_pt, mg.MGOptions(**kw))


def test_vcycle_is_symmetric():
    sc = scene("city200")
    nrm, lev = _hier(sc, coarse_max_nodes=16)
    assert len(lev) >= 3
    rng = np.random.default_rng(2)
    x, y = rng.normal(size=9 * sc.n_cam), rng.normal(size=9 * sc.n_cam)
    Mx, My = mg.vcycle(lev, x), mg.vcycle(lev, y)
    assert abs(Mx @ y - x @ My) <= 1e-12 * np.sqrt((Mx @ x) * (My @ y))
    assert Mx @ x > 0 and My @ y > 0


def test_single_level_hierarchy_solves_in_one_iteration():
    sc = scene("ring20")            # 20 cameras <= 128: the coarsest level is level 0
    nrm, lev = _hier(sc)
    assert len(lev) == 1
    res = mg.pcg(nrm.S_apply, lambda r: mg.vcycle(lev, r), nrm.rhs(), 1e-8)
    assert res.iters == 1


def test_mg_pcg_converges_to_direct_solution():
    sc = scene("ring64")
    full = step.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="full")
    res = step.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="mg", rtol=1e-12,
                       opts=mg.MGOptions(coarse_max_nodes=8))
    assert res.converged and len(res.levels) >= 3
    assert np.linalg.norm(res.delta_c - full.delta_c) <= 1e-7 * np.linalg.norm(full.delta_c)
    assert np.linalg.norm(res.delta_p - full.delta_p) <= 1e-7 * np.linalg.norm(full.delta_p)


def test_mg_beats_block_jacobi_on_street_scene():
    sc = scene("city200")
    bj = step.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="bj", rtol=1e-6)
    m = step.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="mg", rtol=1e-6,
                     opts=mg.MGOptions(coarse_max_nodes=16))
    assert m.converged and bj.converged
    assert m.iters < bj.iters


def test_strength_order_is_exact():
    # The neighbour order against an independent exact formulation: sorting by
    # the squared strength G_ij^2 = W_ij^2 / (W_ii W_jj) as an exact rational
    # (descending; ties by index). Random rows with many exact ties.
    from fractions import Fraction
    rng = np.random.default_rng(11)
    for _ in range(20):
        n = 30
        V = (rng.random((n, 12)) < 0.3).astype(np.int64)
        V[:, 0] = 1                           # every pair covisible
        W = V @ V.T
        orders = ag.neighbour_order(sp.csr_matrix(W))
        for i in range(n):
            ref = sorted((j for j in range(n) if j != i and W[i, j] > 0),
                         key=lambda j: (-Fraction(int(W[i, j]) ** 2, int(W[i, i]) * int(W[j, j])), j))
            assert orders[i] == ref
