"""GPU parity of smoothed-aggregation multigrid (the alternative prolongator
that Section 3.5 and the scaling experiment of Section 5.2 weigh against the
paper's unsmoothed one) against the oracle's smooth_prolongator variant,
through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import multigrid as omg, step as ostep
from tests._fixtures import scene
from tests._gpu import host, inputs, plan_for, rel
from tests.test_gpu_step import TOL_U, _full_rank, rhs_abs, schur_abs

pytestmark = pytest.mark.gpu

OMEGA = 4.0 / 3.0


def _oracle_levels(sc):
    nrm = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
    lev = ostep.hierarchy_for(nrm, sc.cams, sc.obs_cam, sc.obs_pt,
                              omg.MGOptions(coarse_max_nodes=16, smooth_prolongator=True))
    return nrm, lev


def _tentative_dense(Pb, agg, n_next):
    """Dense [n bs][n_next 16] matrix of tentative blocks Pb [n][bs][16]."""
    n, bs, _ = Pb.shape
    P = np.zeros((n * bs, n_next * 16))
    for i in range(n):
        P[i * bs:(i + 1) * bs, 16 * agg[i]:16 * agg[i] + 16] = Pb[i]
    return P


def _blockdiag(B):
    n, bs, _ = B.shape
    D = np.zeros((n * bs, n * bs))
    for i in range(n):
        D[i * bs:(i + 1) * bs, i * bs:(i + 1) * bs] = B[i]
    return D


@pytest.mark.parametrize("name", ["ring64", "city200"])
def test_smoothed_prolongator_and_galerkin_on_gpu_data(name):
    """On every level, from the GPU's own P_t, D^-1, lambda_max and operator:
    P_s = (I - w/lambda D^-1 S) P_t and S_{l+1} = P_s^T S_l P_s, within the
    rounding bound of the products' terms."""
    sc = scene(name)
    plan, opts = plan_for(sc, precond="mg", coarse_max_nodes=16, prolongator="smoothed")
    plan.prepare(*inputs(sc), opts=opts)
    nodes = plan.mg_levels()
    print(f"[gpu] {name} smoothed levels {nodes}", flush=True)
    assert len(nodes) >= 3
    for l in range(len(nodes) - 1):
        S = host(plan.mg_level_data(l, "operator"))
        Pt = _tentative_dense(host(plan.mg_level_data(l, "P")), host(plan.mg_aggregates(l)), nodes[l + 1])
        Dinv = _blockdiag(host(plan.mg_level_data(l, "Dinv")))
        lam = float(host(plan.mg_level_data(l, "lmax"))[0])
        Ps = host(plan.mg_level_data(l, "P_smoothed"))
        c = OMEGA / lam
        ref = Pt - c * (Dinv @ (S @ Pt))
        bound = np.abs(Pt) + c * (np.abs(Dinv) @ (np.abs(S) @ np.abs(Pt)))
        assert np.all(np.abs(Ps - ref) <= TOL_U * bound), l
        # the pattern: nonzero exactly where some operator neighbour's aggregate is
        assert np.count_nonzero(Ps) > np.count_nonzero(Pt)
        S1 = host(plan.mg_level_data(l + 1, "operator"))
        ref1 = Ps.T @ S @ Ps
        bound1 = np.abs(Ps).T @ np.abs(S) @ np.abs(Ps)
        assert np.all(np.abs(S1 - ref1) <= TOL_U * bound1), l
        assert np.allclose(S1, S1.T, rtol=0, atol=TOL_U * bound1.max())


def test_smoothed_prolongator_matches_oracle():
    """Level 0 against the oracle by value: lambda_max of D^-1 S (five steps of
    generalized Lanczos, Section 3.4) and every column block P_s[:, a] of an
    aggregate whose K_a has full column rank (that block depends only on a's
    own tentative blocks, which are then unique)."""
    sc = scene("city200")
    plan, opts = plan_for(sc, precond="mg", coarse_max_nodes=16, prolongator="smoothed")
    plan.prepare(*inputs(sc), opts=opts)
    nrm, lev = _oracle_levels(sc)
    L0 = lev[0]
    assert np.array_equal(host(plan.mg_aggregates(0)), L0.agg)
    assert plan.mg_levels() == [l.S.shape[0] // l.bs for l in lev]
    lam = float(host(plan.mg_level_data(0, "lmax"))[0])
    assert abs(lam - L0.lmax) <= 1e-10 * L0.lmax
    Ps = host(plan.mg_level_data(0, "P_smoothed"))
    Ps_ref = L0.P.toarray()
    S0 = nrm.S_dense()
    Dinv = np.abs(_blockdiag(np.linalg.inv(omg.block_diagonal(S0, 9))))
    Pt = np.abs(_tentative_dense(L0.Pb, L0.agg, L0.n_agg))
    mag = Pt + (OMEGA / L0.lmax) * (Dinv @ (np.abs(S0) @ Pt))
    full = [a for a in range(L0.n_agg) if _full_rank(L0.Kc[a])]
    assert len(full) >= L0.n_agg // 3
    for a in full:
        cols = slice(16 * a, 16 * a + 16)
        tol = (2e-13 * np.linalg.cond(L0.Kc[a]) + 1e-10) * mag[:, cols]
        assert np.all(np.abs(Ps[:, cols] - Ps_ref[:, cols]) <= tol), a
    print(f"[gpu] P_s column blocks compared by value: {len(full)} of {L0.n_agg}", flush=True)


@pytest.mark.parametrize("level0_op", ["auto", "implicit"])
@pytest.mark.parametrize("name", ["ring64", "city200"])
def test_smoothed_step_matches_oracle(name, level0_op):
    """The PCG step with the smoothed-aggregation V-cycle reaches the oracle's
    step, in about the oracle's iterations, and in fewer iterations than the
    unsmoothed hierarchy on the same scene (the observation of Section 3.5)."""
    sc = scene(name)
    plan, opts = plan_for(sc, precond="mg", rtol=1e-10, coarse_max_nodes=16, prolongator="smoothed",
                          level0_op=level0_op)
    dc, dp, st = plan.lm_step(*inputs(sc))
    ref = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="mg", rtol=1e-10,
                        opts=omg.MGOptions(coarse_max_nodes=16, smooth_prolongator=True))
    plain, _ = plan_for(sc, precond="mg", rtol=1e-10, coarse_max_nodes=16)
    _, _, st_plain = plain.lm_step(*inputs(sc))
    print(f"[gpu] {name} smoothed ({level0_op}): iters {st.iters} (oracle {ref.iters}, unsmoothed "
          f"{st_plain.iters}) err_vs_oracle {rel(host(dc), ref.delta_c):.2e}", flush=True)
    assert st.converged and st.rel_res <= 1e-10
    nrm = ref.normal
    r = nrm.rhs() - nrm.S_apply(host(dc).ravel())
    slack = TOL_U * np.linalg.norm(schur_abs(nrm, host(dc)) + rhs_abs(nrm))
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(nrm.rhs()) + slack
    assert abs(st.iters - ref.iters) <= 2
    assert rel(host(dc), ref.delta_c) <= 1e-6
    assert rel(host(dp), ref.delta_p) <= 1e-6
    assert st.iters < st_plain.iters


def test_smoothed_fill_in_and_workspace():
    """The smoothed hierarchy's coarse operators are wider (Section 3.5's
    fill-in; the oracle's patterns, block for block) and its workspace larger."""
    sc = scene("city200")
    plan, opts = plan_for(sc, precond="mg", coarse_max_nodes=16, prolongator="smoothed")
    plain, popts = plan_for(sc, precond="mg", coarse_max_nodes=16)
    plan.prepare(*inputs(sc), opts=opts)
    plain.prepare(*inputs(sc), opts=popts)
    _, lev = _oracle_levels(sc)
    for l in range(1, len(lev)):
        S = host(plan.mg_level_data(l, "operator"))
        n = S.shape[0] // 16
        blocks = np.abs(S).reshape(n, 16, n, 16).max(axis=(1, 3)) > 0
        ref = np.abs(lev[l].S.toarray()).reshape(n, 16, n, 16).max(axis=(1, 3)) > 0
        assert np.array_equal(blocks, ref), l
        Sp = host(plain.mg_level_data(l, "operator"))
        nz_plain = np.count_nonzero(np.abs(Sp).reshape(n, 16, n, 16).max(axis=(1, 3)))
        print(f"[gpu] level {l}: {blocks.sum()} blocks smoothed, {nz_plain} unsmoothed", flush=True)
        assert blocks.sum() > nz_plain
    assert plan.workspace_bytes() > plain.workspace_bytes()


def test_smoothed_deterministic_mode_is_bitwise_reproducible():
    sc = scene("city200")
    plan, opts = plan_for(sc, precond="mg", rtol=1e-10, coarse_max_nodes=16, prolongator="smoothed",
                          deterministic=True)
    a = plan.lm_step(*inputs(sc))
    b = plan.lm_step(*inputs(sc))
    assert a[2].iters == b[2].iters
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_smoothed_option_errors():
    """Mixed-precision multigrid with the smoothed prolongator is refused, and
    so is a step whose prolongator differs from the plan's (C ABI)."""
    import paper_2007_01941_amd as bamg
    from paper_2007_01941_amd import _lib
    sc = scene("ring64")
    with pytest.raises(bamg.BAError) as e:
        plan_for(sc, precond="mg", precision="mixed", prolongator="smoothed")
    assert e.value.status == -1
    plan, opts = plan_for(sc, precond="mg", coarse_max_nodes=16, prolongator="smoothed")
    cams, pts, uv = inputs(sc)
    o = opts.to_c()
    o.prolongator = _lib.PROLONG_TENTATIVE
    dc = torch.empty((sc.n_cam, 9), dtype=torch.float64, device="cuda")
    dp = torch.empty((sc.n_pt, 3), dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = _lib.LIB.ba_lm_step(plan._h, ctypes.byref(o), p(cams), p(pts), p(uv), None, None, 0, p(dc), p(dp), None,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == -1 and b"smoothed" in _lib.LIB.ba_last_error()
    # the same plan still steps with its own prolongator
    _, _, s2 = plan.lm_step(cams, pts, uv)
    assert s2.converged
