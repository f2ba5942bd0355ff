"""GPU parity of the two added forms: mixed precision (FP32 Schur product and
V-cycle inside FP64 iterative refinement) and differentiation (adjoint)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle import multigrid as omg
from oracle import step as ostep
from tests._fixtures import scene
from tests._gpu import dev, host, inputs, plan_for, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pc", ["bj", "mg"])
def test_mixed_precision_refinement(pc):
    sc = scene("city200")
    plan, opts = plan_for(sc, precond=pc, precision="mixed", rtol=1e-8, coarse_max_nodes=16)
    dc, dp, st = plan.lm_step(*inputs(sc))
    # the direct solve by dense Cholesky of S (the same exact step as the sparse
    # solve of the full system, in a fraction of its time)
    ref = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="schur")
    nrm = ref.normal
    res = np.linalg.norm(nrm.rhs() - nrm.S_apply(host(dc).ravel())) / np.linalg.norm(nrm.rhs())
    print(f"[gpu] mixed {pc}: refine {st.refine_steps} inner iters {st.iters} rel_res {st.rel_res:.2e} "
          f"oracle residual {res:.2e} err_vs_direct {rel(host(dc), ref.delta_c):.2e}", flush=True)
    assert st.converged and st.refine_steps >= 1
    # the FP64 outer residual is what refinement drives down; the oracle agrees
    assert st.rel_res <= 1e-8
    assert res <= 1e-7


def test_mixed_inner_solve_alone_is_fp32_accurate():
    # one refinement step: the FP32 solve alone reaches its inner tolerance
    sc = scene("city200")
    plan, opts = plan_for(sc, precond="mg", precision="mixed", rtol=1e-3, inner_rtol=1e-3,
                          max_refine=1, coarse_max_nodes=16)
    dc, dp, st = plan.lm_step(*inputs(sc))
    assert st.refine_steps == 1 and st.rel_res <= 2e-3


@pytest.mark.parametrize("pc", ["bj", "mg"])
def test_adjoint_matches_oracle_gradient(pc):
    sc = scene("ring20")
    plan, opts = plan_for(sc, precond=pc, rtol=1e-13, max_iter=5000, coarse_max_nodes=4)
    cams, pts, uv = inputs(sc)
    dc, dp, st = plan.lm_step(cams, pts, uv)
    gc, gp, gu, st2 = plan.backward(cams, pts, uv, dc, dp, 2 * dc, 2 * dp)
    (_, _), (rc, rp, ru), _ = oadj.step_and_gradient(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv,
                                                     oadj.gbar_sq)
    e = [rel(host(gc), rc), rel(host(gp), rp), rel(host(gu), ru)]
    print(f"[gpu] adjoint {pc}: rel err cams {e[0]:.2e} pts {e[1]:.2e} uv {e[2]:.2e} iters {st2.iters}",
          flush=True)
    assert max(e) <= 1e-5


def test_adjoint_directional_finite_differences():
    import paper_2007_01941_amd as bamg
    sc = scene("ring20")
    plan, opts = plan_for(sc, precond="mg", rtol=1e-13, max_iter=5000, coarse_max_nodes=4)
    cams, pts, uv = inputs(sc)
    cams.requires_grad_(True)
    pts.requires_grad_(True)
    uv.requires_grad_(True)
    dc, dp = bamg.LMStep.apply(cams, pts, uv, plan, opts)
    L = (dc * dc).sum() + (dp * dp).sum()
    L.backward()
    rng = np.random.default_rng(3)

    def loss(c, p, u):
        a, b, _ = plan.lm_step(c, p, u)
        return float((a * a).sum() + (b * b).sum())

    h = 1e-4
    for _ in range(6):
        vc, vp, vu = (torch.as_tensor(rng.normal(size=t.shape), device="cuda") for t in (cams, pts, uv))
        s = float(torch.sqrt((vc ** 2).sum() + (vp ** 2).sum() + (vu ** 2).sum()))
        vc, vp, vu = vc / s, vp / s, vu / s
        with torch.no_grad():
            fd = (loss(cams + h * vc, pts + h * vp, uv + h * vu) - loss(cams - h * vc, pts - h * vp, uv - h * vu)) / (2 * h)
        an = float((cams.grad * vc).sum() + (pts.grad * vp).sum() + (uv.grad * vu).sum())
        print(f"[gpu] fd {fd:.8e} adjoint {an:.8e}", flush=True)
        assert abs(fd - an) <= 2e-5 * abs(an) + 1e-6


def test_adjoint_with_explicit_damping():
    """A step taken with an explicit damping diagonal D (held constant): the
    backward pass solves with the same H = J^T J + D, and its gradient matches
    central differences of the loss with D fixed."""
    import paper_2007_01941_amd as bamg
    sc = scene("ring20")
    plan, opts = plan_for(sc, precond="mg", rtol=1e-13, max_iter=5000, coarse_max_nodes=4)
    nrm0 = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv)
    rng = np.random.default_rng(17)
    D = dev(np.concatenate([nrm0.Dc.ravel(), nrm0.Dp.ravel()]) * rng.uniform(0.5, 5.0, 9 * sc.n_cam + 3 * sc.n_pt))
    cams, pts, uv = inputs(sc)
    for t in (cams, pts, uv):
        t.requires_grad_(True)
    dc, dp = bamg.LMStep.apply(cams, pts, uv, plan, opts, D)
    ((dc * dc).sum() + (dp * dp).sum()).backward()

    def loss(c, p, u):
        a, b, _ = plan.lm_step(c, p, u, D=D)
        return float((a * a).sum() + (b * b).sum())

    h = 1e-4
    for _ in range(4):
        vc, vp, vu = (torch.as_tensor(rng.normal(size=t.shape), device="cuda") for t in (cams, pts, uv))
        s = float(torch.sqrt((vc ** 2).sum() + (vp ** 2).sum() + (vu ** 2).sum()))
        vc, vp, vu = vc / s, vp / s, vu / s
        with torch.no_grad():
            fd = (loss(cams + h * vc, pts + h * vp, uv + h * vu) - loss(cams - h * vc, pts - h * vp, uv - h * vu)) / (2 * h)
        an = float((cams.grad * vc).sum() + (pts.grad * vp).sum() + (uv.grad * vu).sum())
        print(f"[gpu] explicit D: fd {fd:.8e} adjoint {an:.8e}", flush=True)
        assert abs(fd - an) <= 2e-5 * abs(an) + 1e-6
