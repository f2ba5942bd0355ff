"""The step-accuracy protocol on the ring scene (64 cameras, 4,000 points,
32,000 observations): the error triple |d - d*| / |d*|, |d - d*|_S / |d*|_S
and |b - S d| / |b| against the oracle's dense solve d*, with cond(S) from the
oracle's eigenvalues (about 1e10 here: the gauge directions are held only by
the damping), at a loose and at a tight tolerance."""
import numpy as np
import pytest

from oracle import step as ostep
from tests._fixtures import scene
from tests._gpu import host, inputs, plan_for
from tests.test_gpu_step import TOL_U, rhs_abs, schur_abs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring():
    sc = scene("ring64")
    ref = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="schur")
    ev = np.linalg.eigvalsh(ref.normal.S_dense())
    return sc, ref, float(ev[-1] / ev[0])


@pytest.mark.parametrize("pc", ["mg", "bj"])
@pytest.mark.parametrize("rtol", [1e-8, 1e-12])
def test_error_triple(ring, pc, rtol):
    sc, ref, kappa = ring
    kw = dict(coarse_max_nodes=16) if pc == "mg" else {}
    plan, _ = plan_for(sc, precond=pc, rtol=rtol, max_iter=20000, **kw)
    dc, _, st = plan.lm_step(*inputs(sc))
    dc = host(dc)
    nrm, b = ref.normal, ref.b
    e_rel, e_S, res = ostep.error_triple(dc, ref.delta_c, nrm, b)
    # rounding of the oracle's own product and right-hand side
    slack = TOL_U * np.linalg.norm(schur_abs(nrm, dc) + rhs_abs(nrm)) / np.linalg.norm(b)
    print(f"[gpu] ring64 {pc} rtol {rtol:.0e}: iters {st.iters} "
          f"cond(S) {kappa:.2e}  |d-d*|/|d*| {e_rel:.2e}  |d-d*|_S/|d*|_S {e_S:.2e}  "
          f"|b-Sd|/|b| {res:.2e}", flush=True)
    assert st.converged
    assert res <= 2 * rtol + slack
    # for SPD S the relative error is at most cond(S) times the relative residual,
    # and the S-norm error at most sqrt(cond(S)) times it
    assert e_rel <= kappa * (res + slack) * 1.01
    assert e_S <= np.sqrt(kappa) * (res + slack) * 1.01
    if rtol <= 1e-12:
        # at a tight tolerance the step itself agrees with the dense solve to 1e-8
        assert e_rel <= 1e-8


@pytest.mark.parametrize("pc", ["mg", "bj"])
def test_error_triple_mixed_refined(ring, pc):
    """The precision form (FP32 Schur product and preconditioner inside FP64
    iterative refinement) at a tight outer tolerance: refinement drives the
    FP64 residual, so the step reaches the dense solve as the FP64 path does:
    within 1e-6 relative, with the same conditioning bounds."""
    sc, ref, kappa = ring
    kw = dict(coarse_max_nodes=16) if pc == "mg" else {}
    rtol = 1e-12
    plan, _ = plan_for(sc, precond=pc, precision="mixed", rtol=rtol, max_iter=20000, max_refine=40, **kw)
    dc, _, st = plan.lm_step(*inputs(sc))
    dc = host(dc)
    nrm, b = ref.normal, ref.b
    e_rel, e_S, res = ostep.error_triple(dc, ref.delta_c, nrm, b)
    slack = TOL_U * np.linalg.norm(schur_abs(nrm, dc) + rhs_abs(nrm)) / np.linalg.norm(b)
    print(f"[gpu] ring64 mixed {pc} rtol {rtol:.0e}: refine {st.refine_steps} inner iters {st.iters} "
          f"|d-d*|/|d*| {e_rel:.2e}  |d-d*|_S/|d*|_S {e_S:.2e}  |b-Sd|/|b| {res:.2e}", flush=True)
    assert st.converged and st.refine_steps >= 2
    assert res <= 2 * rtol + slack
    assert e_rel <= kappa * (res + slack) * 1.01
    assert e_rel <= 1e-6


@pytest.mark.parametrize("pc", ["mg", "bj"])
def test_error_single_fp32_solve(ring, pc):
    """One FP32 inner solve and no refinement: the step carries the FP32
    operator's rounding. Its FP64 residual is bounded by the inner tolerance
    plus the FP32 product's relative error (|S32 - S| x against b, measured
    by the oracle's |S| |x| bound with u = 2^-24), and the S-norm error of a
    residual that small stays within sqrt(cond) of it in the S-norm; with the
    multigrid preconditioner (error spread over the spectrum, not left in the
    smooth modes) the S-norm error is within 1e-5."""
    sc, ref, kappa = ring
    kw = dict(coarse_max_nodes=16) if pc == "mg" else {}
    inner = 1e-6
    plan, _ = plan_for(sc, precond=pc, precision="mixed", rtol=inner, inner_rtol=inner, max_refine=1,
                       max_iter=20000, **kw)
    dc, _, st = plan.lm_step(*inputs(sc))
    dc = host(dc)
    nrm, b = ref.normal, ref.b
    e_rel, e_S, res = ostep.error_triple(dc, ref.delta_c, nrm, b)
    u32 = 2.0 ** -24
    fp32_floor = 8 * u32 * np.linalg.norm(schur_abs(nrm, dc) + rhs_abs(nrm)) / np.linalg.norm(b)
    print(f"[gpu] ring64 single FP32 solve {pc}: inner iters {st.iters} |d-d*|/|d*| {e_rel:.2e}  "
          f"|d-d*|_S/|d*|_S {e_S:.2e}  |b-Sd|/|b| {res:.2e}  (FP32 floor {fp32_floor:.1e}, "
          f"cond {kappa:.1e})", flush=True)
    assert st.refine_steps == 1
    assert res <= inner + fp32_floor
    assert e_S <= np.sqrt(kappa) * res * 1.01
    if pc == "mg":
        assert e_S <= 1e-5
