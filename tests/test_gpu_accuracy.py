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
