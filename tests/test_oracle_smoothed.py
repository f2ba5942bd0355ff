"""Pins of the oracle's smoothed-aggregation variant (the alternative Section
3.5 weighs against the unsmoothed prolongator the paper uses)."""
import numpy as np

from oracle import aggregation as agglib, multigrid as mg, step as ostep
from oracle.nullspace import camera_nullspace
from tests._fixtures import scene


def test_smoothing_keeps_the_gauge_modes():
    """At D = 0 the seven gauge modes are in S's nullspace, so the smoothing
    sweep leaves them alone: P_s K_c = K on those columns (and P_tent K_c = K
    on all 16)."""
    sc = scene("city200")
    nrm = ostep.normal_for(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, lam=0.0)
    S = nrm.S_sparse()
    K = camera_nullspace(sc.cams)                      # [n_cam, 9, 16]
    W = agglib.covisibility(sc.obs_cam, sc.obs_pt, sc.n_cam, sc.n_pt)
    agg, n_agg = agglib.aggregate(W, 20)
    Pb, Kc, P = mg.tentative_prolongator(K, agg, n_agg)
    Kf = K.reshape(-1, 16)
    Kcm = Kc.reshape(-1, 16)
    assert np.allclose(P @ Kcm, Kf, atol=1e-10 * np.abs(Kf).max())
    Dinv = np.linalg.inv(mg.block_diagonal(S, 9))
    lmax = mg.lanczos_lmax(lambda x: S @ x, Dinv, mg.lanczos_start(S.shape[0], 0), 5)
    Ps = mg.smoothed_prolongator(S, 9, P, lmax)
    gauge = slice(9, 16)
    err = np.abs(Ps @ Kcm[:, gauge] - Kf[:, gauge]).max()
    assert err <= 1e-6 * np.abs(Kf[:, gauge]).max()
    # the constant columns are not in S's nullspace: smoothing changes them
    assert np.abs(Ps @ Kcm[:, :9] - Kf[:, :9]).max() > 1e-3 * np.abs(Kf[:, :9]).max()


def test_smoothing_trades_fill_in_for_iterations():
    """The paper's observation on street scenes: a smoothed prolongator cuts
    the PCG iterations but fills in the coarse operators (here the first coarse
    operator holds more entries than the fine one)."""
    sc = scene("city200")
    runs = {}
    for smooth in (False, True):
        o = mg.MGOptions(coarse_max_nodes=16, smooth_prolongator=smooth)
        runs[smooth] = ostep.lm_step(sc.cams, sc.pts, sc.obs_cam, sc.obs_pt, sc.uv, method="mg", rtol=1e-8, opts=o)
    plain, smooth = runs[False], runs[True]
    assert [l.S.shape for l in plain.levels] == [l.S.shape for l in smooth.levels]
    print(f"iterations {plain.iters} -> {smooth.iters}; level-1 entries {plain.levels[1].S.nnz} -> "
          f"{smooth.levels[1].S.nnz} (level 0: {plain.levels[0].S.nnz})")
    assert smooth.converged and smooth.iters < plain.iters
    assert smooth.levels[1].S.nnz > 2 * plain.levels[1].S.nnz
    assert smooth.levels[1].S.nnz > plain.levels[0].S.nnz
