"""ba_cost_noalloc, the entry point for callers that cannot allocate: its
kernels' scratch is a static device array, so a call allocates nothing. Its
cost and invalid count must equal ba_cost's on the same inputs (the same
kernels and the same ordered reductions), on two calls in a row, the second
on a smaller plan, with no change to the plans' or torch's device memory.
(Named to be collected last: it must pass alone and after every other test.)"""
import ctypes

import numpy as np
import pytest
import torch

from scenes import tiny_scene
from tests._fixtures import scene
from tests._gpu import inputs, plan_for

pytestmark = pytest.mark.gpu


def _noalloc_cost(plan, opts, cams, pts, uv):
    from paper_2007_01941_amd import _lib
    fn = _lib.LIB.ba_cost_noalloc
    c = ctypes.c_double()
    bad = ctypes.c_int64()
    o = opts.to_c()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = fn(plan._h, ctypes.byref(o), ctypes.c_void_p(cams.data_ptr()), ctypes.c_void_p(pts.data_ptr()),
            ctypes.c_void_p(uv.data_ptr()), ctypes.byref(c), ctypes.byref(bad), s)
    return st, c.value, bad.value


def test_noalloc_cost_matches_ba_cost():
    from paper_2007_01941_amd import _lib
    big = scene("city200")
    small = tiny_scene(12, 200, seed=3, k_min=2, k_max=6)
    # the first call on the larger plan, the second on the smaller one
    for sc, loss in ((big, "huber"), (small, "squared")):
        plan, opts = plan_for(sc, precond="bj", loss=loss, loss_scale=2.0)
        cams, pts, uv = inputs(sc)
        # move point 0 just behind one of its cameras (x_cam.z > 0), so that the
        # invalid count is exercised: X = C + 1e-3 R^T e_z with C = -R^T t
        from oracle.camera import rotation_matrix
        c0 = int(sc.obs_cam[np.nonzero(sc.obs_pt == 0)[0][0]])
        R = rotation_matrix(sc.cams[c0:c0 + 1, 0:3])[0]
        X = -R.T @ sc.cams[c0, 3:6] + 1e-3 * R[2]
        pts_bad = pts.clone()
        pts_bad[0] = torch.as_tensor(X, device=pts.device)
        for P_ in (pts, pts_bad):
            ref_cost, ref_bad = plan.cost(cams, P_, uv, opts=opts)
            torch.cuda.synchronize()
            before_plan = int(_lib.LIB.ba_plan_bytes(plan._h))
            before_torch = torch.cuda.memory_allocated()
            st, c, bad = _noalloc_cost(plan, opts, cams, P_, uv)
            torch.cuda.synchronize()
            print(f"[gpu] {sc.name} {loss}: noalloc {c!r} ({bad} invalid), ba_cost {ref_cost!r} ({ref_bad})",
                  flush=True)
            assert st == 0
            assert c == ref_cost and bad == ref_bad
            if P_ is pts_bad:
                assert bad >= 1
            assert int(_lib.LIB.ba_plan_bytes(plan._h)) == before_plan
            assert torch.cuda.memory_allocated() == before_torch


def test_noalloc_rejects_null_arguments():
    from paper_2007_01941_amd import _lib
    sc = tiny_scene(12, 200, seed=3, k_min=2, k_max=6)
    plan, opts = plan_for(sc, precond="bj")
    cams, pts, uv = inputs(sc)
    fn = _lib.LIB.ba_cost_noalloc
    c = ctypes.c_double()
    assert fn(plan._h, None, ctypes.c_void_p(cams.data_ptr()), None, ctypes.c_void_p(uv.data_ptr()),
              ctypes.byref(c), None, None) == -1
