"""The memory contract of the C ABI: the plan's persistent arrays come from the
caller's allocation callbacks (here torch tensors), each step runs in a
caller-owned workspace of ba_workspace_bytes() bytes, a short workspace is
BA_ERR_WORKSPACE, and without a workspace the plan keeps its own (allocated
through the same callbacks). All through the C ABI on ring64."""
import ctypes

import numpy as np
import pytest
import torch

from tests._fixtures import scene
from tests._gpu import host, inputs, plan_for

pytestmark = pytest.mark.gpu


def _raw_step(plan, o, cams, pts, uv, ws, ws_bytes):
    from paper_2007_01941_amd import _lib
    dc = torch.empty((plan.n_cam, 9), dtype=torch.float64, device="cuda")
    dp = torch.empty((plan.n_pt, 3), dtype=torch.float64, device="cuda")
    st = _lib._Stats()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    status = _lib.LIB.ba_lm_step(plan._h, ctypes.byref(o), ctypes.c_void_p(cams.data_ptr()),
                                 ctypes.c_void_p(pts.data_ptr()), ctypes.c_void_p(uv.data_ptr()), None, ws,
                                 ctypes.c_size_t(ws_bytes), ctypes.c_void_p(dc.data_ptr()),
                                 ctypes.c_void_p(dp.data_ptr()), ctypes.byref(st), s)
    return status, dc, dp


def test_torch_owned_memory_and_workspace():
    from paper_2007_01941_amd import _lib
    sc = scene("ring64")
    plan, opts = plan_for(sc, precond="mg", rtol=1e-10, coarse_max_nodes=16, deterministic=True)
    persistent = plan._mem.bytes
    # every persistent array of the plan came through the callbacks
    assert persistent > 0 and int(_lib.LIB.ba_plan_bytes(plan._h)) == persistent
    cams, pts, uv = inputs(sc)
    dc, dp, st = plan.lm_step(cams, pts, uv)
    assert st.converged
    # the step ran in the torch workspace: no memory of the plan's own was added
    assert int(_lib.LIB.ba_plan_bytes(plan._h)) == persistent == plan._mem.bytes
    o = opts.to_c()
    need = plan.workspace_bytes(opts)
    assert plan._ws.numel() >= need
    # a workspace one byte short is refused, nothing written
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    status, _, _ = _raw_step(plan, o, cams, pts, uv, ctypes.c_void_p(ws.data_ptr()), need - 1)
    assert status == _lib.BA_ERR_WORKSPACE and b"need" in _lib.LIB.ba_last_error()
    # a workspace not aligned to 256 bytes is refused
    status, _, _ = _raw_step(plan, o, cams, pts, uv, ctypes.c_void_p(ws.data_ptr() + 8), need - 8)
    assert status == -1 and b"aligned" in _lib.LIB.ba_last_error()
    # another workspace of exactly the size needed: the same step, bitwise
    status, dc2, dp2 = _raw_step(plan, o, cams, pts, uv, ctypes.c_void_p(ws.data_ptr()), need)
    assert status == 0
    assert np.array_equal(host(dc2), host(dc)) and np.array_equal(host(dp2), host(dp))
    # no workspace: the plan allocates its own through the callbacks
    status, dc3, dp3 = _raw_step(plan, o, cams, pts, uv, None, 0)
    assert status == 0
    assert np.array_equal(host(dc3), host(dc)) and np.array_equal(host(dp3), host(dp))
    own = int(_lib.LIB.ba_plan_bytes(plan._h)) - persistent
    assert own >= need and plan._mem.bytes == persistent + own


def test_workspace_sizes_follow_the_options():
    import paper_2007_01941_amd as bamg
    from paper_2007_01941_amd import _lib
    sc = scene("ring64")
    plan, _ = plan_for(sc, precond="mg", coarse_max_nodes=16)
    bj = plan.workspace_bytes(bamg.Options(precond="bj"))
    mg = plan.workspace_bytes(bamg.Options(precond="mg", coarse_max_nodes=16))
    mixed = plan.workspace_bytes(bamg.Options(precond="mg", precision="mixed", coarse_max_nodes=16))
    back = plan.workspace_bytes(bamg.Options(precond="mg", coarse_max_nodes=16), _lib.USE_BACKWARD)
    lm = plan.workspace_bytes(bamg.Options(precond="mg", coarse_max_nodes=16), _lib.USE_LM)
    assert bj < mg < mixed and mg < back and mg < lm
    # the per-observation Jacobian planes alone: F, E, f (26 doubles per observation)
    assert bj >= 26 * 8 * sc.n_obs
