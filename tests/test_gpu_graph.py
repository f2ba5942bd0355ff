"""The PCG iteration replayed from a captured HIP graph gives the same steps as
the same launches made one by one: bitwise, in deterministic mode, for every
preconditioner and precision, over several steps on one plan with eager work
(and host waits) between the replays, and after the workspace moves."""
import numpy as np
import pytest
import torch

from tests._fixtures import scene
from tests._gpu import host, inputs, plan_for

pytestmark = pytest.mark.gpu

CASES = [("mg", "fp64"), ("mg", "mixed"), ("bj", "fp64"), ("bj", "mixed"), ("cj", "fp64")]


@pytest.mark.parametrize("pc,prec", CASES)
def test_graph_replays_match_eager_launches(pc, prec):
    import paper_2007_01941_amd as bamg
    sc = scene("city200")
    plan, opts = plan_for(sc, precond=pc, precision=prec, rtol=1e-10, coarse_max_nodes=16, deterministic=True,
                          graph=True)
    eager = bamg.Options(precond=pc, precision=prec, rtol=1e-10, coarse_max_nodes=16, deterministic=True,
                         graph=False)
    cams, pts, uv = inputs(sc)
    rng = np.random.default_rng(3)
    for k in range(3):
        # a different linearization point per step, shared by both forms
        c = cams + torch.as_tensor(1e-4 * rng.normal(size=tuple(cams.shape)), device=cams.device)
        g_dc, g_dp, g_st = plan.lm_step(c, pts, uv, opts=opts)
        torch.cuda.synchronize()
        e_dc, e_dp, e_st = plan.lm_step(c, pts, uv, opts=eager)
        print(f"[gpu] {pc} {prec} step {k}: iters graph {g_st.iters} eager {e_st.iters}", flush=True)
        assert g_st.converged and e_st.converged
        assert g_st.iters == e_st.iters
        assert torch.equal(g_dc, e_dc) and torch.equal(g_dp, e_dp)


def test_graph_follows_a_moved_workspace():
    """A step in a caller workspace, then in the plan's own, then in another
    caller workspace: each replays its own capture, all bitwise equal."""
    import ctypes
    import paper_2007_01941_amd as bamg
    from paper_2007_01941_amd import _lib
    sc = scene("ring64")
    plan, opts = plan_for(sc, precond="mg", rtol=1e-10, coarse_max_nodes=16, deterministic=True, graph=True)
    cams, pts, uv = inputs(sc)
    ref_dc, ref_dp, _ = plan.lm_step(cams, pts, uv, opts=opts)
    o = opts.to_c()
    need = int(_lib.LIB.ba_workspace_bytes(plan._h, ctypes.byref(o), _lib.USE_STEP))
    for trial in range(2):
        ws = torch.empty(need + 4096 * trial, dtype=torch.uint8, device="cuda")
        dc = torch.empty_like(ref_dc)
        dp = torch.empty_like(ref_dp)
        st = _lib.LIB.ba_lm_step(plan._h, ctypes.byref(o), ctypes.c_void_p(cams.data_ptr()),
                                 ctypes.c_void_p(pts.data_ptr()), ctypes.c_void_p(uv.data_ptr()), None,
                                 ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                 ctypes.c_void_p(dc.data_ptr()), ctypes.c_void_p(dp.data_ptr()), None,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0, _lib.LIB.ba_last_error()
        torch.cuda.synchronize()
        assert torch.equal(dc, ref_dc) and torch.equal(dp, ref_dp)
        del ws
        again_dc, again_dp, _ = plan.lm_step(cams, pts, uv, opts=opts)
        assert torch.equal(again_dc, ref_dc) and torch.equal(again_dp, ref_dp)


def test_graph_lm_loop_matches_eager():
    """Whole LM runs (prepare and solve per iteration, accept and reject) with
    and without the graph: identical histories in deterministic mode."""
    import paper_2007_01941_amd as bamg
    sc = scene("ring64")
    plan, opts = plan_for(sc, precond="mg", rtol=1e-10, coarse_max_nodes=16, deterministic=True,
                          stop_rule="nash_sofer", forcing=0.1, graph=True)
    eager = bamg.Options(precond="mg", rtol=1e-10, coarse_max_nodes=16, deterministic=True, stop_rule="nash_sofer",
                         forcing=0.1, graph=False)
    outs = []
    for o in (opts, eager, opts):
        cams, pts, uv = inputs(sc)
        outs.append(plan.lm_solve(cams, pts, uv, opts=o, lm_opts=bamg.LMOptions(max_iters=8)))
    for out in outs[1:]:
        assert out.iters == outs[0].iters and out.pcg_iters == outs[0].pcg_iters
        assert [h.cost_candidate for h in out.history] == [h.cost_candidate for h in outs[0].history]
        assert out.cost == outs[0].cost
