"""Error paths of the C ABI, forced from the host (no kernel faults)."""
import numpy as np
import pytest
import torch

from scenes import tiny_scene
from tests._gpu import dev, inputs

pytestmark = pytest.mark.gpu


def _plan(sc, oc=None, op=None, **kw):
    import paper_2007_01941_amd as bamg
    return bamg.Plan(sc.n_cam, sc.n_pt, dev(sc.obs_cam if oc is None else oc, torch.int32),
                     dev(sc.obs_pt if op is None else op, torch.int32), bamg.Options(**kw))


def test_index_out_of_range():
    import paper_2007_01941_amd as bamg
    sc = tiny_scene(6, 30, seed=2)
    oc = sc.obs_cam.copy()
    oc[3] = sc.n_cam
    with pytest.raises(bamg.BAError) as e:
        _plan(sc, oc=oc)
    assert e.value.name == "BA_ERR_INDEX"


def test_point_with_one_view_and_duplicates():
    import paper_2007_01941_amd as bamg
    sc = tiny_scene(6, 30, seed=2, k_min=3)
    op = sc.obs_pt.copy()
    first = np.nonzero(op == 0)[0]
    op[first[1:]] = 1            # point 0 keeps one view
    with pytest.raises(bamg.BAError) as e:
        _plan(sc, op=op)
    assert e.value.name == "BA_ERR_STRUCTURE"
    oc = sc.obs_cam.copy()
    i = np.nonzero(sc.obs_pt == 2)[0]
    oc[i[1]] = oc[i[0]]           # camera sees point 2 twice
    with pytest.raises(bamg.BAError) as e:
        _plan(sc, oc=oc)
    assert e.value.name == "BA_ERR_STRUCTURE"


def test_point_behind_camera_and_nonfinite():
    import paper_2007_01941_amd as bamg
    sc = tiny_scene(6, 30, seed=2)
    plan = _plan(sc, precond="bj")
    pts = sc.pts.copy()
    c = sc.obs_cam[0]
    # put point obs_pt[0] behind its camera: mirror it through the camera centre
    from oracle.camera import rotation_matrix
    R = rotation_matrix(sc.cams[c:c + 1, 0:3])[0]
    center = -R.T @ sc.cams[c, 3:6]
    pts[sc.obs_pt[0]] = 2 * center - pts[sc.obs_pt[0]]
    with pytest.raises(bamg.BAError) as e:
        plan.lm_step(*inputs(sc, pts=pts))
    assert e.value.name == "BA_ERR_GEOMETRY"
    uv = sc.uv.copy()
    uv[5, 0] = np.nan
    with pytest.raises(bamg.BAError) as e:
        plan.lm_step(*inputs(sc, uv=uv))
    assert e.value.name == "BA_ERR_GEOMETRY"
    # the plan stays usable after an error
    dc, dp, st = plan.lm_step(*inputs(sc))
    assert st.converged


def test_not_converged_returns_last_iterate():
    import warnings

    import paper_2007_01941_amd as bamg
    sc = tiny_scene(10, 80, seed=4)
    plan = _plan(sc, precond="bj", max_iter=1, rtol=1e-12, check_every=1)
    with warnings.catch_warnings(record=True) as w:
        warnings.simplefilter("always")
        dc, dp, st = plan.lm_step(*inputs(sc))
    assert not st.converged and st.iters == 1
    assert any(issubclass(x.category, bamg.NotConverged) for x in w)
    assert torch.isfinite(dc).all() and torch.isfinite(dp).all()


def test_bad_shapes_rejected_before_the_library():
    sc = tiny_scene(6, 30, seed=2)
    plan = _plan(sc)
    c, p, u = inputs(sc)
    with pytest.raises(ValueError):
        plan.lm_step(c[:-1], p, u)
    with pytest.raises(TypeError):
        plan.lm_step(c.float(), p, u)
