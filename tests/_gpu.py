"""Helpers of the GPU tests: moving seeded scenes to the device and building plans."""
import numpy as np
import torch

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def plan_for(sc, **opt_kw):
    import paper_2007_01941_amd as bamg
    opts = bamg.Options(**opt_kw)
    print(f"[gpu] plan {sc.name}: n_cam={sc.n_cam} n_pt={sc.n_pt} n_obs={sc.n_obs} opts={opt_kw}",
          flush=True)
    return bamg.Plan(sc.n_cam, sc.n_pt, dev(sc.obs_cam, torch.int32), dev(sc.obs_pt, torch.int32),
                     opts), opts


def inputs(sc, cams=None, pts=None, uv=None):
    return (dev(sc.cams if cams is None else cams), dev(sc.pts if pts is None else pts),
            dev(sc.uv if uv is None else uv))


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
