"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`plan_check_sanitized` (built by `build()`: the whole library plus a driver of
every host-side path -- plan creation and its error paths, workspace binding,
steps with every preconditioner and precision, the adjoint, the cost, the LM
loop, hierarchy inspection -- with instrumented host code and the usual GPU
code) runs on seeded scenes whose observations are shuffled, one process per
scene, and must finish without a sanitizer report."""
import os
import struct
import subprocess

import numpy as np
import pytest

from scenes import tiny_scene
from tests._fixtures import scene

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2007_01941_amd", "plan_check_sanitized")


def _write(path, sc, seed):
    perm = np.random.default_rng(seed).permutation(sc.n_obs)
    with open(path, "wb") as f:
        f.write(struct.pack("<iiq", sc.n_cam, sc.n_pt, sc.n_obs))
        f.write(np.ascontiguousarray(sc.obs_cam[perm], dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(sc.obs_pt[perm], dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(sc.cams, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(sc.pts, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(sc.uv[perm], dtype=np.float64).tobytes())


@pytest.mark.parametrize("name", ["tiny", "ring64", "city200"])
def test_host_code_is_clean_under_sanitizers(tmp_path, name):
    assert os.path.exists(EXE), f"{EXE} is not built; run __graft_entry__.build()"
    sc = tiny_scene(40, 600, seed=7, k_min=2, k_max=9) if name == "tiny" else scene(name)
    path = tmp_path / "scene.bin"
    _write(path, sc, seed=11)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    print(f"[gpu] sanitized host checker on {name} ({sc.n_cam} cameras, {sc.n_obs} observations)", flush=True)
    p = subprocess.run([EXE, str(path)], capture_output=True, text=True, timeout=240, env=env)
    print(p.stdout[-2500:], flush=True)
    print(p.stderr[-4000:], flush=True)
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr
    assert p.returncode == 0
    assert "[check] OK" in p.stdout
