"""bench.py without a GPU: more than one GPU is refused before anything
touches a device, with a JSON message; the committed counter summaries it
reads belong to the current kernels."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_traffic_summaries_match_the_current_kernels():
    """The committed counter summaries were taken on the tile kernels as they
    are now (their source hash matches), so the bench line reports measured
    traffic; and their algorithmic bytes follow the survey's formula for the
    tile kernel, n_o (24 s + 4) + n_p (6 s + 4) + 27 s n_c."""
    sys.path.insert(0, ROOT)
    import bench
    sizes = {"city2k": (3475014, 600000, 2000), "path10k": (24997392, 4000000, 10000),
             "city30k": (78397954, 12000000, 30000)}
    for scene, (n_o, n_p, n_c) in sizes.items():
        vals = {}
        for line in open(os.path.join(ROOT, "profiles", f"k_schur_groups_{scene}_traffic.txt")):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
        for prec, s in (("fp64", 8), ("fp32", 4)):
            traffic = bench.read_traffic(scene, prec)
            assert traffic is not None and traffic > 0, (scene, prec)
            alg = n_o * (24 * s + 4) + n_p * (6 * s + 4) + 27 * s * n_c
            assert bench.kernel_bytes(n_o, n_p, n_c, s) == alg
            assert int(vals[f"algorithmic_bytes_per_launch_{prec}"]) == alg
        # the FP64 kernel recomputes F and E: it moves a fraction of B_k
        assert bench.read_traffic(scene, "fp64") < 0.3 * (n_o * 196 + n_p * 52 + 216 * n_c)
    assert bench.kernel_flops_rc(10, 3) == 10 * 242 + 3 * 15
