"""Benchmark: one Levenberg-Marquardt linear solve of multigrid bundle adjustment
on one MI355X.

A step is one pass of the whole hot path on a fixed synthetic street-view
scene (city grid, 2,000 cameras, 600,000 points, ~3.48M observations):
residual and Jacobian, normal blocks, multigrid setup (near-nullspace QR,
explicit level-0 Schur complement, Galerkin products, Lanczos, coarse
factorization), PCG on the implicitly applied Schur complement to rtol 1e-6,
and back-substitution. Inputs are resident in HBM before timing starts; the
integer plan (layout, covisibility, aggregation) is built once beforehand, as
in an LM loop over a fixed visibility graph, and timed separately.

Besides the headline workload the default run measures two more scenes, each
in its own entry of "legs": the long path without loop closures (10,000
cameras, ~25M observations), where the precision form (FP32 product and
V-cycle inside FP64 refinement) is compared with the FP64 path, and the
largest single-GPU scene (30,000 cameras, ~78M observations), measured in
the precision form with the adjoint solve.

Prints ONE JSON line (the driver's contract); see the design doc for the fields.
"""
import argparse
import hashlib
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RCS solve s to rtol 1e-6 (MG vs block-Jacobi, FP32 vs FP64); matvec GB/s"
HBM_PEAK_GBPS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")
WORKLOADS = {
    "city2k": "city-grid street-view scene",
    "path10k": "5 km street path without loop closures",
    "city30k": "4x4 km city grid with loop closures, heavy-tailed track lengths",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def schur_bytes(n_obs, n_pt, n_cam, s):
    """Algorithmic bytes of one implicit Schur product y = A x - F^T E C^-1 E^T F x:
    F_o, E_o (24 s) + a 4-byte index per observation; C_p^-1 (6 s) + a 4-byte
    offset per point; x, A (45 packed), y per camera (63 s)."""
    return n_obs * (24 * s + 4) + n_pt * (6 * s + 4) + n_cam * 63 * s


def kernel_bytes(n_obs, n_pt, n_cam, s):
    """Algorithmic bytes of the tile kernel alone (y -= W C^-1 W^T x): F_o, E_o
    and a 4-byte index per observation; C_p^-1 and a 4-byte offset per point;
    x read, y read and written per camera (27 s)."""
    return n_obs * (24 * s + 4) + n_pt * (6 * s + 4) + n_cam * 27 * s


FP64_VECTOR_PEAK_TFLOPS = 78.6


def kernel_flops_rc(n_obs, n_pt):
    """FP64 operations of one launch of the FP64 tile kernel, which recomputes
    F_o and E_o: per observation the projection and its Jacobian blocks (148:
    camera transform 18, 1/z, projection and distortion 12, d pi / d x_cam 27,
    E_o 30, F_o's rotation columns 48, its intrinsic columns 12) and the
    product (94: F x 36, E^T s 9, the point sum 3, E u 10, F^T w 27, the camera
    sum 9); per point C_p^-1 z (15)."""
    return n_obs * (148 + 94) + n_pt * 15


def kernel_source_hash():
    """Hash of the sources the tile kernels are built from: their file, the
    layout constants, the plan code that groups the tiles, and the projection
    (in step_kernels.hip) that the FP64 kernel recomputes."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2007_01941_amd", "csrc")
    for f in ("schur_kernels.hip", "common.hpp", "layout.cpp"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    step = open(os.path.join(csrc, "step_kernels.hip"), "rb").read()
    i = step.index(b"__device__ __forceinline__ void project_jacobian(")
    h.update(step[i:step.index(b"\n}\n", i) + 3])
    return h.hexdigest()[:16]


def read_traffic(scene, prec):
    """HBM bytes per launch of the tile kernel of `prec` on `scene` from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a copy
    kernel), if it was taken on the current kernel source; else None."""
    path = os.path.join(PROFILE_DIR, f"k_schur_groups_{scene}_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_hash():
        return None
    try:
        return float(vals[f"traffic_bytes_per_launch_{prec}"])
    except (KeyError, ValueError):
        return None


def to_device(sc, torch, dev):
    T = lambda a, dt=torch.float64: torch.as_tensor(__import__("numpy").ascontiguousarray(a), dtype=dt, device=dev)
    return T(sc.cams), T(sc.pts), T(sc.uv), T(sc.obs_cam, torch.int32), T(sc.obs_pt, torch.int32)


def time_steps(plan, cams, pts, uv, opts, steps, warmup):
    """Whole LM steps, timed with HIP events around `steps` back-to-back calls.
    Returns (ms per step, wall s, stats of the last step, dc, dp)."""
    import torch
    for _ in range(warmup):
        plan.lm_step(cams, pts, uv, opts=opts)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.time()
    ev0.record()
    for _ in range(steps):
        dc, dp, st = plan.lm_step(cams, pts, uv, opts=opts)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps, time.time() - t_wall, st, dc, dp


def time_launches(fn, reps):
    """Seconds per call of fn (device work enqueued on the current stream)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps / 1e3


def measure_products(bamg, plan, sc, cams, pts, uv, base, reps=50):
    """The implicit Schur product (A x included) per precision, and the tile
    kernel alone (k_schur_groups: y -= W C^-1 W^T x, one launch per call) with
    its roofline per precision."""
    import torch
    x = torch.randn(sc.n_cam, 9, dtype=torch.float64, device="cuda:0")
    y = torch.zeros_like(x)
    mat, roof = {}, {}
    for prec, s, mode in (("fp64", 8, "fp64"), ("fp32", 4, "mixed")):
        plan.prepare(cams, pts, uv, opts=bamg.Options(precond="bj", precision=mode, **base))
        t = time_launches(lambda: plan.schur_apply(x, mode), reps)
        B = schur_bytes(sc.n_obs, sc.n_pt, sc.n_cam, s)
        mat[prec] = {"s_per_apply": t, "algorithmic_bytes": B, "GBps": B / t / 1e9}
        tk = time_launches(lambda: plan.schur_offdiag_apply(x, y, mode), reps)
        Bk = kernel_bytes(sc.n_obs, sc.n_pt, sc.n_cam, s)
        a = Bk / tk / 1e9
        if prec == "fp64":
            # F_o and E_o are recomputed, not read: the GB/s are the method's bytes B over the
            # time (what a kernel streaming the stored blocks would have to reach), `traffic` the
            # bytes the counters see move, and `alu` the FP64 arithmetic against the vector peak
            fl = kernel_flops_rc(sc.n_obs, sc.n_pt)
            roof[prec] = {"kernel": "k_schur_groups_rc<double>: y -= W C^-1 W^T x, F_o and E_o recomputed "
                                    "(implicit Schur product)",
                          "bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                          "frac": a / HBM_PEAK_GBPS, "traffic": read_traffic(sc.name, prec),
                          "algorithmic_bytes": Bk, "s_per_launch": tk,
                          "alu": {"achieved": fl / tk / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": fl / tk / 1e12 / FP64_VECTOR_PEAK_TFLOPS, "flops": fl}}
        else:
            roof[prec] = {"kernel": "k_schur_groups<float>: y -= W C^-1 W^T x (implicit Schur product)",
                          "bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                          "frac": a / HBM_PEAK_GBPS, "traffic": read_traffic(sc.name, prec),
                          "algorithmic_bytes": Bk, "s_per_launch": tk}
        log(f"[bench] {sc.name} Schur product {prec}: {t * 1e6:.1f} us/apply ({B / t / 1e9:.0f} GB/s); "
            f"tile kernel {tk * 1e6:.1f} us/launch, {a:.0f} GB/s = {a / HBM_PEAK_GBPS:.3f} of peak"
            + (f", {roof[prec]['alu']['achieved']:.1f} TFLOP/s FP64" if prec == "fp64" else ""))
    return mat, roof


def step_entry(ms, st, dc=None, ref=None):
    import torch
    e = {"s_per_step": ms / 1e3, "pcg_iters": st.iters, "refine_steps": st.refine_steps,
         "fp64_fallback": st.fallback_fp64, "rel_res": st.rel_res,
         "phases_ms": {"jacobian_and_blocks": st.t_jacobian_ms, "setup": st.t_setup_ms, "solve": st.t_solve_ms}}
    if dc is not None and ref is not None:
        e["rel_diff_vs_mg_fp64"] = float(torch.linalg.norm(dc - ref) / torch.linalg.norm(ref))
    return e


def true_residual(plan, bamg, cams, pts, uv, dc, base):
    """|b - S dc| / |b| with the FP64 product of a freshly prepared FP64 step."""
    import torch
    plan.prepare(cams, pts, uv, opts=bamg.Options(precond="bj", precision="fp64", **base))
    b = plan.step_blocks()[0]
    r = b - plan.schur_apply(dc.contiguous(), "fp64")
    return float(torch.linalg.norm(r) / torch.linalg.norm(b))


def run_leg(bamg, name, cache, steps, warmup):
    """One extra workload: multigrid and block Jacobi in FP64 and in the
    precision form, the products and tile-kernel rooflines, the true residual
    of each step under the FP64 product, and (largest scene) the adjoint."""
    import torch
    from scenes import cached_scene
    t0 = time.time()
    sc = cached_scene(name, cache)
    log(f"[bench] leg {name}: scene {sc.summary()} ready in {time.time() - t0:.1f}s")
    cams, pts, uv, oc, op = to_device(sc, torch, "cuda:0")
    base = dict(rtol=1e-6, max_iter=5000)
    t0 = time.time()
    plan = bamg.Plan(sc.n_cam, sc.n_pt, oc, op, bamg.Options(precond="mg", **base))
    torch.cuda.synchronize()
    leg = {"workload": f"{name}: {WORKLOADS[name]}, {sc.n_cam} cameras, {sc.n_pt} points, {sc.n_obs} "
                       f"observations (seeded)",
           "plan_s": time.time() - t0, "levels": plan.mg_levels(),
           "device_GiB": plan.device_bytes / 2 ** 30}
    log(f"[bench] leg {name}: plan {leg['plan_s']:.1f}s, levels {leg['levels']}, {leg['device_GiB']:.1f} GiB")
    runs = {}
    ref = None
    for key, pc, prec, n, w in (("mg_fp64", "mg", "fp64", steps, warmup), ("mg_mixed", "mg", "mixed", steps, warmup),
                                ("bj_fp64", "bj", "fp64", 1, 1), ("bj_mixed", "bj", "mixed", 1, 1)):
        o = bamg.Options(precond=pc, precision=prec, **base)
        ms, _, st, dc, dp = time_steps(plan, cams, pts, uv, o, n, w)
        if key == "mg_fp64":
            ref = dc.clone()
        runs[key] = step_entry(ms, st, dc, ref)
        runs[key]["true_rel_res"] = true_residual(plan, bamg, cams, pts, uv, dc, base)
        log(f"[bench] leg {name} {key}: {ms:.2f} ms/step, iters {st.iters} (refine {st.refine_steps}), "
            f"true residual {runs[key]['true_rel_res']:.2e}")
        if key == "mg_mixed":
            dc_m, dp_m = dc.clone(), dp.clone()
    leg["steps"] = runs
    leg["matvec"], leg["roofline"] = measure_products(bamg, plan, sc, cams, pts, uv, base)
    if name == "city30k":
        # the differentiation form in the precision form: backward of the step
        # (loss |delta|^2), adjoint PCG with the same hierarchy
        mixed = bamg.Options(precond="mg", precision="mixed", **base)
        bw = []
        for i in range(2):
            torch.cuda.synchronize()
            t1 = time.time()
            g = plan.backward(cams, pts, uv, dc_m, dp_m, 2 * dc_m, 2 * dp_m, opts=mixed)
            torch.cuda.synchronize()
            if i > 0:
                bw.append(time.time() - t1)
        gst = g[3]
        leg["adjoint"] = {"s_per_backward": sum(bw) / len(bw), "pcg_iters": gst.iters,
                          "adjoint_solve_and_gradients_ms": gst.t_solve_ms,
                          "setup_ms": gst.t_setup_ms, "jacobian_and_blocks_ms": gst.t_jacobian_ms}
        log(f"[bench] leg {name} adjoint: {leg['adjoint']['s_per_backward'] * 1e3:.1f} ms "
            f"(solve and gradients {gst.t_solve_ms:.1f} ms, {gst.iters} PCG)")
    del plan
    torch.cuda.empty_cache()
    return leg


def kernel_only(bamg, name, cache, reps):
    """Only the tile kernel, for counter collection: reps launches of
    k_schur_groups_rc<double>, then of k_schur_groups<float>, on `name`."""
    import torch
    from scenes import cached_scene
    sc = cached_scene(name, cache)
    cams, pts, uv, oc, op = to_device(sc, torch, "cuda:0")
    base = dict(rtol=1e-6, max_iter=5000)
    plan = bamg.Plan(sc.n_cam, sc.n_pt, oc, op, bamg.Options(precond="bj", **base))
    x = torch.randn(sc.n_cam, 9, dtype=torch.float64, device="cuda:0")
    y = torch.zeros_like(x)
    out = {"scene": name, "reps": reps, "n_obs": int(sc.n_obs), "n_pt": int(sc.n_pt), "n_cam": int(sc.n_cam)}
    for prec, mode, s in (("fp64", "fp64", 8), ("fp32", "mixed", 4)):
        plan.prepare(cams, pts, uv, opts=bamg.Options(precond="bj", precision=mode, **base))
        torch.cuda.synchronize()
        for _ in range(reps):
            plan.schur_offdiag_apply(x, y, mode)
        torch.cuda.synchronize()
        out[f"algorithmic_bytes_{prec}"] = kernel_bytes(sc.n_obs, sc.n_pt, sc.n_cam, s)
    out["kernel_source_sha"] = kernel_source_hash()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scene", default="city2k")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the long-path and largest-scene legs")
    ap.add_argument("--legs", default="path10k,city30k", help="comma-separated extra workloads")
    ap.add_argument("--scene-cache", default=None,
                    help="directory for generated scenes (npz), reused by later runs on the same machine")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only launch the Schur tile kernel (FP64 then FP32) on --scene, for counters")
    ap.add_argument("--lm-iters", type=int, default=100, help="iteration cap of the LM loop runs (100 as in the paper)")
    ap.add_argument("--scaling", default=None,
                    help="comma-separated k: run the scaling study on k x k city grids with a sine-wave "
                         "long-range error instead of the benchmark (one JSON line per run, then a summary)")
    ap.add_argument("--scaling-lm", action="store_true",
                    help="with --scaling: time whole LM runs (Nash-Sofer tau 0.01) to a common final cost")
    ap.add_argument("--scaling-lambda", type=float, default=1e-4,
                    help="Marquardt damping of the --scaling linear solves (smaller: closer to the late LM "
                         "iterations, whose large trust radius leaves the long-range modes nearly undamped)")
    ap.add_argument("--scaling-loss", default="huber", choices=["huber", "squared"],
                    help="loss of the --scaling-lm runs (Huber, as in the paper's LM experiment)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device 5 times (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(2 ** 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 2 ** 30, "copy_bytes_written_per_launch": 2 ** 30}),
              flush=True)
        return

    import paper_2007_01941_amd as bamg
    from scenes import cached_scene

    if args.kernel_only:
        kernel_only(bamg, args.scene, args.scene_cache, 5)
        return

    if args.scaling:
        ks = [int(k) for k in args.scaling.split(",")]
        if args.scaling_lm:
            run_scaling_lm(ks, args.lm_iters, args.scaling_loss)
        else:
            run_scaling(ks, max(1, args.steps), args.warmup, args.scaling_lambda)
        return

    dev = torch.device("cuda:0")
    t0 = time.time()
    sc = cached_scene(args.scene, args.scene_cache)
    log(f"[bench] scene {sc.summary()} ready in {time.time() - t0:.1f}s")
    cams, pts, uv, oc, op = to_device(sc, torch, dev)
    torch.cuda.synchronize()

    base = dict(rtol=1e-6, max_iter=5000)
    t0 = time.time()
    plan = bamg.Plan(sc.n_cam, sc.n_pt, oc, op, bamg.Options(precond="mg", **base))
    torch.cuda.synchronize()
    plan_s = time.time() - t0
    log(f"[bench] plan built in {plan_s:.2f}s, levels {plan.mg_levels()}, "
        f"device bytes {plan.device_bytes / 2**30:.2f} GiB")

    # ---- headline: MG, FP64
    mg64 = bamg.Options(precond="mg", precision="fp64", **base)
    ms, wall, st, dc, dp = time_steps(plan, cams, pts, uv, mg64, args.steps, args.warmup)
    log(f"[bench] MG FP64: {ms:.2f} ms/step (iters {st.iters}, rel_res {st.rel_res:.2e}, "
        f"jac {st.t_jacobian_ms:.2f} setup {st.t_setup_ms:.2f} solve {st.t_solve_ms:.2f} ms)")
    result = {
        "metric": METRIC, "value": ms / 1e3, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{sc.name}: {WORKLOADS.get(sc.name, 'synthetic scene')}, {sc.n_cam} cameras, "
                               f"{sc.n_pt} points, {sc.n_obs} observations (seeded)",
                   "precond": "multigrid", "precision": "fp64", "rtol": 1e-6, "lambda": 1e-4,
                   "parallelism": "single GPU"},
        "phases_ms": {"jacobian_and_blocks": st.t_jacobian_ms, "mg_setup": st.t_setup_ms,
                      "pcg_and_backsub": st.t_solve_ms},
        "pcg_iters": st.iters, "rel_res": st.rel_res, "levels": st.nodes,
        "plan_s": plan_s,
    }

    # ---- dominant kernel: the Schur tile kernel, timed on the library's stream
    mat, roof = measure_products(bamg, plan, sc, cams, pts, uv, base)
    result["matvec"] = mat
    result["roofline"] = roof["fp64"]
    result["roofline_fp32"] = roof["fp32"]

    # ---- comparison variants
    if not args.no_variants:
        var = {}
        for name, opts in (("bj_fp64", bamg.Options(precond="bj", precision="fp64", **base)),
                           ("cj_fp64", bamg.Options(precond="cj", precision="fp64", **base)),
                           ("mg_mixed", bamg.Options(precond="mg", precision="mixed", **base)),
                           ("bj_mixed", bamg.Options(precond="bj", precision="mixed", **base)),
                           ("mg_fp64_deterministic", bamg.Options(precond="mg", precision="fp64",
                                                                  deterministic=True, **base)),
                           ("mg_fp64_graph", bamg.Options(precond="mg", precision="fp64", graph=True, **base))):
            vms, _, s2, vdc, _ = time_steps(plan, cams, pts, uv, opts, max(2, args.steps // 2), 1)
            var[name] = step_entry(vms, s2, vdc, dc)
            log(f"[bench] {name}: {vms:.2f} ms/step, iters {s2.iters}, rel_res {s2.rel_res:.2e}")
        # smoothed aggregation needs a plan built for it (its coarse patterns fill in)
        t0 = time.time()
        sa_opts = bamg.Options(precond="mg", precision="fp64", prolongator="smoothed", **base)
        sa_plan = bamg.Plan(sc.n_cam, sc.n_pt, oc, op, sa_opts)
        torch.cuda.synchronize()
        sa_plan_s = time.time() - t0
        vms, _, s2, vdc, _ = time_steps(sa_plan, cams, pts, uv, sa_opts, max(2, args.steps // 2), 1)
        var["mg_fp64_smoothed"] = dict(step_entry(vms, s2, vdc, dc), plan_s=sa_plan_s,
                                       device_bytes=sa_plan.device_bytes)
        log(f"[bench] mg_fp64_smoothed: {vms:.2f} ms/step, iters {s2.iters}, setup {s2.t_setup_ms:.2f} ms, "
            f"solve {s2.t_solve_ms:.2f} ms, plan {sa_plan_s:.2f} s, {sa_plan.device_bytes / 2**30:.2f} GiB")
        del sa_plan
        result["variants"] = var

    # ---- differentiation form: the adjoint of the step (loss |delta|^2, so dL/d delta = 2 delta)
    if not args.no_variants:
        bw = []
        for i in range(3):
            torch.cuda.synchronize()
            t0 = time.time()
            g = plan.backward(cams, pts, uv, dc, dp, 2 * dc, 2 * dp, opts=mg64)
            torch.cuda.synchronize()
            if i > 0:
                bw.append(time.time() - t0)
        gst = g[3]
        result["adjoint"] = {"s_per_backward": sum(bw) / len(bw), "pcg_iters": gst.iters,
                             "phases_ms": {"jacobian_and_blocks": gst.t_jacobian_ms, "setup": gst.t_setup_ms,
                                           "adjoint_solve_and_gradients": gst.t_solve_ms}}
        log(f"[bench] adjoint (backward of the step): {result['adjoint']['s_per_backward'] * 1e3:.2f} ms, "
            f"iters {gst.iters}")

    # ---- the Levenberg-Marquardt loop with the Nash-Sofer rule at the paper's
    # constant forcing tolerances, multigrid vs block Jacobi (the linear solves
    # of every nonlinear iteration, as in the paper's timing)
    if not args.no_variants:
        lmres = {}
        for pc, tau, loss in (("mg", 0.1, "squared"), ("bj", 0.1, "squared"), ("mg", 0.01, "squared"),
                              ("bj", 0.01, "squared"), ("mg", 0.01, "huber"), ("bj", 0.01, "huber")):
            o = bamg.Options(precond=pc, precision="fp64", rtol=1e-10, max_iter=5000,
                             stop_rule="nash_sofer", forcing=tau, loss=loss)
            c2, p2 = cams.clone(), pts.clone()
            torch.cuda.synchronize()
            t0 = time.time()
            out = plan.lm_solve(c2, p2, uv, opts=o, lm_opts=bamg.LMOptions(max_iters=args.lm_iters))
            torch.cuda.synchronize()
            wall = time.time() - t0
            key = f"{pc}_tau{tau}" + ("_huber" if loss == "huber" else "")
            lmres[key] = {"s": wall, "lm_iters": out.iters, "accepted": out.accepted, "pcg_iters": out.pcg_iters,
                          "termination": out.termination, "cost0": out.cost0, "cost": out.cost}
            log(f"[bench] LM {pc} tau {tau} {loss}: {wall * 1e3:.1f} ms, {out.iters} iterations "
                f"({out.accepted} accepted, {out.pcg_iters} PCG), cost {out.cost0:.4e} -> {out.cost:.6e}, "
                f"stop: {out.termination}")
        result["lm_solve"] = lmres

    # ---- CPU baseline: the oracle on a bounded sample of the same workload
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(sc, st.iters)

    # ---- the other workloads of the metric, each on its own plan
    del plan
    torch.cuda.empty_cache()
    if not args.no_legs:
        result["legs"] = {name: run_leg(bamg, name, args.scene_cache, 3, 1)
                          for name in args.legs.split(",") if name and name != sc.name}
    print(json.dumps(result), flush=True)


SCALING_PRECONDS = ("mg", "sa", "bj", "cj")


def scaling_plans(sc, dev):
    """One plan per hierarchy kind on a scene: the unsmoothed one (serves mg,
    bj and cj) and one built for the smoothed prolongator (sa)."""
    import numpy as np
    import torch
    import paper_2007_01941_amd as bamg
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.int32, device=dev)
    plain = bamg.Plan(sc.n_cam, sc.n_pt, T(sc.obs_cam), T(sc.obs_pt), bamg.Options(precond="mg"))
    smooth = bamg.Plan(sc.n_cam, sc.n_pt, T(sc.obs_cam), T(sc.obs_pt),
                       bamg.Options(precond="mg", prolongator="smoothed"))
    return {"mg": plain, "bj": plain, "cj": plain, "sa": smooth}


def scaling_opts(pc, **kw):
    import paper_2007_01941_amd as bamg
    if pc == "sa":
        return bamg.Options(precond="mg", prolongator="smoothed", **kw)
    return bamg.Options(precond=pc, **kw)


def fit_exponents(rows, keys):
    import numpy as np
    fits = {}
    for pc in SCALING_PRECONDS:
        r = [x for x in rows if x["precond"] == pc]
        if len(r) >= 2:
            n = np.log([x["n_cam"] for x in r])
            fits[pc] = {k: float(np.polyfit(n, np.log([max(x[k], 1e-9) for x in r]), 1)[0]) for k in keys}
    return fits


def run_scaling(ks, steps, warmup, lam=1e-4):
    """Fig. 6's experiment: one LM linear solve (FP64, rtol 1e-6) with
    multigrid (unsmoothed and smoothed aggregation), point block Jacobi and
    visibility-based block Jacobi on k x k city grids whose initial values carry
    a sine-wave long-range error (problems of growing diameter). Reported per
    solve: the linear solve time without the preconditioner setup (the
    figure's quantity, also per camera), the setup time, and the whole step;
    the summary fits time ~ n_cam^e per preconditioner."""
    import numpy as np
    import torch
    from scenes import make_scene

    dev = torch.device("cuda:0")
    rows = []
    for k in ks:
        sc = make_scene(f"sine{k}")
        T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        cams, pts, uv = T(sc.cams), T(sc.pts), T(sc.uv)
        plans = scaling_plans(sc, dev)
        for pc in SCALING_PRECONDS:
            plan = plans[pc]
            o = scaling_opts(pc, rtol=1e-6, max_iter=50000, lam=lam)
            for _ in range(warmup):
                plan.lm_step(cams, pts, uv, opts=o)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            solve = setup = 0.0
            e0.record()
            for _ in range(steps):
                _, _, st = plan.lm_step(cams, pts, uv, opts=o)
                solve += st.t_solve_ms
                setup += st.t_setup_ms
            e1.record()
            torch.cuda.synchronize()
            row = {"k": k, "n_cam": sc.n_cam, "n_pt": sc.n_pt, "n_obs": sc.n_obs, "precond": pc, "lambda": lam,
                   "ms_per_solve": e0.elapsed_time(e1) / steps, "solve_ms": solve / steps,
                   "setup_ms": setup / steps, "solve_us_per_cam": 1e3 * solve / steps / sc.n_cam,
                   "pcg_iters": st.iters, "levels": st.nodes, "rel_res": st.rel_res}
            rows.append(row)
            log(f"[scaling] k={k} n_cam={sc.n_cam} {pc}: solve {row['solve_ms']:.2f} ms "
                f"({row['solve_us_per_cam']:.2f} us/camera), setup {row['setup_ms']:.2f} ms, "
                f"{st.iters} iterations")
            print(json.dumps(row), flush=True)
        del plans
    print(json.dumps({"metric": "scaling: LM linear solve to rtol 1e-6 vs n_cam, sine-wave long-range error",
                      "lambda": lam, "fits": fit_exponents(rows, ("solve_ms", "setup_ms", "ms_per_solve", "pcg_iters"))}),
          flush=True)


def run_scaling_lm(ks, lm_iters, loss):
    """Fig. 7's protocol over the grids of Fig. 6: for each k x k sine-noise
    city grid, LM runs (Nash-Sofer rule, constant tau = 0.01, FP64, the given
    loss) with every preconditioner; each run is timed up to the first
    iteration at which its cost reaches the highest final cost of all runs (so
    that all end at the same objective), summing the iterations' times (linear
    solve, setup, cost evaluations)."""
    import numpy as np
    import torch
    import paper_2007_01941_amd as bamg
    from scenes import make_scene

    dev = torch.device("cuda:0")
    rows = []
    for k in ks:
        sc = make_scene(f"sine{k}")
        T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        cams, pts, uv = T(sc.cams), T(sc.pts), T(sc.uv)
        plans = scaling_plans(sc, dev)
        runs = {}
        for pc in SCALING_PRECONDS:
            o = scaling_opts(pc, rtol=1e-10, max_iter=5000, stop_rule="nash_sofer", forcing=0.01, loss=loss)
            runs[pc] = plans[pc].lm_solve(cams.clone(), pts.clone(), uv, opts=o,
                                          lm_opts=bamg.LMOptions(max_iters=lm_iters))
        target = max(r.cost for r in runs.values())
        for pc, out in runs.items():
            t, cost, n_it, pcg = 0.0, out.cost0, 0, 0
            for h in out.history:
                t += h.t_ms
                pcg += h.pcg_iters
                n_it += 1
                if h.accepted:
                    cost = h.cost_candidate
                if cost <= target * (1 + 1e-12):
                    break
            row = {"k": k, "n_cam": sc.n_cam, "n_obs": sc.n_obs, "precond": pc, "loss": loss,
                   "ms_to_target": t, "lm_iters_to_target": n_it, "pcg_iters_to_target": pcg,
                   "target_cost": target, "cost0": out.cost0, "final_cost": out.cost, "lm_iters": out.iters,
                   "costs": [h.cost_candidate if h.accepted else None for h in out.history]}
            rows.append(row)
            log(f"[scaling-lm] k={k} n_cam={sc.n_cam} {pc}: {t:.1f} ms to cost {target:.6e} "
                f"({n_it} LM iterations, {pcg} PCG; final cost {out.cost:.6e})")
            print(json.dumps(row), flush=True)
        del plans
    print(json.dumps({"metric": "scaling: LM time to a common cost vs n_cam (tau 0.01, sine-wave long-range error)",
                      "loss": loss, "fits": fit_exponents(rows, ("ms_to_target", "pcg_iters_to_target"))}),
          flush=True)


def subsample_points(sc, every):
    """The scene restricted to every `every`-th point (all cameras kept)."""
    import numpy as np
    keep = np.zeros(sc.n_pt, dtype=bool)
    keep[::every] = True
    remap = -np.ones(sc.n_pt, dtype=np.int64)
    remap[keep] = np.arange(int(keep.sum()))
    m = keep[sc.obs_pt]
    return (sc.cams, sc.pts[keep], sc.obs_cam[m], remap[sc.obs_pt[m]].astype(np.int32), sc.uv[m])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample_run(cams, pts, oc, op, uv, sample_iters):
    """The oracle's phases on one sample: (jacobian s, setup s, s per MG-PCG
    iteration, CPU seconds used, wall seconds)."""
    from oracle import multigrid as omg
    from oracle import step as ostep
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    w0 = time.time()
    t = time.time()
    nrm = ostep.normal_for(cams, pts, oc, op, uv)
    b = nrm.rhs()
    t_jac = time.time() - t
    t = time.time()
    levels = ostep.hierarchy_for(nrm, cams, oc, op, omg.MGOptions())
    t_setup = time.time() - t
    t = time.time()
    omg.pcg(nrm.S_apply, lambda r: omg.vcycle(levels, r), b, 1e-30, max_iter=sample_iters)
    t_iter = (time.time() - t) / sample_iters
    wall = time.time() - w0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return t_jac, t_setup, t_iter, cpu, wall


def cpu_baseline(sc, gpu_iters):
    """The oracle (numpy/scipy FP64, as written) timed on a bounded sample of the
    workload: every 4th point of the same scene with all its cameras. Residual,
    Jacobian and normal blocks, the multigrid hierarchy setup, and 3 MG-PCG
    iterations are timed, once with the host's default thread count (all cores
    available to BLAS) and once restricted to one thread; every phase scales
    with the observation count, so the per-step estimate scales them by
    n_obs(full)/n_obs(sample) and the iterations to the GPU's iteration count."""
    from threadpoolctl import threadpool_limits

    log("[bench] oracle CPU baseline on a point subsample ...")
    cams, pts, oc, op, uv = subsample_points(sc, 4)
    scale = sc.n_obs / oc.shape[0]
    sample_iters = 3
    out = {}
    for key, limit in (("all_cores", None), ("one_thread", 1)):
        with threadpool_limits(limits=limit):
            t_jac, t_setup, t_iter, cpu, wall = oracle_sample_run(cams, pts, oc, op, uv, sample_iters)
        est = scale * (t_jac + t_setup + gpu_iters * t_iter)
        out[key] = {"s_per_step": est, "cores": round(cpu / wall, 2), "sample_wall_s": round(wall, 1),
                    "phases_s": {"jacobian_and_blocks": scale * t_jac, "mg_setup": scale * t_setup,
                                 "pcg": scale * gpu_iters * t_iter, "per_pcg_iteration": scale * t_iter}}
        log(f"[bench] oracle ({key}): jac {t_jac:.1f}s setup {t_setup:.1f}s {t_iter:.2f}s/iter "
            f"(x{scale:.2f}) -> {est:.1f}s per step at {gpu_iters} iterations, {cpu / wall:.2f} cores")
    a = out["all_cores"]
    return {"value": a["s_per_step"], "unit": "s", "cores": a["cores"], "kind": "oracle",
            "sample": (f"oracle (numpy/scipy FP64) on every 4th point of {sc.name} with all "
                       f"{sc.n_cam} cameras ({oc.shape[0]} of {sc.n_obs} observations): residual, "
                       f"Jacobian and normal blocks, multigrid setup and {sample_iters} MG-PCG iterations "
                       f"timed; scaled by the observation ratio {scale:.2f} and to the GPU's {gpu_iters} "
                       f"iterations"),
            "phases_s": a["phases_s"], "one_thread": out["one_thread"], "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(), "sample_wall_s": a["sample_wall_s"]}


if __name__ == "__main__":
    main()
