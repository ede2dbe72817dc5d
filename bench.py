"""Throughput of the FTK hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fp32|bf16x3|all]

One step = one pass of the whole hot path over one batch of synthetic
input already resident in HBM: transform of the 512 images and the 2048
templates (n = 128) to Fourier-Bessel coefficients, Step 1 (image x template
contraction per mode), Step 3 (shift contraction, 197 shifts), the rotation
FFT over all 256 rotations and the best pose of every pair.  Planning and
the shift table are built once, outside the timed region.

Prints one JSON line: the metric's value is whole-job pairs/s for the chosen
form; the plain FP32 form is reported beside it, with per-stage times from
HIP events, the roofline of the dominant kernel, and the FP64 CPU oracle
timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pairs/s (N shifts × all rotations) at eps=1e-3, chosen form vs plain FTK"
WORKLOAD = dict(name="cryoem_n128", n_images=512, n_templates=2048, n=128, M=64, Qa=256, R=4.0, nblob=60,
                snr=0.05, eps=1e-3, seed=2)
PEAK_FP32_MFMA = 157.3e12
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12

# HBM bytes per Step 3 launch on this workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by a 1 GiB copy: x2.000 and x1.000), with the SHA-1 of
# the kernel sources they were taken on; a changed kernel reports null.
# Source: profiles/step3_<form>_cryoem_n128.md.
TRAFFIC = {
    "bf16x3": {"bytes_per_launch": 1.979e9, "sources": ["kern_align_bf16.hip", "device_common.h", "kernels.h"],
               "sha1": "198454c973ab97fce6fc65c1b050615ff55b03a3"},
    "fp32": {"bytes_per_launch": 1.947e9, "sources": ["kern_align.hip", "device_common.h", "kernels.h"],
             "sha1": "cabab2a75e782c8bc8b41310b0042a7371882c1f"},
}


def measured_traffic(form):
    import hashlib
    t = TRAFFIC.get(form)
    if t is None:
        return None
    h = hashlib.sha1()
    for name in t["sources"]:
        with open(os.path.join(ROOT, "paper_1905_12317_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return t["bytes_per_launch"] if h.hexdigest() == t["sha1"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(w):
    import synth
    s = synth.make_alignment_set(w["seed"], w["n"], w["n_templates"], w["n_images"], w["nblob"], w["R"],
                                 w["snr"])
    return s


def flops_per_pair(H, M, N, Qa):
    """Algorithmic FLOP of one image-template pair (real-input symmetry: modes
    q = 0..Qa/2 of Step 1; Step 3 on the Qa/2 packed modes)."""
    step1 = 8.0 * H * M * (Qa // 2 + 1)
    step3 = 8.0 * N * H * (Qa // 2)
    fft = 2.5 * N * Qa * math.log2(Qa)
    return step1, step3, fft


def run_form(form, inputs, w, steps, warmup, shifts):
    import torch
    from paper_1905_12317_amd import ftk
    dev = torch.device("cuda:0")
    P = ftk.Plan(w["n"], w["M"], w["Qa"], w["R"], w["eps"], precision=form)
    P.set_shifts(shifts)
    info = P.info()
    images = torch.as_tensor(inputs.images, dtype=torch.float32, device=dev).contiguous()
    templates = torch.as_tensor(inputs.templates, dtype=torch.float32, device=dev).contiguous()
    nA, nB = images.shape[0], templates.shape[0]
    best = torch.empty((nA, nB, 3), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        P.align(images, templates, best=best, stream=stream)
    torch.cuda.synchronize()
    P.profile(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        P.align(images, templates, best=best, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    stages = P.stage_times()
    P.profile(False)
    poses = ftk.poses_numpy(best)
    ms_step = ms_total / steps
    return dict(form=form, info=info, ms_per_step=ms_step, wall_s=wall, pairs_per_s=nA * nB / (ms_step / 1e3),
                stages=stages, poses=poses)


def recall(poses, inputs, shifts, Qa):
    """Fraction of images whose best template over all templates is the one
    they were made from (the paper's consistency check)."""
    v = poses["value"].astype(np.float64)
    best_t = np.argmax(v, axis=1)
    return float(np.mean(best_t == inputs.true_template))


def cpu_baseline(inputs, w, shifts, n_img=8, n_tmp=48):
    """The FP64 oracle as it stands (direct NUDFT transform + FP64 FTK) on a
    bounded sample of the same workload, timed on the host."""
    from oracle import ftk as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    plan = O.set_shifts(O.make_plan(w["n"], w["M"], w["Qa"], w["R"], w["eps"]), shifts)
    t = time.perf_counter()
    a = [O.fb_coefficients(x, plan) for x in inputs.images[:n_img]]
    b = [O.fb_coefficients(x, plan) for x in inputs.templates[:n_tmp]]
    for ai in a:
        for bj in b:
            X = O.ftk_X(ai, bj, plan)
            O.best_pose(X)
    dt = time.perf_counter() - t
    return {"value": n_img * n_tmp / dt, "unit": "pairs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {n_img} images x {n_tmp} templates ({n_img * n_tmp} pairs) of the same workload: "
                      f"direct FP64 NUDFT transform of the {n_img + n_tmp} images + FP64 FTK + argmax, "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", default="all", choices=["fp32", "bf16x3", "all"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (3 times) and exit; "
                         "used to scale the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.calibrate_copy_mib > 0:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.calibrate_copy_mib, "bytes_read": n * 4, "bytes_written": n * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard templates across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    import synth
    w = WORKLOAD
    t = time.perf_counter()
    inputs = make_inputs(w)
    shifts = synth.shift_lattice(w["R"])
    log(f"inputs generated in {time.perf_counter() - t:.1f} s: {w['n_images']} x {w['n_templates']} "
        f"n={w['n']} N={len(shifts)}")
    forms = ["fp32", "bf16x3"] if args.form == "all" else [args.form]
    results = {}
    for f in forms:
        try:
            results[f] = run_form(f, inputs, w, args.steps, args.warmup, shifts)
            r = results[f]
            log(f"[{f}] {r['ms_per_step']:.2f} ms/step, {r['pairs_per_s']:.4g} pairs/s, stages {r['stages']}")
        except Exception as e:  # a form that is not available is reported, not fatal
            log(f"[{f}] failed: {e}")
    if not results:
        sys.exit(1)
    chosen = max(results, key=lambda k: results[k]["pairs_per_s"])
    r = results[chosen]
    info = r["info"]
    H, M, N, Qa = info["H"], info["M"], info["N"], info["Qa"]
    s1, s3, fft = flops_per_pair(H, M, N, Qa)
    pairs = w["n_images"] * w["n_templates"]
    ms3, n3 = r["stages"]["step3"]
    ms1, n1 = r["stages"]["step1"]
    # dominant kernel: Step 3 (shift contraction + FFT + argmax), MFMA bound
    per_launch_pairs = pairs * args.steps / max(n3, 1)
    avg3 = ms3 / max(n3, 1) / 1e3
    achieved = s3 * per_launch_pairs / avg3 if avg3 > 0 else 0.0
    peak = PEAK_FP32_MFMA if chosen == "fp32" else PEAK_BF16_MFMA
    traffic = measured_traffic(chosen)
    out = {
        "metric": METRIC, "value": r["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if chosen == "fp32" else "bf16x3->f32", "data": "synthetic",
        "config": {"workload": f"{w['name']}: {w['n_images']} images x {w['n_templates']} templates, n={w['n']}, "
                               f"60-blob templates, SNR {w['snr']}, M={M}, Qa={Qa} rotations, N={N} shifts "
                               f"(0.5 px lattice, R={w['R']} px), eps={w['eps']}, H={H}",
                   "form": chosen, "pairs": pairs,
                   "forms": {k: {"pairs_per_s": v["pairs_per_s"], "ms_per_step": v["ms_per_step"],
                                 "stage_ms_per_step": {s: v["stages"][s][0] / args.steps for s in v["stages"]}}
                             for k, v in results.items()},
                   "speedup_vs_plain_fp32": (r["pairs_per_s"] / results["fp32"]["pairs_per_s"]
                                             if "fp32" in results else None),
                   "recall_true_template": recall(r["poses"], inputs, shifts, Qa),
                   "gflop_per_pair": (s1 + s3 + fft) / 1e9},
        "roofline": {"kernel": "step3 (shift contraction on MFMA + rotation FFT + argmax)", "bound": "mfma",
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_GBps": traffic / avg3 / 1e9 if traffic and avg3 > 0 else None,
                     "products_per_mac": 3 if chosen == "bf16x3" else 1,
                     "frac_of_form_ceiling": (achieved / (peak / 3) if chosen == "bf16x3" else achieved / peak),
                     "algorithmic_flop_per_pair": s3, "pairs_per_launch": per_launch_pairs,
                     "avg_launch_ms": avg3 * 1e3,
                     "step1_achieved": (s1 * pairs * args.steps / max(n1, 1)) / (ms1 / max(n1, 1) / 1e3) / 1e12
                     if ms1 > 0 else None},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inputs, w, shifts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
