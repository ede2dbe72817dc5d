"""Throughput of the FTK hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fp32|bf16x3|fp16x3|fp16|fp16+bf16x3|all]

One step = one pass of the whole hot path over one batch of synthetic
input already resident in HBM: transform of the 512 images and the 2048
templates (n = 128) to Fourier-Bessel coefficients, Step 1 (image x template
contraction per mode), Step 3 (shift contraction, 197 shifts), the rotation
FFT over all 256 rotations and the best pose of every pair.  Planning and
the shift table are built once, outside the timed region.

Forms: fp32, bf16x3 (split bf16, three products), fp16x3 (split fp16 on
power-of-two scaled operands, three products), fp16 (one product), and
fp16+bf16x3 (the FP16 form over every pair, then the split form on each
image's four best FP16 templates; its per-image best comes from the second
pass).

Prints one JSON line: the metric's value is whole-job pairs/s for the chosen
form (the fastest whose per-image best poses agree with the FP32 form's on
at least 99 % of images); the plain FP32 form is reported beside it, with per-stage times from
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
PEAK_BF16_MFMA = 2.5e15  # dense bf16 and fp16
PEAK_HBM = 8.0e12

# HBM bytes per Step 3 launch on this workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by a 1 GiB copy: x2.000 and x1.000), with the SHA-1 of
# the kernel sources they were taken on; a changed kernel reports null.
# Source: profiles/step3_<form>_cryoem_n128.md.
TRAFFIC = {
    "bf16x3": {"bytes_per_launch": 8.791e+09, "sources": ["kern_align_bf16.hip", "step3_epilogue.h", "device_common.h", "kernels.h"],
        "sha1": "5687834082d6ed5b4696aa9481364c1488e58666"},
    "fp32": {"bytes_per_launch": 9.627e+09, "sources": ["kern_align.hip", "step3_epilogue.h", "device_common.h", "kernels.h"],
        "sha1": "700029d305407183e020a799f8ad560623527315"},
    "fp16": {"bytes_per_launch": 8.626e+09, "sources": ["kern_align_fp16.hip", "step3_epilogue.h", "device_common.h", "kernels.h"],
        "sha1": "256126cff62d64aa3273599c0e60be1a69efba83"},
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


REFINE_K = 4  # templates per image re-aligned by the split form in the two-pass form
# joint translation-CTF measurement: 300 kV, Cs 2.7 mm, 7 % amplitude contrast,
# 2 A pixels, a 14000-16000 A defocus window searched at 5 values
CTF_PARAMS = dict(wavelength_A=0.019687, cs_mm=2.7, amplitude_contrast=0.07, pixel_A=2.0,
                  defocus_min_A=14000.0, defocus_max_A=16000.0)
CTF_DEFOCI = [14000.0, 14500.0, 15000.0, 15500.0, 16000.0]
BFR_TEMPLATES = 256  # templates of the brute-force-rotation sample (all images)
UPSAMPLE = 5  # rotation upsampling factor of the upsampled measurement (5 x 256 = 1280 rotations)
WEIGHTED_EPS = 5e-3  # eps of the weighted-SVD plan: the paper plan's accuracy at eps = 1e-3 (see main)


def run_form(form, inputs, w, steps, warmup, shifts, eps=None, weight=None, up=1, ctf=None, defoci=None,
             n_images=None, n_templates=None):
    """One form over the workload.  "fp16+bf16x3" is the two-pass form: the
    FP16 form over every pair, then the split form on each image's REFINE_K
    best FP16 templates (ftk_align_refined).  "bft": brute-force
    translations (ftk_bft_align, FP32), "bfr": brute-force rotations
    (ftk_bfr_align, FP32), the paper's comparison methods.  eps / weight: a
    plan other than the workload's (the k-side weighted operator SVD).
    n_images / n_templates: the first ones only (a sample of the workload)."""
    import torch
    from paper_1905_12317_amd import ftk
    dev = torch.device("cuda:0")
    two = form == "fp16+bf16x3"
    bft = form == "bft"
    bfr = form == "bfr"
    prec = "fp16" if two else ("fp32" if (bft or bfr) else form)
    P = ftk.Plan(w["n"], w["M"], w["Qa"], w["R"], eps or w["eps"], precision=prec, weight=weight, ctf=ctf)
    if ctf is not None:
        # poses: every shift at every defocus value
        P.set_poses(np.repeat(shifts, len(defoci), axis=0), np.tile(np.asarray(defoci, float), len(shifts)))
    else:
        P.set_shifts(shifts)
    if up > 1:
        P.set_rotations(up)
    Pf = None
    if two:
        Pf = ftk.Plan(w["n"], w["M"], w["Qa"], w["R"], w["eps"], precision="bf16x3")
        Pf.set_shifts(shifts)
    info = P.info()
    images = torch.as_tensor(inputs.images[:n_images], dtype=torch.float32, device=dev).contiguous()
    templates = torch.as_tensor(inputs.templates[:n_templates], dtype=torch.float32, device=dev).contiguous()
    nA, nB = images.shape[0], templates.shape[0]
    best = torch.empty((nA, nB, 3), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    if two:
        ca = torch.empty((nA, w["Qa"], w["M"]), dtype=torch.complex64, device=dev)
        cb = torch.empty((nB, w["Qa"], w["M"]), dtype=torch.complex64, device=dev)

    per_image = {}

    def step():
        if two:
            P.transform(images, ca, stream=stream)
            P.transform(templates, cb, stream=stream)
            _, per_image["t"], per_image["pose"] = ftk.align_refined(P, Pf, ca, cb, REFINE_K, best=best,
                                                                      stream=stream)
        elif bft:
            P.bft_align(images, templates, best=best, stream=stream)
        elif bfr:
            P.bfr_align(images, templates, best=best, stream=stream)
        else:
            P.align(images, templates, best=best, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    for q in (P, Pf):
        if q is not None:
            q.profile(True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        step()
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    stages = P.stage_times()
    if Pf is not None:
        fs = Pf.stage_times()
        stages["refine"] = (sum(v[0] for v in fs.values()), sum(v[1] for v in fs.values()))
    for q in (P, Pf):
        if q is not None:
            q.profile(False)
    poses = ftk.poses_numpy(best)
    if two:  # the refined pairs' best, as ftk_align_refined reports it
        bt = per_image["t"].cpu().numpy().astype(np.int64)
        bp = ftk.poses_numpy(per_image["pose"])
        img_best = (bt, bp["shift"], bp["rot"])
    else:
        img_best = image_best(poses)
    ms_step = ms_total / steps
    return dict(form=form, info=info, ms_per_step=ms_step, wall_s=wall, pairs_per_s=nA * nB / (ms_step / 1e3),
                stages=stages, poses=poses, img_best=img_best)


def bfr_flop_per_pair(n, R, shifts):
    """Algorithmic flop of brute-force rotations per pair: per rotation the
    product Ahat conj(Bhat_r) on the half-disk rows (6 per point), the sums
    over u for every x offset (8 per point and offset) and the real parts
    over v for every (x, y) offset (4 per row and offset pair)."""
    V = n // 2
    pts = sum(2 * math.isqrt(V * V - v * v) + 1 for v in range(V + 1))
    dx = len(np.unique(np.asarray(shifts)[:, 0]))
    dy = len(np.unique(np.asarray(shifts)[:, 1]))
    return R * (6 * pts + 8 * dx * pts + 4 * dx * dy * (V + 1))


def oracle_best_pose(inputs, w, shifts, results, chosen, n_img=16, seed=17):
    """Part of the CPU-oracle leg: the FP64 oracle's per-image best
    (template, shift, rotation) on a seeded sample of images against the
    chosen form's and the FP32 form's.  Candidates per image: every template
    whose FP32 best value lies within twice the FP32 error bound (1e-5 of the
    pair scale, bounded through sqrt(X_BB(0, 0)) <= 4 pi for unit-L2
    templates) of the image's FP32 best, plus the chosen form's pick.  The
    oracle's answer counts as decided for a form where its margin over every
    other candidate pose and over the bound of the other templates exceeds
    twice that form's bar (FP32 1e-5 of the pair scale; the reduced forms
    1e-3); both forms are compared on the images decided at the FP32 bar,
    and the chosen form also on those decided at its own bar."""
    from oracle import ftk as O
    plan = O.set_shifts(O.make_plan(w["n"], w["M"], w["Qa"], w["R"], w["eps"]), shifts)
    v32 = results["fp32"]["poses"]
    ct, cs, cr = results[chosen]["img_best"]
    bar = 1e-5 if chosen == "fp32" else 1e-3
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(len(inputs.images), n_img, replace=False))
    sb = 4.0 * math.pi
    decided = same_chosen = 0
    d32 = same32 = same_c32 = 0
    t0 = time.perf_counter()
    for i in sample:
        a = O.fb_coefficients(inputs.images[i], plan)
        e32 = 1e-5 * math.sqrt(O.pair_scale(a, a, plan)) * sb
        vals = v32["value"][i].astype(np.float64)
        cand = sorted(set(np.nonzero(vals >= vals.max() - 2 * e32)[0].tolist()) | {int(ct[i])})
        outside = np.delete(vals, cand)
        others = [outside.max() + e32] if outside.size else []
        best = None
        for j in cand:
            b = O.fb_coefficients(inputs.templates[j], plan)
            X = np.real(O.ftk_X(a, b, plan))
            v, si, ri, margin = O.best_pose(X)
            if best is None or v > best[0]:
                if best is not None:
                    others.append(best[0])
                best = (v, j, si, ri, margin, O.pair_scale(a, b, plan))
            else:
                others.append(v)
        v, j, si, ri, margin, sc = best
        margin = min([margin] + [v - o for o in others])
        ch_eq = (int(ct[i]), int(cs[i]), int(cr[i])) == (j, si, ri)
        j32 = int(np.argmax(vals))
        f32_eq = (j32, int(v32["shift"][i, j32]), int(v32["rot"][i, j32])) == (j, si, ri)
        if margin > 2e-5 * sc:
            d32 += 1
            same32 += int(f32_eq)
            same_c32 += int(ch_eq)
        if margin > 2 * bar * sc:
            decided += 1
            same_chosen += int(ch_eq)
    return {"images": n_img, "decided_at_fp32_bar": d32, "fp32_equal": same32, "chosen_form_equal": same_c32,
            "decided_at_chosen_bar": decided, "chosen_form_equal_there": same_chosen,
            "seconds": time.perf_counter() - t0}


def image_best(poses):
    """Per image: the template with the largest best value (the lower
    template number on ties) and its pose's shift and rotation."""
    bt = np.argmax(poses["value"], axis=1)
    i = np.arange(bt.size)
    return bt, poses["shift"][i, bt], poses["rot"][i, bt]


def agreement(best, ref):
    """Fraction of images whose best template and its pose (shift, rotation)
    under a form equal those under the FP32 form."""
    return float(np.mean((best[0] == ref[0]) & (best[1] == ref[1]) & (best[2] == ref[2])))


def recall(best, inputs):
    """Fraction of images whose best template over all templates is the one
    they were made from (the paper's consistency check)."""
    return float(np.mean(best[0] == inputs.true_template))


def cpu_baseline(inputs, w, shifts, n_img=8, n_tmp=48, n_dir=(2, 4)):
    """The FP64 oracle as it stands, timed on the host on bounded samples of
    the same workload: the FP64 FTK (direct NUDFT transform + eq. fbk3 +
    argmax) on n_img x n_tmp pairs, and the direct inner product on the polar
    quadrature (eq. Xdg discretised, no SVD; polar samples by direct sum +
    argmax) on n_dir[0] x n_dir[1] pairs."""
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
    t = time.perf_counter()
    ah = [O.polar_ft(x, plan.k, plan.Qa) for x in inputs.images[:n_dir[0]]]
    bh = [O.polar_ft(x, plan.k, plan.Qa) for x in inputs.templates[:n_dir[1]]]
    for ai in ah:
        for bj in bh:
            O.best_pose(np.real(O.direct_X(ai, bj, plan.k, plan.w, shifts, w["n"])))
    dt_dir = time.perf_counter() - t
    n_d = n_dir[0] * n_dir[1]
    return {"value": n_img * n_tmp / dt, "unit": "pairs/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 FTK: first {n_img} images x {n_tmp} templates ({n_img * n_tmp} pairs) of the same "
                      f"workload, direct FP64 NUDFT transform of the {n_img + n_tmp} images + FP64 FTK + argmax, "
                      f"{dt:.1f} s; direct inner product (no SVD): first {n_dir[0]} x {n_dir[1]} pairs, {dt_dir:.1f} s",
            "direct_X_pairs_per_s": n_d / dt_dir}


RAGGED = dict(name="ragged_c4", stacks=64, seed=4, nblob=60, snr=0.05, eps=1e-3)
PROPOSAL = dict(name="proposal_c5", n=128, M=64, Qa=256, R=4.0, n_templates=8192, n_clean=16384, n_val=1024,
                n_test=2048, nblob=60, snr=0.05, eps=1e-3, epochs=12, topk=32, hidden=1024, seed=5)
# rings and modes of each feature kind (2048 inputs each); "power" is the
# workload's own: |a(k; q)|^2 over 64 radii x the 32 lowest modes
PROPOSAL_FEATURES = {"power": (64, 32), "cross": (16, 8), "invariant": (64, 32)}


def bench_ragged(args):
    """64 stacks of uneven n, template and image counts and shift radii (the
    ragged workload, image and template counts scaled by --ragged-scale), in
    the --ragged-form precision form: one ftk_batch run (--lanes lanes, one
    hipGraph, autotuned launch shapes) against the same stacks aligned one
    ftk_align at a time."""
    import torch
    import synth
    from paper_1905_12317_amd import ftk
    w = RAGGED
    t0 = time.perf_counter()
    specs = synth.ragged_stack_specs(w["seed"], count=w["stacks"], scale=args.ragged_scale)
    stacks, flop = [], 0.0
    for i, sp in enumerate(specs):
        s = synth.make_alignment_set(1000 * w["seed"] + i, sp["n"], sp["n_templates"], sp["n_images"], w["nblob"],
                                     sp["R"], w["snr"])
        shifts = synth.shift_lattice(sp["R"])
        P = ftk.Plan(sp["n"], sp["M"], sp["Qa"], sp["R"], w["eps"], args.ragged_form)
        P.set_shifts(shifts)
        inf = P.info()
        imgs = torch.as_tensor(s.images, dtype=torch.float32, device="cuda")
        tmps = torch.as_tensor(s.templates, dtype=torch.float32, device="cuda")
        best = torch.empty((imgs.shape[0], tmps.shape[0], 3), dtype=torch.int32, device="cuda")
        stacks.append(dict(plan=P, images=imgs, templates=tmps, best=best))
        flop += imgs.shape[0] * tmps.shape[0] * sum(flops_per_pair(inf["H"], inf["M"], inf["N"], inf["Qa"])[:2])
        if i % 16 == 15:
            log(f"  {i + 1} stacks generated ({time.perf_counter() - t0:.1f} s)")
    pairs = sum(st["images"].shape[0] * st["templates"].shape[0] for st in stacks)
    log(f"ragged inputs in {time.perf_counter() - t0:.1f} s: {len(stacks)} stacks, {pairs} pairs")
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    B = ftk.Batch(stacks, lanes=args.lanes, graph=True, autotune=True, stream=stream)
    tune_s = time.perf_counter() - t0
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup + 1):  # the first run captures the graph
        B.run(stream)
    stream.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        B.run(stream)
    ev1.record(stream)
    stream.synchronize()
    ms_batch = ev0.elapsed_time(ev1) / args.steps
    # the same stacks one after another on one lane, no graph, default launch
    # shapes: the single-stack ftk_align path, sharing one workspace (64
    # plans holding a staging buffer each would not fit at full size)
    S = ftk.Batch(stacks, lanes=1, graph=False, autotune=False, stream=stream)
    S.run(stream)
    stream.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        S.run(stream)
    ev1.record(stream)
    stream.synchronize()
    ms_seq = ev0.elapsed_time(ev1) / args.steps
    info = B.info()
    achieved = flop / (ms_batch / 1e3)
    out = {
        "metric": "pairs/s over a ragged batch of 64 stacks (uneven n, templates, images, shift radius)",
        "value": pairs / (ms_batch / 1e3), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_batch, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": f"{args.ragged_form}->f32", "data": "synthetic",
        "config": {"workload": f"{w['name']}: 64 stacks, n in {{64,96,128,192}}, M=n/2, Qa=2n, templates "
                               f"log-uniform 100-4000 and images 16-256 scaled by {args.ragged_scale}, shift radius "
                               f"2-8 px (0.5 px lattice), 60-blob templates, SNR {w['snr']}, eps={w['eps']}",
                   "form": args.ragged_form, "pairs": pairs, "lanes": info["lanes"], "graph_nodes": info["graph_nodes"],
                   "autotune_s": tune_s, "sequential_ms_per_step": ms_seq, "batch_speedup": ms_seq / ms_batch},
        "roofline": {"kernel": "whole batch (Step 1 + Step 3 algorithmic flop)", "bound": "mfma",
                     "achieved": achieved / 1e12, "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_MFMA, "traffic": None},
    }
    print(json.dumps(out), flush=True)


def bench_proposal(args):
    """Learned proposal on the 8192-template workload at n = 128: train on
    re-noised images labelled each epoch by the two-pass search (FP16 over
    every template, split bf16 on each image's best 4), choose the threshold
    on a validation split, then time the proposal search (with and without
    shift windows) against the full split-bf16 search on a test split."""
    import torch
    import synth
    from paper_1905_12317_amd import ftk
    from paper_1905_12317_amd import proposal as PR
    w = PROPOSAL
    t0 = time.perf_counter()
    n_all = w["n_clean"] + w["n_val"] + w["n_test"]
    s = synth.make_alignment_set(w["seed"], w["n"], w["n_templates"], n_all, w["nblob"], w["R"], w["snr"],
                                 keep_clean=True)
    gen_s = time.perf_counter() - t0
    log(f"[proposal] data {gen_s:.1f} s: {w['n_templates']} templates, {n_all} images")
    shifts = synth.shift_lattice(w["R"])
    bins = PR.shift_bins(shifts)
    kind = args.proposal_features
    n_r, n_q = PROPOSAL_FEATURES[kind]
    n_t, n_s = w["n_templates"], int(bins.max()) + 1
    P = ftk.Plan(w["n"], w["M"], w["Qa"], w["R"], w["eps"], "bf16x3")
    P.set_shifts(shifts)
    P16 = ftk.Plan(w["n"], w["M"], w["Qa"], w["R"], w["eps"], "fp16")
    P16.set_shifts(shifts)
    tmps = torch.as_tensor(s.templates, dtype=torch.float32, device="cuda")
    tc = P.transform(tmps)
    nc = w["n_clean"]
    clean = torch.as_tensor(s.clean[:nc], dtype=torch.float32, device="cuda")
    sig = s.noise_sigma[:nc]
    dims = [ftk.feature_count(kind, n_r, n_q), w["hidden"], w["hidden"], w["hidden"], n_t + n_s]
    net = ftk.MLP(dims, n_t, n_s, "bf16", max_batch=1024)
    net.set_params(synth.mlp_init(w["seed"], dims))
    perms = [synth.permutation(100 + e, nc) for e in range(w["epochs"])]
    labeler = PR.refined_labeler(P16, P, tc, 4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = PR.train_online(net, P, clean, tc, bins, lambda e: synth.gaussian_noise(7000 + e, sig, w["n"]), perms,
                             kind, n_r, n_q, batch=256, lr=2e-3, wd=1e-2, labeler=labeler,
                             log=lambda e, l: log(f"  epoch {e}: loss {l:.4f}"))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    labelled_pairs = w["epochs"] * nc * n_t
    # the network's kernels alone: a training step's loss + gradients, and
    # the forward pass, at batch 256
    feats = ftk.features(P, P.transform(clean[:4096].contiguous()), n_r, n_q, kind=kind)
    lab = torch.zeros(4096, dtype=torch.int32, device="cuda")
    idx = torch.arange(256, dtype=torch.int32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    net.gradients(feats, lab, lab, idx)
    e0.record()
    for _ in range(20):
        net.gradients(feats, lab, lab, idx)
    e1.record()
    torch.cuda.synchronize()
    ms_grad = e0.elapsed_time(e1) / 20
    e0.record()
    for _ in range(20):
        net.forward(feats[:256])
    e1.record()
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1) / 20
    params = sum(dims[i] * dims[i + 1] for i in range(len(dims) - 1))
    mlp_flop = 6.0 * 256 * params
    # threshold on the validation split
    vi = torch.as_tensor(s.images[nc:nc + w["n_val"]], dtype=torch.float32, device="cuda")
    vlab, _ = labeler(P.transform(vi))
    vf = ftk.features(P, P.transform(vi), n_r, n_q, kind=kind)
    top, mass, _ = net.propose(vf, w["topk"])
    hit = (top.cpu().numpy() == vlab.cpu().numpy()[:, None]).any(axis=1)
    tau = PR.choose_tau(mass.cpu().numpy(), hit, max_miss=0.003)
    log(f"[proposal] trained {train_s:.1f} s; validation top-{w['topk']} hit {hit.mean():.3f}, tau {tau:.4f}")
    # test split: the full split-bf16 search and the proposal search, with and
    # without shift windows (annuli of +-0.5 px around each shift bin's radius)
    ti = torch.as_tensor(s.images[nc + w["n_val"]:], dtype=torch.float32, device="cuda")
    nA = ti.shape[0]
    tic = P.transform(ti)
    _, full = P.align_coeffs(tic, tc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, full = P.align_coeffs(P.transform(ti), tc)
    fbt, fbp = ftk.best_template(full)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    fbt, fbp = fbt.cpu().numpy(), fbp.cpu().numpy()
    res = {}
    for mode in ("no_window", "window"):
        P.set_shift_windows(0.5 * np.arange(n_s) if mode == "window" else [], 0.5)
        ftk.align_proposed(P, net, ti, tc, n_r, n_q, w["topk"], tau, kind=kind)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt, bp, fb, nfb = ftk.align_proposed(P, net, ti, tc, n_r, n_q, w["topk"], tau, kind=kind)
        torch.cuda.synchronize()
        t_prop = time.perf_counter() - t0
        same = (bt.cpu().numpy() == fbt) & np.all(bp.cpu().numpy() == fbp, axis=1)
        res[mode] = {"recall": float(same.mean()), "fallback": int(nfb), "ms": t_prop * 1e3,
                     "effective_pairs_per_s": nA * n_t / t_prop, "speedup_vs_full_search": t_full / t_prop}
        log(f"[proposal {mode}] recall {same.mean():.4f}, fallback {nfb}/{nA}, {t_prop * 1e3:.1f} ms "
            f"(full search {t_full * 1e3:.1f} ms)")
    r = res["window"]
    out = {
        "metric": "effective pairs/s of the proposal search (images x all templates / time), recall of the full "
                  "search's best pose", "value": r["effective_pairs_per_s"], "unit": "pairs/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": r["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 MLP + bf16x3 FTK", "data": "synthetic",
        "config": {"workload": f"{w['name']}: {n_t} 60-blob templates n=128, M=64, Qa=256, N=197 shifts, SNR "
                               f"{w['snr']}; {nc} training images re-noised and relabelled by the two-pass search "
                               f"each of {w['epochs']} epochs ({labelled_pairs} labelled pairs); {kind} features "
                               f"n_r={n_r} n_q={n_q} ({dims[0]} inputs), MLP {dims}; top-{w['topk']}; "
                               f"test {nA} images",
                   "window": res["window"], "no_window": res["no_window"], "tau": tau,
                   "validation_topk_hit": float(hit.mean()), "full_search_pairs_per_s": nA * n_t / t_full,
                   "train_s": train_s, "labelled_pairs_per_s": labelled_pairs / train_s, "generate_s": gen_s,
                   "loss_first_last": [losses[0], losses[-1]],
                   "mlp_forward_ms_b256": ms_fwd, "mlp_forward_tflops": 2.0 * 256 * params / (ms_fwd / 1e3) / 1e12},
        "roofline": {"kernel": "MLP loss + gradients (bf16 MFMA GEMMs), batch 256", "bound": "mfma",
                     "achieved": mlp_flop / (ms_grad / 1e3) / 1e12, "peak": PEAK_BF16_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": mlp_flop / (ms_grad / 1e3) / PEAK_BF16_MFMA, "traffic": None, "ms_per_step": ms_grad},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="cryoem_n128", choices=["cryoem_n128", "ragged", "proposal"],
                    help="cryoem_n128 (default): the headline metric; ragged / proposal: the batch and the "
                         "learned-proposal measurements, each printing its own JSON line")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", default="all",
                    choices=["fp32", "bf16x3", "fp16x3", "fp16", "fp16+bf16x3", "bft", "bfr", "all"],
                    help="the forms to run (bft: brute-force translations alone, its own JSON line)")
    ap.add_argument("--ragged-scale", type=float, default=1.0,
                    help="ragged workload: image and template counts scaled by this (1.0: the full workload)")
    ap.add_argument("--lanes", type=int, default=4, help="ragged workload: concurrent lanes of the batch (1-4)")
    ap.add_argument("--ragged-form", default="fp16x3", choices=["fp32", "bf16x3", "fp16x3", "fp16"],
                    help="ragged workload: the precision form of every stack")
    ap.add_argument("--proposal-features", default="power", choices=sorted(PROPOSAL_FEATURES),
                    help="proposal workload: the network's input features (power: |a(k; q)|^2, 64 radii x 32 modes; "
                         "cross: rotation-invariant cross-ring products; invariant: shift- and rotation-invariant "
                         "ring-power harmonics)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-weighted", action="store_true", help="skip the weighted-SVD measurement")
    ap.add_argument("--no-bft", action="store_true", help="skip the brute-force-translation measurement")
    ap.add_argument("--no-bfr", action="store_true", help="skip the brute-force-rotation measurement")
    ap.add_argument("--no-upsample", action="store_true", help="skip the rotation-upsampling measurement")
    ap.add_argument("--no-ctf", action="store_true", help="skip the joint translation-CTF measurement")
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
        print(f"bench.py: the FTK path runs on one GPU; --gpus {args.gpus} is not supported "
              "(across GPUs the templates would be sharded, each GPU aligning every image against its share, "
              "and the per-image best poses reduced)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(2)
    if args.workload == "ragged":
        return bench_ragged(args)
    if args.workload == "proposal":
        return bench_proposal(args)
    import synth
    w = WORKLOAD
    t = time.perf_counter()
    inputs = make_inputs(w)
    shifts = synth.shift_lattice(w["R"])
    log(f"inputs generated in {time.perf_counter() - t:.1f} s: {w['n_images']} x {w['n_templates']} "
        f"n={w['n']} N={len(shifts)}")
    if args.form == "bft":
        rb = run_form("bft", inputs, w, args.steps, args.warmup, shifts)
        log(f"[bft] {rb['ms_per_step']:.2f} ms/step, {rb['pairs_per_s']:.4g} pairs/s, stages {rb['stages']}")
        print(json.dumps({"metric": "pairs/s of brute-force translations (the paper's comparison method)",
                          "value": rb["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": rb["ms_per_step"], "higher_is_better": True,
                          "dtype": "f32", "data": "synthetic",
                          "config": {"workload": w["name"],
                                     "stage_ms_per_step": {k: v[0] / args.steps for k, v in rb["stages"].items()}}}),
              flush=True)
        return
    if args.form == "bfr":
        # brute-force rotations over the whole workload (a few seconds per step)
        steps, warm = min(args.steps, 3), min(args.warmup, 1)
        rb = run_form("bfr", inputs, w, steps, warm, shifts)
        log(f"[bfr] {rb['ms_per_step']:.2f} ms/step, {rb['pairs_per_s']:.4g} pairs/s, stages {rb['stages']}")
        pairs = w["n_images"] * w["n_templates"]
        fl = bfr_flop_per_pair(w["n"], w["Qa"], shifts)
        corr_ms = rb["stages"]["bfr_correlation"][0] / steps
        achieved = fl * pairs / (corr_ms / 1e3) / 1e12
        print(json.dumps({"metric": "pairs/s of brute-force rotations (the paper's comparison method)",
                          "value": rb["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": steps,
                          "warmup": warm, "ms_per_step": rb["ms_per_step"], "higher_is_better": True,
                          "dtype": "f32", "data": "synthetic",
                          "config": {"workload": w["name"], "rotations": w["Qa"],
                                     "algorithmic_gflop_per_pair": fl / 1e9,
                                     "stage_ms_per_step": {k: v[0] / steps for k, v in rb["stages"].items()}},
                          "roofline": {"kernel": "bfr_corr (FP32 MFMA u sums + y-offset accumulation, argmax)",
                                       "bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_MFMA / 1e12,
                                       "unit": "TFLOP/s", "frac": achieved / (PEAK_FP32_MFMA / 1e12), "traffic": None}}),
              flush=True)
        return
    forms = ["fp32", "bf16x3", "fp16x3", "fp16", "fp16+bf16x3"] if args.form == "all" else [args.form]
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
    # the reported form: the fastest whose per-image best template and pose
    # agree with the FP32 form's (error <= 1e-5 of the pair scale) on at
    # least 99 % of images
    agree = {k: (agreement(v["img_best"], results["fp32"]["img_best"]) if "fp32" in results else None)
             for k, v in results.items()}
    ok = [k for k in results if agree[k] is None or agree[k] >= 0.99]
    chosen = max(ok or list(results), key=lambda k: results[k]["pairs_per_s"])
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
    traffic = measured_traffic("fp16" if chosen == "fp16+bf16x3" else chosen)
    out = {
        "metric": METRIC, "value": r["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3->f32", "fp16x3": "f16x3->f32", "fp16": "f16->f32",
                  "fp16+bf16x3": "f16->f32, top-4 per image refined in bf16x3->f32"}[chosen],
        "data": "synthetic",
        "config": {"workload": f"{w['name']}: {w['n_images']} images x {w['n_templates']} templates, n={w['n']}, "
                               f"60-blob templates, SNR {w['snr']}, M={M}, Qa={Qa} rotations, N={N} shifts "
                               f"(0.5 px lattice, R={w['R']} px), eps={w['eps']}, H={H}",
                   "form": chosen, "pairs": pairs,
                   "forms": {k: {"pairs_per_s": v["pairs_per_s"], "ms_per_step": v["ms_per_step"],
                                 "best_pose_agreement_vs_fp32": agree[k],
                                 "stage_ms_per_step": {s: v["stages"][s][0] / args.steps for s in v["stages"]}}
                             for k, v in results.items()},
                   "form_rule": "fastest form whose per-image best template and pose agree with the FP32 form "
                                "on at least 99 % of images",
                   "speedup_vs_plain_fp32": (r["pairs_per_s"] / results["fp32"]["pairs_per_s"]
                                             if "fp32" in results else None),
                   "recall_true_template": recall(r["img_best"], inputs),
                   "best_pose_agreement_vs_fp32": agree[chosen],
                   "gflop_per_pair": (s1 + s3 + fft) / 1e9},
        "roofline": {"kernel": ("step3 FP16 (shift contraction and rotation transform on MFMA, argmax)"
                                if chosen.startswith("fp16") else
                                "step3 (shift contraction on MFMA + rotation FFT + argmax)"), "bound": "mfma",
                     "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_GBps": traffic / avg3 / 1e9 if traffic and avg3 > 0 else None,
                     "products_per_mac": 3 if chosen in ("bf16x3", "fp16x3") else 1,
                     "frac_of_form_ceiling": (achieved / (peak / 3) if chosen in ("bf16x3", "fp16x3")
                                              else achieved / peak),
                     "algorithmic_flop_per_pair": s3, "pairs_per_launch": per_launch_pairs,
                     "avg_launch_ms": avg3 * 1e3,
                     "step1_achieved": (s1 * pairs * args.steps / max(n1, 1)) / (ms1 / max(n1, 1) / 1e3) / 1e12
                     if ms1 > 0 else None},
    }
    if "fp16" in results and not args.no_weighted:
        # the k-side weighted operator SVD (Section 4.5 remark) with the blob
        # templates' expected power spectrum as weight, at the eps that gives
        # the paper-weighted plan's accuracy against the direct inner product
        # (max error 2.2e-4 vs 2.4e-4 of s_AB on sampled pairs of this
        # workload, oracle computation): about half the SVD terms
        rw = run_form("fp16", inputs, w, args.steps, args.warmup, shifts, eps=WEIGHTED_EPS,
                      weight=synth.blob_power_spectrum())
        log(f"[fp16 weighted] {rw['ms_per_step']:.2f} ms/step, {rw['pairs_per_s']:.4g} pairs/s, H={rw['info']['H']}")
        out["config"]["weighted_svd"] = {
            "form": "fp16", "eps": WEIGHTED_EPS, "H": rw["info"]["H"], "H_paper_weight": H,
            "weight": "expected radial power spectrum of the blob templates (16 Gaussians in k/Kmax)",
            "pairs_per_s": rw["pairs_per_s"], "ms_per_step": rw["ms_per_step"],
            "speedup_vs_paper_weight_fp16": rw["pairs_per_s"] / results["fp16"]["pairs_per_s"],
            "best_pose_agreement_vs_fp32": agreement(rw["img_best"], results["fp32"]["img_best"])
            if "fp32" in results else None,
            "stage_ms_per_step": {k: v[0] / args.steps for k, v in rw["stages"].items()}}
        if "fp16+bf16x3" in results:
            # two-pass form with the weighted plan as its coarse pass and the
            # paper-weighted split-bf16 plan refining each image's best 4
            r2 = run_form("fp16+bf16x3", inputs, w, args.steps, args.warmup, shifts, eps=WEIGHTED_EPS,
                          weight=synth.blob_power_spectrum())
            log(f"[fp16 weighted+bf16x3] {r2['ms_per_step']:.2f} ms/step, {r2['pairs_per_s']:.4g} pairs/s")
            out["config"]["weighted_svd"]["two_pass"] = {
                "pairs_per_s": r2["pairs_per_s"], "ms_per_step": r2["ms_per_step"],
                "speedup_vs_paper_weight_two_pass": r2["pairs_per_s"] / results["fp16+bf16x3"]["pairs_per_s"],
                "best_pose_agreement_vs_fp32": agreement(r2["img_best"], results["fp32"]["img_best"])
                if "fp32" in results else None}
    if not args.no_bft:
        # brute-force translations (Section 6.2) on the same workload, grids
        # and shifts: the paper's FTK-versus-BFT axis on this GPU
        rb = run_form("bft", inputs, w, args.steps, args.warmup, shifts)
        log(f"[bft] {rb['ms_per_step']:.2f} ms/step, {rb['pairs_per_s']:.4g} pairs/s, stages {rb['stages']}")
        qh = Qa // 2 + 1
        out["config"]["bft"] = {
            "pairs_per_s": rb["pairs_per_s"], "ms_per_step": rb["ms_per_step"],
            "stage_ms_per_step": {k: v[0] / args.steps for k, v in rb["stages"].items()},
            "contraction_gflop_per_pair": 8.0 * N * M * qh / 1e9,
            "ftk_contraction_gflop_per_pair": (s1 + s3) / 1e9,
            "ftk_speedup_over_bft": {k: v["pairs_per_s"] / rb["pairs_per_s"] for k, v in results.items()},
            "best_pose_agreement_vs_ftk_fp32": agreement(rb["img_best"], results["fp32"]["img_best"])
            if "fp32" in results else None,
            "recall_true_template": recall(rb["img_best"], inputs)}
    if not args.no_bfr:
        # brute-force rotations (Section 6.1) on a sample of the workload (all
        # images against the first BFR_TEMPLATES templates, so that the
        # template-side spectra keep their share): the paper's FTK-versus-BFR
        # axis on this GPU
        bs = min(args.steps, 2)
        rr = run_form("bfr", inputs, w, bs, 1, shifts, n_templates=BFR_TEMPLATES)
        log(f"[bfr] {rr['ms_per_step']:.2f} ms/step, {rr['pairs_per_s']:.4g} pairs/s, stages {rr['stages']}")
        fl = bfr_flop_per_pair(w["n"], Qa, shifts)
        nbp = w["n_images"] * BFR_TEMPLATES
        corr_s = rr["stages"]["bfr_correlation"][0] / bs / 1e3
        same = None
        if "fp32" in results:
            fp = results["fp32"]["poses"][:, :BFR_TEMPLATES]
            same = float(np.mean((fp["shift"] == rr["poses"]["shift"]) & (fp["rot"] == rr["poses"]["rot"])))
        out["config"]["bfr"] = {
            "sample": f"{w['n_images']} images x {BFR_TEMPLATES} templates",
            "pairs_per_s": rr["pairs_per_s"], "ms_per_step": rr["ms_per_step"],
            "stage_ms_per_step": {k: v[0] / bs for k, v in rr["stages"].items()},
            "algorithmic_gflop_per_pair": fl / 1e9,
            "correlation_tflops": fl * nbp / corr_s / 1e12,
            "ftk_speedup_over_bfr": {k: v["pairs_per_s"] / rr["pairs_per_s"] for k, v in results.items()},
            "pair_pose_agreement_vs_ftk_fp32": same}
    if not args.no_upsample:
        # rotation upsampling (remark after eq. 1dfft) to 5 Qa = 1280 rotations,
        # about the paper's n pi^2 rotation grid, for the split-fp16 form and BFT
        ups = {}
        for f in ("fp16x3", "bft"):
            ru = run_form(f, inputs, w, args.steps, args.warmup, shifts, up=UPSAMPLE)
            log(f"[{f} x{UPSAMPLE} rotations] {ru['ms_per_step']:.2f} ms/step, {ru['pairs_per_s']:.4g} pairs/s")
            ups[f] = {"pairs_per_s": ru["pairs_per_s"], "ms_per_step": ru["ms_per_step"],
                      "stage_ms_per_step": {k: v[0] / args.steps for k, v in ru["stages"].items()}}
        if not args.no_bfr:
            # brute-force rotations at the same rotation count, on the sample
            ru = run_form("bfr", inputs, w, min(args.steps, 2), 1, shifts, up=UPSAMPLE, n_templates=BFR_TEMPLATES)
            log(f"[bfr x{UPSAMPLE} rotations] {ru['ms_per_step']:.2f} ms/step, {ru['pairs_per_s']:.4g} pairs/s")
            ups["bfr"] = {"pairs_per_s": ru["pairs_per_s"], "ms_per_step": ru["ms_per_step"],
                          "sample": f"{w['n_images']} images x {BFR_TEMPLATES} templates",
                          "stage_ms_per_step": {k: v[0] / min(args.steps, 2) for k, v in ru["stages"].items()}}
            ups["ftk_fp16x3_speedup_over_bfr"] = ups["fp16x3"]["pairs_per_s"] / ups["bfr"]["pairs_per_s"]
        ups["rotations"] = UPSAMPLE * Qa
        ups["ftk_fp16x3_speedup_over_bft"] = ups["fp16x3"]["pairs_per_s"] / ups["bft"]["pairs_per_s"]
        out["config"]["upsampled_rotations"] = ups
    if not args.no_ctf and "fp16" in results:
        # joint translation-CTF factorisation (Section 7.1): shifts x 5 defocus
        # values in one alignment, against 5 plain alignments (one per defocus,
        # each the cost of the plain plan) as the alternative
        rc = run_form("fp16", inputs, w, args.steps, args.warmup, shifts, ctf=CTF_PARAMS, defoci=CTF_DEFOCI)
        log(f"[fp16 ctf] {rc['ms_per_step']:.2f} ms/step, {rc['pairs_per_s']:.4g} pairs/s, H={rc['info']['H']}")
        out["config"]["ctf"] = {
            "form": "fp16", "ctf": CTF_PARAMS, "defocus_A": CTF_DEFOCI, "poses": len(shifts) * len(CTF_DEFOCI),
            "H": rc["info"]["H"], "H_plain": H, "pairs_per_s": rc["pairs_per_s"], "ms_per_step": rc["ms_per_step"],
            "time_vs_one_plain_alignment_per_defocus": rc["ms_per_step"] / (len(CTF_DEFOCI) *
                                                                            results["fp16"]["ms_per_step"]),
            "stage_ms_per_step": {k: v[0] / args.steps for k, v in rc["stages"].items()}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inputs, w, shifts)
        if "fp32" in results:
            out["config"]["oracle_best_pose"] = oracle_best_pose(inputs, w, shifts, results, chosen)
            log(f"[oracle check] {out['config']['oracle_best_pose']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
