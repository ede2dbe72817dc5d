"""The benchmark's own configuration at full size, checked on samples.

512 images x 2048 templates, n = 128, 197 shifts, 256 rotations, eps = 1e-3,
in the launch configuration bench.py times (ftk_align from pixels, best
poses only).  The full X is far too large to compare, so sampled pairs are
recomputed one by one by the FP64 oracle: the best value must match within
the pair's error bar and the pose must match wherever the oracle's margin
exceeds twice that bar.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_12317_amd import ftk
    ftk.lib()
    s = synth.make_alignment_set(2, 128, 2048, 512, 60, 4.0, 0.05)
    shifts = synth.shift_lattice(4.0)
    plan = O.set_shifts(O.make_plan(128, 64, 256, 4.0, 1e-3), shifts)
    return ftk, s, shifts, plan


@pytest.mark.parametrize("form,tol", [("fp32", 1e-5), ("bf16x3", 1e-3), ("fp16", 1e-3), ("fp16x3", 1e-5)])
def test_full_size_sampled_pairs(setup, form, tol):
    ftk, s, shifts, plan = setup
    print(f"[bench shape] form={form} 512x2048 n=128 N=197", flush=True)
    P = ftk.Plan(128, 64, 256, 4.0, 1e-3, precision=form)
    P.set_shifts(shifts)
    dev = torch.device("cuda:0")
    imgs = torch.as_tensor(s.images, dtype=torch.float32, device=dev)
    tmps = torch.as_tensor(s.templates, dtype=torch.float32, device=dev)
    _, best = P.align(imgs, tmps)
    torch.cuda.synchronize()
    poses = ftk.poses_numpy(best)
    assert np.all(poses["shift"] >= 0) and np.all(poses["shift"] < 197)
    assert np.all(poses["rot"] >= 0) and np.all(poses["rot"] < 256)
    rng = np.random.default_rng(5)
    pairs = [(int(i), int(s.true_template[i])) for i in rng.choice(512, 3, replace=False)]
    pairs += [(int(i), int(j)) for i, j in zip(rng.choice(512, 3), rng.choice(2048, 3))]
    worst = 0.0
    for i, j in pairs:
        a = O.fb_coefficients(s.images[i], plan)
        b = O.fb_coefficients(s.templates[j], plan)
        X = np.real(O.ftk_X(a, b, plan))
        sc = O.pair_scale(a, b, plan)
        v, si, ri, margin = O.best_pose(X)
        got = poses[i, j]
        err = abs(float(got["value"]) - v) / sc
        worst = max(worst, err)
        # the value the GPU chose must be what the oracle has at that pose
        err_at = abs(float(got["value"]) - X[got["shift"], got["rot"]]) / sc
        print(f"  pair ({i},{j}): best err {err:.2e}, at-pose err {err_at:.2e}, margin/scale {margin / sc:.2e}",
              flush=True)
        assert err_at <= tol
        if margin > 2 * tol * sc:
            assert (got["shift"], got["rot"]) == (si, ri)
        else:
            assert X[got["shift"], got["rot"]] >= v - 2 * tol * sc
    assert worst <= tol
    sys.stdout.flush()


def test_headline_per_image_best_against_oracle(setup):
    """The benchmark's reported answer, per image, against the FP64 oracle.

    On 32 seeded images of the full workload: every template whose FP32 best
    value lies within twice the FP32 error bound of the image's FP32 best
    (the only templates that can hold the image's true best, given FP32's
    1e-5 bar) is recomputed by the oracle, with the two-pass form's pick.  The
    oracle's per-image best (template, shift, rotation) must equal the FP32
    form's and the two-pass form's wherever its margin over every other
    candidate pose (and over the bound of every non-candidate template)
    exceeds twice the form's error."""
    ftk, s, shifts, plan = setup
    dev = torch.device("cuda:0")
    imgs = torch.as_tensor(s.images, dtype=torch.float32, device=dev)
    tmps = torch.as_tensor(s.templates, dtype=torch.float32, device=dev)
    P32 = ftk.Plan(128, 64, 256, 4.0, 1e-3, precision="fp32")
    P32.set_shifts(shifts)
    _, b32 = P32.align(imgs, tmps)
    P16 = ftk.Plan(128, 64, 256, 4.0, 1e-3, precision="fp16")
    P16.set_shifts(shifts)
    Pbf = ftk.Plan(128, 64, 256, 4.0, 1e-3, precision="bf16x3")
    Pbf.set_shifts(shifts)
    ca, cb = P16.transform(imgs), P16.transform(tmps)
    _, bt, bp = ftk.align_refined(P16, Pbf, ca, cb, 4)
    torch.cuda.synchronize()
    v32 = ftk.poses_numpy(b32)
    two_t = bt.cpu().numpy().astype(np.int64)
    two_p = ftk.poses_numpy(bp)
    rng = np.random.default_rng(17)
    sample = np.sort(rng.choice(512, 32, replace=False))
    bcache = {}

    def bco(j):
        if j not in bcache:
            bcache[j] = O.fb_coefficients(s.templates[j], plan)
        return bcache[j]

    SB = 2.0 * 2.0 * np.pi  # >= sqrt(X_BB(0,0)) of a unit-L2 template (checked on every candidate)
    rows = []
    for i in sample:
        a = O.fb_coefficients(s.images[i], plan)
        sA = np.sqrt(O.pair_scale(a, a, plan))
        e32 = 1e-5 * sA * SB
        vals = v32["value"][i].astype(np.float64)
        cand = set(np.nonzero(vals >= vals.max() - 2 * e32)[0].tolist()) | {int(two_t[i])}
        outside = [vals[j] for j in range(vals.size) if j not in cand]
        bound_out = (max(outside) + e32) if outside else -np.inf
        best = None
        seconds = [bound_out]
        Xs = {}
        for j in sorted(cand):
            b = bco(j)
            assert np.sqrt(O.pair_scale(b, b, plan)) <= SB
            X = np.real(O.ftk_X(a, b, plan))
            Xs[j] = (X, O.pair_scale(a, b, plan))
            v, si, ri, margin = O.best_pose(X)
            if best is None or v > best[0]:
                if best is not None:
                    seconds.append(best[0])
                best = (v, j, si, ri, margin)
            else:
                seconds.append(v)
        v, j, si, ri, margin = best
        margin = min(margin, v - max(seconds))
        sc = Xs[j][1]
        # FP32 form: its per-image best is the argmax of its values
        j32 = int(np.argmax(vals))
        same32 = (j32, int(v32["shift"][i, j32]), int(v32["rot"][i, j32])) == (j, si, ri)
        # two-pass form: its value at its own pick against the oracle there
        X2, sc2 = Xs[int(two_t[i])]
        err2 = abs(float(two_p["value"][i]) - X2[two_p["shift"][i], two_p["rot"][i]]) / sc2
        same2 = (int(two_t[i]), int(two_p["shift"][i]), int(two_p["rot"][i])) == (j, si, ri)
        rows.append((i, len(cand), margin / sc, err2, same32, same2))
        print(f"  image {i:3d}: {len(cand)} candidate(s), oracle best t={j} ({si},{ri}) margin/scale "
              f"{margin / sc:.2e}; fp32 {'=' if same32 else '!='}, two-pass {'=' if same2 else '!='} "
              f"(err at its pick {err2:.2e})", flush=True)
        if margin > 2 * 1e-5 * sc:
            assert same32, i
        assert err2 <= 1e-3
        if margin > 2 * 1e-3 * sc:
            assert same2, i
    err_max = max(r[3] for r in rows)
    agree32 = np.mean([r[4] for r in rows])
    agree2 = np.mean([r[5] for r in rows])
    print(f"  oracle per-image best recovered: fp32 {agree32:.3f}, two-pass {agree2:.3f}; two-pass err max "
          f"{err_max:.2e}", flush=True)
    # the two-pass form's measured error decides the rest: same answer
    # wherever the margin exceeds twice it
    for (i, nc, m, e, s32, s2) in rows:
        if m > 2 * max(err_max, 1e-5):
            assert s2, i
    assert agree2 >= 0.99 or all(r[5] or r[2] <= 2 * max(err_max, 1e-5) for r in rows)
