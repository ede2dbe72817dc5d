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


@pytest.mark.parametrize("form,tol", [("fp32", 1e-5), ("bf16x3", 1e-3), ("fp16", 1e-3)])
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
