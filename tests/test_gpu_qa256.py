"""Element-wise parity of the kernel instances the benchmark runs, against the
FP64 oracle.

Shape of the cryo-EM workload: n = 128, M = 64 radial nodes, Qa = 256
rotations (four 32-column tiles of modes in Step 3, the instances with
CTQ = 4), the 197 shifts of a 0.5 px lattice within 4 px and H = 121 > 64 SVD
terms at eps = 1e-3.  Alignment from pixels (ftk_align), as timed.

300 pairs (3 images x 100 templates) put more pairs into one Step 3 launch
than the GPU has compute units, so the persistent Step 3 forms (FP16 and split
bf16: one workgroup per compute unit looping over pairs) run their pair loop
twice and store the next pair's first Zhat chunk during the last chunk of the
current pair.  Whole X arrays [197][256] of pairs taken by the first and by
the second pass of that loop are compared with the oracle.  A second run with
a 16 MiB staging buffer (the images in several chunks, hence several Step 1 /
Step 3 launches) must give the same X and poses bitwise.

One image against 150 templates (FP16): ten 16-template tiles, so the Step 1
wave that takes tiles 0 and 1 also takes tiles 8 and 9 (the last one partial,
6 templates), with the next-tile operand loads clamped past the end; sampled
templates from every such tile against the oracle.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N_IMG, N_TMP = 3, 100
# (image, template): pairs 0, 1, 137, 255 go to the first pass of the
# persistent loop (pair p is taken by workgroup p mod 256), 256, 257, 298, 299
# to the second
PAIRS = [(0, 0), (0, 1), (1, 37), (2, 55), (2, 56), (2, 57), (2, 98), (2, 99)]
# the split-fp16 form is held to 1e-5 here, the bar it claims for any eps
BARS = {"fp32": 1e-5, "bf16x3": 1e-3, "fp16": 1e-3, "fp16x3": 1e-5}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_12317_amd import ftk
    ftk.lib()
    s = synth.make_alignment_set(12, 128, N_TMP, N_IMG, 60, 4.0, 0.05)
    shifts = synth.shift_lattice(4.0)
    plan = O.set_shifts(O.make_plan(128, 64, 256, 4.0, 1e-3), shifts)
    assert plan.H > 64 and len(shifts) == 197
    a = {i: O.fb_coefficients(s.images[i], plan) for i in {p[0] for p in PAIRS}}
    b = {j: O.fb_coefficients(s.templates[j], plan) for j in {p[1] for p in PAIRS}}
    ref = {}
    for i, j in PAIRS:
        ref[(i, j)] = (np.real(O.ftk_X(a[i], b[j], plan)), O.pair_scale(a[i], b[j], plan))
    return ftk, s, shifts, ref


def _align(ftk, s, shifts, form, stage_mib=0):
    P = ftk.Plan(128, 64, 256, 4.0, 1e-3, precision=form)
    P.set_shifts(shifts)
    if stage_mib:
        P.set_tuning(stage_mib=stage_mib)
    dev = torch.device("cuda:0")
    X, best = P.align(torch.as_tensor(s.images, dtype=torch.float32, device=dev),
                      torch.as_tensor(s.templates, dtype=torch.float32, device=dev), want_X=True)
    torch.cuda.synchronize()
    return X.cpu().numpy(), ftk.poses_numpy(best)


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16", "fp16x3"])
def test_benchmark_instances_elementwise(case, form):
    ftk, s, shifts, ref = case
    bar = BARS[form]
    _say(f"[qa256] form={form} n=128 M=64 Qa=256 N=197 pairs={N_IMG * N_TMP} (bar {bar:g} of s_AB)")
    X, poses = _align(ftk, s, shifts, form)
    assert X.shape == (N_IMG, N_TMP, 197, 256)
    assert np.all(np.isfinite(X))
    worst = 0.0
    for i, j in PAIRS:
        Xr, sc = ref[(i, j)]
        err = float(np.max(np.abs(X[i, j] - Xr))) / sc
        worst = max(worst, err)
        v, si, ri, margin = O.best_pose(Xr)
        got = poses[i, j]
        _say(f"  pair {i * N_TMP + j:3d} ({i},{j}): rel err {err:.3e}, margin/scale {margin / sc:.2e}, "
             f"pose ({got['shift']},{got['rot']}) oracle ({si},{ri})")
        assert err <= bar, (i, j, err)
        if margin > 2 * err * sc:
            assert (got["shift"], got["rot"]) == (si, ri), (i, j)
        else:
            assert Xr[got["shift"], got["rot"]] >= v - 2 * err * sc
    _say(f"  worst rel err {worst:.3e}")
    # every pose is the argmax of the X the kernel wrote, its value that maximum
    for i in range(N_IMG):
        for j in range(0, N_TMP, 7):
            v, si, ri, _ = O.best_pose(X[i, j])
            assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (si, ri)
            assert poses[i, j]["value"] == np.float32(v)
    # the images in several chunks: the same results bitwise
    X2, poses2 = _align(ftk, s, shifts, form, stage_mib=16)
    assert np.array_equal(X.view(np.uint32), X2.view(np.uint32))
    for k in ("value", "shift", "rot"):
        assert np.array_equal(poses[k], poses2[k])


def test_fp16_step1_second_tile_pass(case):
    ftk = case[0]
    nB = 150
    s = synth.make_alignment_set(21, 128, nB, 1, 60, 4.0, 0.05)
    shifts = synth.shift_lattice(4.0)
    plan = O.set_shifts(O.make_plan(128, 64, 256, 4.0, 1e-3), shifts)
    _say(f"[qa256] fp16, 1 image x {nB} templates (10 template tiles)")
    X, poses = _align(ftk, s, shifts, "fp16")
    assert X.shape == (1, nB, 197, 256) and np.all(np.isfinite(X))
    a = O.fb_coefficients(s.images[0], plan)
    worst = 0.0
    for j in (0, 17, 40, 127, 128, 135, 143, 144, 149):
        b = O.fb_coefficients(s.templates[j], plan)
        Xr, sc = np.real(O.ftk_X(a, b, plan)), O.pair_scale(a, b, plan)
        err = float(np.max(np.abs(X[0, j] - Xr))) / sc
        worst = max(worst, err)
        assert err <= BARS["fp16"], (j, err)
        v, si, ri, _ = O.best_pose(X[0, j])
        assert (poses[0, j]["shift"], poses[0, j]["rot"]) == (si, ri), j
    _say(f"  worst rel err {worst:.3e} over 9 templates in tiles 0, 1, 2, 7, 8, 9")
