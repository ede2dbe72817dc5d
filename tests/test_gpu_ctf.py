"""GPU parity of plans with the joint translation-CTF factorisation
(ftk_plan_create_ctf / ftk_set_poses, Section 7.1) against the oracle's FTK
with the same factorisation, element by element over (pose, rotation), and
the best pose (shift, defocus, rotation) against the oracle's wherever its
margin exceeds twice the pair's error.  Bars as everywhere: FP32 and split
fp16 1e-5, split bf16 and FP16 eps, of the pair scale s_AB.

Poses are a product grid of shifts and defocus values; the oracle's
factorisation is pinned (tests/test_oracle_ctf.py) to the direct inner
product with the CTF-filtered image.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ctf as C
from oracle import ftk as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CTFD = dict(wavelength_A=0.019687, cs_mm=2.7, amplitude_contrast=0.07, pixel_A=2.0,
            defocus_min_A=14000.0, defocus_max_A=16000.0)
CM = C.CtfModel(0.019687, 2.7, 0.07, 2.0)
BARS = {"fp32": 1e-5, "bf16x3": 1e-3, "fp16x3": 1e-5, "fp16": 1e-3}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ftk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_12317_amd import ftk as F
    F.lib()  # raises if the library is missing: no fallback
    return F


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def _poses(R, defoci):
    sh = synth.shift_lattice(R)
    return np.repeat(sh, len(defoci), axis=0), np.tile(np.asarray(defoci, dtype=np.float64), len(sh))


@pytest.fixture(scope="module")
def small():
    n, M, Qa, R = 32, 16, 64, 2.0
    s = synth.workload_set("plain_n32", 1)
    sh, df = _poses(R, [14000.0, 14750.0, 15500.0, 16000.0])
    plan = C.set_poses(C.make_ctf_plan(n, M, Qa, R, 1e-3, CM, 14000.0, 16000.0), sh, df)
    a = [O.fb_coefficients(x, plan) for x in s.images]
    b = [O.fb_coefficients(x, plan) for x in s.templates]
    return n, M, Qa, R, s, sh, df, plan, a, b


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16x3", "fp16"])
def test_ctf_plan_small(ftk, small, form):
    n, M, Qa, R, s, sh, df, plan, a, b = small
    P = ftk.Plan(n, M, Qa, R, 1e-3, precision=form, ctf=CTFD)
    P.set_poses(sh, df)
    inf = P.info()
    assert inf["ctf"] == 1 and inf["H"] == plan.H and inf["N"] == len(sh)
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    poses = ftk.poses_numpy(best)
    worst, decided = 0.0, 0
    for i in range(len(s.images)):
        for j in range(len(s.templates)):
            Xr = np.real(O.ftk_X(a[i], b[j], plan))
            sc = O.pair_scale(a[i], b[j], plan)
            err = float(np.max(np.abs(X[i, j] - Xr))) / sc
            worst = max(worst, err)
            v, si, ri, margin = O.best_pose(Xr)
            got = poses[i, j]
            if margin > 2 * err * sc:
                assert (got["shift"], got["rot"]) == (si, ri), (i, j)
                decided += 1
            else:
                assert Xr[got["shift"], got["rot"]] >= v - 2 * err * sc
    _say(f"[ctf] form={form} H={plan.H} poses={len(sh)}: worst rel err {worst:.3e}, decided {decided}/32")
    assert worst <= BARS[form]


def test_ctf_plan_benchmark_shape(ftk):
    """n = 128, M = 64, Qa = 256, 197 shifts x 3 defocus values (H = 296 >
    256 SVD terms), split fp16, sampled pairs against the oracle."""
    n, M, Qa, R = 128, 64, 256, 4.0
    s = synth.make_alignment_set(12, n, 30, 2, 60, R, 0.05)
    sh, df = _poses(R, [14000.0, 15000.0, 16000.0])
    plan = C.set_poses(C.make_ctf_plan(n, M, Qa, R, 1e-3, CM, 14000.0, 16000.0), sh, df)
    P = ftk.Plan(n, M, Qa, R, 1e-3, precision="fp16x3", ctf=CTFD)
    P.set_poses(sh, df)
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    poses = ftk.poses_numpy(best)
    worst = 0.0
    for i, j in [(0, 0), (1, 29)]:
        a = O.fb_coefficients(s.images[i], plan)
        b = O.fb_coefficients(s.templates[j], plan)
        Xr = np.real(O.ftk_X(a, b, plan))
        sc = O.pair_scale(a, b, plan)
        err = float(np.max(np.abs(X[i, j] - Xr))) / sc
        worst = max(worst, err)
        v, si, ri, margin = O.best_pose(Xr)
        if margin > 2 * err * sc:
            assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (si, ri)
    _say(f"[ctf] benchmark shape H={plan.H} poses={len(sh)}: worst rel err {worst:.3e}")
    assert worst <= 1e-5


def test_ctf_plan_refuses_plain_calls(ftk):
    P = ftk.Plan(32, 16, 64, 2.0, 1e-3, ctf=CTFD)
    with pytest.raises(ftk.FTKError):
        P.set_shifts(synth.shift_lattice(2.0))
    sh, df = _poses(2.0, [15000.0])
    P.set_poses(sh, df)
    x = torch.zeros((1, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(ftk.FTKError):
        P.bft_align(x, x)
    with pytest.raises(ftk.FTKError):
        P.set_poses(sh, np.full(len(sh), 20000.0))
