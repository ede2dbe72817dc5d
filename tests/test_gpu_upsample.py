"""GPU parity of rotation upsampling (ftk_plan_set_rotations; the remark
after eq. 1dfft): X on U Qa rotations against the oracle's zero-padded
angular sum, element by element, for the FTK forms that support it (FP32,
split bf16, split fp16) and for brute-force translations.

Bars: FP32 and split fp16 1e-5, split bf16 eps, of the pair scale s_AB; the
best pose equal to the oracle's wherever its margin exceeds twice the error.
Also: every U-th rotation of the upsampled X equals the plain alignment's X
to rounding, U = 1 restores the plain result bitwise, the benchmark's shape
at U = 5 (1280 rotations, about the paper's n pi^2) on sampled pairs, the
FP16 form refuses, and a batch runs an upsampled plan.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BARS = {"fp32": 1e-5, "bf16x3": 1e-3, "fp16x3": 1e-5}


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


def _check(X, poses, ref, scale, bar, tag):
    worst = 0.0
    for (i, j), Xr in ref.items():
        err = float(np.max(np.abs(X[i, j] - Xr))) / scale[(i, j)]
        worst = max(worst, err)
        assert err <= bar, (tag, i, j, err)
        v, si, ri, margin = O.best_pose(Xr)
        got = poses[i, j]
        if margin > 2 * err * scale[(i, j)]:
            assert (got["shift"], got["rot"]) == (si, ri), (tag, i, j)
        else:
            assert Xr[got["shift"], got["rot"]] >= v - 2 * err * scale[(i, j)]
        v2, s2, r2, _ = O.best_pose(X[i, j])
        assert (got["shift"], got["rot"]) == (s2, r2)
    return worst


@pytest.mark.parametrize("form,U", [("fp32", 3), ("bf16x3", 2), ("fp16x3", 4)])
def test_ftk_upsampled_small(ftk, form, U):
    n, M, Qa, R, eps = 32, 16, 64, 2.0, 1e-3
    s = synth.workload_set("plain_n32", 1)
    shifts = synth.shift_lattice(R)
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, eps), shifts)
    a = [O.fb_coefficients(x, plan) for x in s.images]
    b = [O.fb_coefficients(x, plan) for x in s.templates]
    pairs = [(0, 0), (1, 3), (2, 5), (3, 7)]
    ref = {(i, j): np.real(O.ftk_X_upsampled(a[i], b[j], plan, U)) for i, j in pairs}
    scale = {(i, j): O.pair_scale(a[i], b[j], plan) for i, j in pairs}
    P = ftk.Plan(n, M, Qa, R, eps, precision=form)
    P.set_shifts(shifts)
    X1, _ = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    P.set_rotations(U)
    assert P.info()["rotations"] == U * Qa
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    X, X1 = X.cpu().numpy(), X1.cpu().numpy()
    assert X.shape == (4, 8, len(shifts), U * Qa)
    poses = ftk.poses_numpy(best)
    worst = _check(X, poses, ref, scale, BARS[form], form)
    # every U-th rotation is the plain rotation grid
    d = float(np.max(np.abs(X[:, :, :, ::U] - X1)))
    _say(f"[upsample] form={form} U={U}: worst rel err {worst:.3e}; coarse-grid difference {d:.2e}")
    assert d <= 1e-5 * float(np.max(np.abs(X1)))
    # U = 1 again: the plain kernels, bitwise
    P.set_rotations(1)
    X2, _ = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    assert np.array_equal(X2.cpu().numpy().view(np.uint32), X1.view(np.uint32))


def test_bft_upsampled(ftk):
    n, M, Qa, R, U = 48, 24, 128, 1.5, 3
    s = synth.make_alignment_set(41, n, 9, 3, 12, R, 0.1)
    shifts = synth.shift_lattice(R)
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, 1e-3), shifts)
    pairs = [(0, 0), (1, 4), (2, 8)]
    Ah = {i: O.polar_ft(s.images[i], plan.k, Qa) for i in range(3)}
    bb = {j: O.ring_coefficients(O.polar_ft(s.templates[j], plan.k, Qa)) for j in (0, 4, 8)}
    ref = {(i, j): np.real(O.bft_X_upsampled(Ah[i], bb[j], plan, U)) for i, j in pairs}
    scale = {(i, j): O.pair_scale(O.ring_coefficients(Ah[i]), bb[j], plan) for i, j in pairs}
    P = ftk.Plan(n, M, Qa, R, 1e-3)
    P.set_shifts(shifts)
    P.set_rotations(U)
    X, best = P.bft_align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    worst = _check(X.cpu().numpy(), ftk.poses_numpy(best), ref, scale, 1e-5, "bft")
    _say(f"[upsample] bft U={U}: worst rel err {worst:.3e}")


def test_benchmark_shape_u5(ftk):
    """n = 128, M = 64, Qa = 256, 197 shifts, U = 5: 1280 rotations; the
    split-fp16 form on 2 x 40 pairs, sampled pairs against the oracle."""
    n, M, Qa, R, eps, U = 128, 64, 256, 4.0, 1e-3, 5
    s = synth.make_alignment_set(12, n, 40, 2, 60, R, 0.05)
    shifts = synth.shift_lattice(R)
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, eps), shifts)
    pairs = [(0, 0), (1, 39)]
    a = {i: O.fb_coefficients(s.images[i], plan) for i in (0, 1)}
    b = {j: O.fb_coefficients(s.templates[j], plan) for j in (0, 39)}
    ref = {(i, j): np.real(O.ftk_X_upsampled(a[i], b[j], plan, U)) for i, j in pairs}
    scale = {(i, j): O.pair_scale(a[i], b[j], plan) for i, j in pairs}
    P = ftk.Plan(n, M, Qa, R, eps, precision="fp16x3")
    P.set_shifts(shifts)
    P.set_rotations(U)
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    worst = _check(X.cpu().numpy(), ftk.poses_numpy(best), ref, scale, 1e-5, "fp16x3 u5")
    _say(f"[upsample] benchmark shape U={U} fp16x3: worst rel err {worst:.3e}")


def test_fp16_form_refuses(ftk):
    P = ftk.Plan(32, 16, 64, 2.0, 1e-3, precision="fp16")
    P.set_shifts(synth.shift_lattice(2.0))
    P.set_rotations(2)
    x = torch.zeros((1, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(ftk.FTKError):
        P.align(x, x)
    with pytest.raises(ftk.FTKError):
        P.set_rotations(0)


def test_batch_with_upsampled_plan(ftk):
    n, M, Qa, R, U = 32, 16, 64, 2.0, 2
    s = synth.workload_set("plain_n32", 3)
    shifts = synth.shift_lattice(R)
    P = ftk.Plan(n, M, Qa, R, 1e-3, precision="bf16x3")
    P.set_shifts(shifts)
    P.set_rotations(U)
    ref = P.align(_dev(s.images), _dev(s.templates))[1]
    imgs, tmps = _dev(s.images), _dev(s.templates)
    best = torch.empty((imgs.shape[0], tmps.shape[0], 3), dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    B = ftk.Batch([{"plan": P, "images": imgs, "templates": tmps, "best": best}], lanes=1, graph=True,
                  stream=stream)
    for _ in range(3):
        best.fill_(-1)
        torch.cuda.synchronize()
        B.run(stream)
        stream.synchronize()
        assert torch.equal(best, ref)
        assert int(best[..., 2].max()) < U * Qa
