"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Element-by-element on seeded inputs at sizes the oracle finishes in seconds
(several tiles plus ragged tails), with the error of every result stated
relative to the pair scale s_AB = sqrt(X_AA(0,0) X_BB(0,0)), which bounds
|X| on the quadrature.  FP32 bar: rel_err <= 1e-5 per pair.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP32_TOL = 1e-5


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


def _dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _oracle_case(n, M, Qa, R, eps, images, templates, shifts):
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, eps), shifts)
    a = np.array([O.fb_coefficients(x, plan) for x in images])
    b = np.array([O.fb_coefficients(x, plan) for x in templates])
    return plan, a, b


def _ftk_all(plan, a, b):
    return np.array([[np.real(O.ftk_X(ai, bj, plan)) for bj in b] for ai in a])


def _scales(plan, a, b):
    return np.array([[O.pair_scale(ai, bj, plan) for bj in b] for ai in a])


def _rel_errs(X, Xref, S):
    return np.max(np.abs(X - Xref), axis=(2, 3)) / S


# ----------------------------------------------------------------- transform

@pytest.mark.parametrize("n,M,Qa,kind", [(32, 16, 64, "blobs"), (32, 16, 64, "noise"), (64, 32, 128, "noise"),
                                         (96, 48, 192, "blobs"), (128, 64, 256, "blobs")])
def test_transform_matches_oracle(ftk, n, M, Qa, kind):
    _say(f"[transform] n={n} M={M} Qa={Qa} {kind}")
    if kind == "blobs":
        imgs = synth.make_alignment_set(3, n, 3, 2, 20, 2.0, 0.1).templates
    else:
        imgs = synth.white_noise_images(4, 3, n)
    plan = O.make_plan(n, M, Qa, 2.0, 1e-3)
    # oracle rows are rings [M][Qa]; the library stores [Qa][M]
    ref = np.array([O.fb_coefficients(x, plan).T for x in imgs])
    P = ftk.Plan(n, M, Qa, 2.0, 1e-3)
    got = P.transform(_dev(imgs)).cpu().numpy()
    torch.cuda.synchronize()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  max rel coeff err {err:.3e}")
    assert err < 2e-6


@pytest.mark.parametrize("n,M,Qa", [(64, 32, 128), (96, 48, 192), (128, 64, 256), (192, 96, 384), (64, 32, 256)])
def test_transform_repeatable(ftk, n, M, Qa):
    """Regression: the first transform of a fresh plan (scratch never
    written) equals later ones bitwise, in any image order, on the shapes of
    the compile-time kernel (2n = Qa) and a generic one; the workgroups of one
    image must not read its grid before every wave has written it."""
    imgs = synth.white_noise_images(11, 96, n)
    P = ftk.Plan(n, M, Qa, 2.0, 1e-3)
    d = _dev(imgs)
    first = P.transform(d).cpu().numpy()
    again = P.transform(d).cpu().numpy()
    rev = P.transform(torch.flip(d, dims=[0]).contiguous()).cpu().numpy()[::-1]
    torch.cuda.synchronize()
    _say(f"[transform repeat] n={n} Qa={Qa}: first vs again max {np.max(np.abs(first - again)):.3e}")
    assert np.array_equal(first.view(np.uint32), again.view(np.uint32))
    assert np.array_equal(first.view(np.uint32), rev.view(np.uint32))
    if n <= 64:
        plan = O.make_plan(n, M, Qa, 2.0, 1e-3)
        ref = np.array([O.fb_coefficients(x, plan).T for x in imgs[:2]])
        assert np.max(np.abs(first[:2] - ref)) / np.max(np.abs(ref)) < 2e-6


# ------------------------------------------------------------------ alignment

def test_align_from_oracle_coefficients_fp32(ftk):
    """Steps 1-3 + argmax fed the oracle's own coefficients (stage isolated)."""
    n, M, Qa, R, eps = 32, 16, 64, 2.0, 1e-3
    s = synth.workload_set("plain_n32", 1)
    shifts = synth.shift_lattice(R)
    plan, a, b = _oracle_case(n, M, Qa, R, eps, s.images, s.templates, shifts)
    Xref = _ftk_all(plan, a, b)
    S = _scales(plan, a, b)
    _say(f"[align coeffs fp32] nA={a.shape[0]} nB={b.shape[0]} N={len(shifts)} H={plan.H}")
    P = ftk.Plan(n, M, Qa, R, eps)
    P.set_shifts(shifts)
    X, best = P.align_coeffs(_dev(a.transpose(0, 2, 1), torch.complex64),
                             _dev(b.transpose(0, 2, 1), torch.complex64), want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    errs = _rel_errs(X, Xref, S)
    _say(f"  rel err max {errs.max():.3e} median {np.median(errs):.3e}")
    assert errs.max() <= FP32_TOL
    poses = ftk.poses_numpy(best)
    # the pose array must be the argmax of the X the kernel wrote
    for i in range(a.shape[0]):
        for j in range(b.shape[0]):
            v, si, ri, _ = O.best_pose(X[i, j])
            assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (si, ri)
            assert poses[i, j]["value"] == np.float32(v)


def _check_poses(poses, Xref, errs_abs):
    """Best pose identical to the oracle's wherever its margin exceeds twice
    the pair's error; elsewhere the chosen pose must be within that error of
    the oracle's maximum."""
    checked = 0
    for i in range(Xref.shape[0]):
        for j in range(Xref.shape[1]):
            v, si, ri, margin = O.best_pose(Xref[i, j])
            got = poses[i, j]
            if margin > 2 * errs_abs[i, j]:
                assert (got["shift"], got["rot"]) == (si, ri), (i, j)
                checked += 1
            else:
                assert Xref[i, j, got["shift"], got["rot"]] >= v - 2 * errs_abs[i, j]
    return checked


def test_align_end_to_end_fp32_plain_n32(ftk):
    """Pixels to poses on the 4 x 8, n = 32 workload (shifts: 49-point lattice)."""
    n, M, Qa, R, eps = 32, 16, 64, 2.0, 1e-3
    s = synth.workload_set("plain_n32", 1)
    shifts = synth.shift_lattice(R)
    plan, a, b = _oracle_case(n, M, Qa, R, eps, s.images, s.templates, shifts)
    Xref = _ftk_all(plan, a, b)
    S = _scales(plan, a, b)
    _say(f"[align pixels fp32] n={n} nA=4 nB=8")
    P = ftk.Plan(n, M, Qa, R, eps)
    P.set_shifts(shifts)
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    errs = _rel_errs(X, Xref, S)
    _say(f"  rel err max {errs.max():.3e}")
    assert errs.max() <= FP32_TOL
    checked = _check_poses(ftk.poses_numpy(best), Xref, errs * S)
    _say(f"  poses compared exactly: {checked}/32")
    assert checked >= 24


@pytest.mark.parametrize("case", ["ragged", "wide_shift", "n96"])
def test_align_ragged_shapes_fp32(ftk, case):
    """Tails everywhere: template counts off the 32/64 tiles, shift counts
    off the 16-row tiles, H off the 64-term padding, off-lattice shifts."""
    rng = np.random.default_rng(17)
    if case == "ragged":
        n, M, Qa, R, eps, nA, nB = 32, 16, 128, 2.5, 1e-3, 3, 37
        shifts = np.array([synth.area_uniform_disk(rng, R) for _ in range(30)])
    elif case == "wide_shift":
        n, M, Qa, R, eps, nA, nB = 64, 24, 64, 6.0, 1e-2, 2, 70
        shifts = synth.shift_lattice(R, 1.0)
    else:
        n, M, Qa, R, eps, nA, nB = 96, 48, 192, 3.0, 1e-3, 2, 5
        shifts = synth.shift_lattice(R)
    s = synth.make_alignment_set(5, n, nB, nA, 20, min(R, 2.0), 0.1)
    plan, a, b = _oracle_case(n, M, Qa, R, eps, s.images, s.templates, shifts)
    _say(f"[ragged {case}] n={n} M={M} Qa={Qa} H={plan.H} N={len(shifts)} nA={nA} nB={nB}")
    Xref = _ftk_all(plan, a, b)
    S = _scales(plan, a, b)
    P = ftk.Plan(n, M, Qa, R, eps)
    P.set_shifts(shifts)
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    errs = _rel_errs(X.cpu().numpy(), Xref, S)
    _say(f"  rel err max {errs.max():.3e}")
    assert errs.max() <= FP32_TOL
    _check_poses(ftk.poses_numpy(best), Xref, errs * S)


def test_degenerate_inputs(ftk):
    n, M, Qa, R = 32, 16, 64, 2.0
    P = ftk.Plan(n, M, Qa, R, 1e-3)
    img = _dev(synth.white_noise_images(1, 2, n))
    # align before set_shifts is a state error
    with pytest.raises(ftk.FTKError) as e:
        P.align(img, img)
    assert e.value.code == -5
    # a shift outside the planned disk is rejected
    with pytest.raises(ftk.FTKError) as e:
        P.set_shifts(np.array([[2.5, 0.0]]))
    assert e.value.code == -4
    # a single zero shift: X(0, r) must equal the direct polar inner product
    P.set_shifts(np.zeros((1, 2)))
    X, best = P.align(img, img, want_X=True)
    empty = torch.empty((0, n, n), device="cuda")
    P.align(empty, img)  # nA = 0 is a no-op
    torch.cuda.synchronize()
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, 1e-3), np.zeros((1, 2)))
    imgs = img.cpu().numpy().astype(np.float64)
    Ah = [O.polar_ft(x, plan.k, Qa) for x in imgs]
    for i in range(2):
        for j in range(2):
            Xd = np.real(O.direct_X(Ah[i], Ah[j], plan.k, plan.w, np.zeros((1, 2)), n))
            a_, b_ = O.ring_coefficients(Ah[i]), O.ring_coefficients(Ah[j])
            sc = O.pair_scale(a_, b_, plan)
            assert np.max(np.abs(X[i, j].cpu().numpy() - Xd)) / sc < 2 * plan.eps
    # self-alignment peaks at zero shift and zero rotation
    poses = ftk.poses_numpy(best)
    for i in range(2):
        assert (poses[i, i]["shift"], poses[i, i]["rot"]) == (0, 0)


# ------------------------------------------------------- split-bf16 form

@pytest.mark.parametrize("eps", [1e-3, pytest.param(1e-5, marks=pytest.mark.xfail(
    reason="a two-term bf16 split keeps about 16 bits per product; its error, about 1e-5 of the pair "
           "scale, sits at this eps", strict=False))])
def test_align_bf16x3_against_fp64_oracle(ftk, eps):
    """Split-bf16 form (3 products, FP32 accumulation) on the n = 32
    workload; its error against the FP64 oracle is stated for every pair.
    Bar: rel_err <= eps (the truncation level the plan was built for)."""
    n, M, Qa, R = 32, 16, 64, 2.0
    s = synth.workload_set("plain_n32", 1)
    shifts = synth.shift_lattice(R)
    plan, a, b = _oracle_case(n, M, Qa, R, eps, s.images, s.templates, shifts)
    Xref = _ftk_all(plan, a, b)
    S = _scales(plan, a, b)
    _say(f"[bf16x3] eps={eps} H={plan.H}")
    P = ftk.Plan(n, M, Qa, R, eps, precision="bf16x3")
    P.set_shifts(shifts)
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    errs = _rel_errs(X.cpu().numpy(), Xref, S)
    _say(f"  rel err per pair: max {errs.max():.3e} median {np.median(errs):.3e} min {errs.min():.3e}")
    assert errs.max() <= eps
    checked = _check_poses(ftk.poses_numpy(best), Xref, errs * S)
    _say(f"  poses compared exactly: {checked}/32")


@pytest.mark.parametrize("case", ["ragged", "n96"])
def test_align_bf16x3_ragged(ftk, case):
    rng = np.random.default_rng(23)
    if case == "ragged":
        n, M, Qa, R, eps, nA, nB = 32, 16, 128, 2.5, 1e-3, 3, 37
        shifts = np.array([synth.area_uniform_disk(rng, R) for _ in range(30)])
    else:
        n, M, Qa, R, eps, nA, nB = 96, 48, 192, 3.0, 1e-3, 2, 5
        shifts = synth.shift_lattice(R)
    s = synth.make_alignment_set(6, n, nB, nA, 20, min(R, 2.0), 0.1)
    plan, a, b = _oracle_case(n, M, Qa, R, eps, s.images, s.templates, shifts)
    _say(f"[bf16x3 ragged {case}] H={plan.H} N={len(shifts)} nA={nA} nB={nB}")
    Xref = _ftk_all(plan, a, b)
    S = _scales(plan, a, b)
    P = ftk.Plan(n, M, Qa, R, eps, precision="bf16x3")
    P.set_shifts(shifts)
    X, best = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    errs = _rel_errs(X.cpu().numpy(), Xref, S)
    _say(f"  rel err max {errs.max():.3e}")
    assert errs.max() <= eps
    _check_poses(ftk.poses_numpy(best), Xref, errs * S)
