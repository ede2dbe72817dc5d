"""GPU parity of the split-fp16 form (FTK_FP16X3: hi + lo fp16 operands,
three products hi.hi + hi.lo + lo.hi per term, FP32 accumulation, on the
power-of-two scaled operands of the FP16 form) against the FP64 oracle.

Bar: rel_err <= eps of the pair scale s_AB on every pair at eps = 1e-3 and at
eps = 1e-5 (the accuracy form of the precision workload), and the oracle's
best pose wherever its margin exceeds twice the pair's error.  The error of
every pair is printed.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def _run(ftk, n, M, Qa, R, eps, images, templates, shifts, tag):
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, eps), shifts)
    a = [O.fb_coefficients(x, plan) for x in images]
    b = [O.fb_coefficients(x, plan) for x in templates]
    Xref = np.array([[np.real(O.ftk_X(ai, bj, plan)) for bj in b] for ai in a])
    S = np.array([[O.pair_scale(ai, bj, plan) for bj in b] for ai in a])
    _say(f"[fp16x3 {tag}] n={n} Qa={Qa} eps={eps} H={plan.H} N={len(shifts)} nA={len(images)} nB={len(templates)}")
    P = ftk.Plan(n, M, Qa, R, eps, precision="fp16x3")
    P.set_shifts(shifts)
    X, best = P.align(_dev(images), _dev(templates), want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    errs = np.max(np.abs(X - Xref), axis=(2, 3)) / S
    for i in range(errs.shape[0]):
        _say("  rel err image %d: %s" % (i, " ".join(f"{e:.2e}" for e in errs[i])))
    _say(f"  rel err max {errs.max():.3e} median {np.median(errs):.3e}")
    poses = ftk.poses_numpy(best)
    checked = 0
    for i in range(Xref.shape[0]):
        for j in range(Xref.shape[1]):
            v, si, ri, margin = O.best_pose(Xref[i, j])
            got = poses[i, j]
            if margin > 2 * errs[i, j] * S[i, j]:
                assert (got["shift"], got["rot"]) == (si, ri), (i, j)
                checked += 1
            else:
                assert Xref[i, j, got["shift"], got["rot"]] >= v - 2 * errs[i, j] * S[i, j]
            # the pose is the argmax of the X the kernel wrote, its value that maximum
            vx, sx, rx, _ = O.best_pose(X[i, j])
            assert (got["shift"], got["rot"]) == (sx, rx)
            assert got["value"] == np.float32(vx)
    _say(f"  poses compared exactly: {checked}/{errs.size}")
    return errs


@pytest.mark.parametrize("eps", [1e-3, 1e-5])
def test_align_fp16x3_against_fp64_oracle(ftk, eps):
    n, M, Qa, R = 32, 16, 64, 2.0
    s = synth.workload_set("plain_n32", 1)
    errs = _run(ftk, n, M, Qa, R, eps, s.images, s.templates, synth.shift_lattice(R), "plain_n32")
    assert errs.max() <= eps


@pytest.mark.parametrize("case", ["ragged", "n96", "noise", "qa384", "qa256"])
def test_align_fp16x3_shapes_eps_1e5(ftk, case):
    """At eps = 1e-5: ragged tails (37 templates, 30 off-lattice shifts),
    n = 96 / Qa = 192, white-noise images and templates (a flat spectrum: no
    small high-frequency coefficients to hide rounding), Qa = 384, and the
    n = 128 / Qa = 256 shape of the cryo-EM workload."""
    rng = np.random.default_rng(41)
    eps = 1e-5
    if case == "ragged":
        n, M, Qa, R, nA, nB = 32, 16, 128, 2.5, 3, 37
        shifts = np.array([synth.area_uniform_disk(rng, R) for _ in range(30)])
    elif case == "n96":
        n, M, Qa, R, nA, nB = 96, 48, 192, 3.0, 2, 5
        shifts = synth.shift_lattice(R)
    elif case == "noise":
        n, M, Qa, R, nA, nB = 32, 16, 64, 2.0, 3, 4
        shifts = synth.shift_lattice(R)
    elif case == "qa384":
        n, M, Qa, R, nA, nB = 64, 32, 384, 2.0, 2, 3
        shifts = synth.shift_lattice(R)
    else:
        n, M, Qa, R, nA, nB = 128, 64, 256, 4.0, 2, 3
        shifts = synth.shift_lattice(R)
    if case == "noise":
        images = synth.white_noise_images(31, nA, n)
        templates = synth.white_noise_images(32, nB, n)
    else:
        st = synth.make_alignment_set(6, n, nB, nA, 20 if n < 128 else 60, min(R, 2.0), 0.1)
        images, templates = st.images, st.templates
    errs = _run(ftk, n, M, Qa, R, eps, images, templates, shifts, case)
    assert errs.max() <= eps


def test_align_fp16x3_input_scale(ftk):
    """The data scales are powers of two taken from the inputs: images x 2^13
    and templates x 2^-9 give exactly 2^4 times the X and pose values and the
    same poses."""
    n, M, Qa, R, eps = 32, 16, 64, 2.0, 1e-5
    s = synth.workload_set("plain_n32", 2)
    P = ftk.Plan(n, M, Qa, R, eps, precision="fp16x3")
    P.set_shifts(synth.shift_lattice(R))
    X0, b0 = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    X1, b1 = P.align(_dev(s.images * 2.0 ** 13), _dev(s.templates * 2.0 ** -9), want_X=True)
    torch.cuda.synchronize()
    X0, X1 = X0.cpu().numpy(), X1.cpu().numpy()
    p0, p1 = ftk.poses_numpy(b0), ftk.poses_numpy(b1)
    _say(f"[fp16x3 scale] max |X1 - 16 X0| = {np.max(np.abs(X1 - 16.0 * X0)):.3e}")
    assert np.array_equal(X1, 16.0 * X0)
    assert np.array_equal(p1["shift"], p0["shift"]) and np.array_equal(p1["rot"], p0["rot"])
    assert np.array_equal(p1["value"], 16.0 * p0["value"])
