"""GPU parity of the FP16 form (one fp16 product per term, FP32 accumulation,
power-of-two scales per call and per SVD term) against the FP64 oracle.

Bar, as for every reduced-precision form: rel_err <= eps of the pair scale
s_AB = sqrt(X_AA(0,0) X_BB(0,0)) on every pair, and the oracle's best pose
wherever its margin exceeds twice the pair's error.  The error of every
result is printed.
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


def _oracle(n, M, Qa, R, eps, images, templates, shifts):
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, eps), shifts)
    a = np.array([O.fb_coefficients(x, plan) for x in images])
    b = np.array([O.fb_coefficients(x, plan) for x in templates])
    Xref = np.array([[np.real(O.ftk_X(ai, bj, plan)) for bj in b] for ai in a])
    S = np.array([[O.pair_scale(ai, bj, plan) for bj in b] for ai in a])
    return plan, a, b, Xref, S


def _check_poses(poses, Xref, errs_abs):
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


def _run(ftk, n, M, Qa, R, eps, images, templates, shifts, tag):
    plan, a, b, Xref, S = _oracle(n, M, Qa, R, eps, images, templates, shifts)
    _say(f"[fp16 {tag}] n={n} Qa={Qa} eps={eps} H={plan.H} N={len(shifts)} nA={len(images)} nB={len(templates)}")
    P = ftk.Plan(n, M, Qa, R, eps, precision="fp16")
    P.set_shifts(shifts)
    X, best = P.align(_dev(images), _dev(templates), want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    errs = np.max(np.abs(X - Xref), axis=(2, 3)) / S
    _say(f"  rel err per pair: max {errs.max():.3e} median {np.median(errs):.3e} min {errs.min():.3e}")
    return X, ftk.poses_numpy(best), Xref, errs, S


@pytest.mark.parametrize("eps", [1e-3, pytest.param(1e-5, marks=pytest.mark.xfail(
    reason="one fp16 product keeps about 11 bits per operand; its error, a few 1e-4 of the pair scale, "
           "is above this eps", strict=False))])
def test_align_fp16_against_fp64_oracle(ftk, eps):
    n, M, Qa, R = 32, 16, 64, 2.0
    s = synth.workload_set("plain_n32", 1)
    X, poses, Xref, errs, S = _run(ftk, n, M, Qa, R, eps, s.images, s.templates, synth.shift_lattice(R), "plain_n32")
    assert errs.max() <= eps
    checked = _check_poses(poses, Xref, errs * S)
    _say(f"  poses compared exactly: {checked}/32")
    # the pose values are the maxima of the X the kernel wrote
    for i in range(X.shape[0]):
        for j in range(X.shape[1]):
            v, si, ri, _ = O.best_pose(X[i, j])
            assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (si, ri)
            assert poses[i, j]["value"] == np.float32(v)


@pytest.mark.parametrize("case", ["ragged", "n96", "noise", "qa384"])
def test_align_fp16_shapes(ftk, case):
    """Ragged tails (37 templates, 30 off-lattice shifts), n = 96 / Qa = 192,
    white-noise images and templates, and Qa = 384 (six column tiles)."""
    rng = np.random.default_rng(29)
    if case == "ragged":
        n, M, Qa, R, eps, nA, nB = 32, 16, 128, 2.5, 1e-3, 3, 37
        shifts = np.array([synth.area_uniform_disk(rng, R) for _ in range(30)])
    elif case == "n96":
        n, M, Qa, R, eps, nA, nB = 96, 48, 192, 3.0, 1e-3, 2, 5
        shifts = synth.shift_lattice(R)
    elif case == "noise":
        n, M, Qa, R, eps, nA, nB = 32, 16, 64, 2.0, 1e-3, 3, 4
        shifts = synth.shift_lattice(R)
    else:
        n, M, Qa, R, eps, nA, nB = 64, 32, 384, 2.0, 1e-3, 2, 3
        shifts = synth.shift_lattice(R)
    if case == "noise":
        images = synth.white_noise_images(31, nA, n)
        templates = synth.white_noise_images(32, nB, n)
    else:
        st = synth.make_alignment_set(6, n, nB, nA, 20, min(R, 2.0), 0.1)
        images, templates = st.images, st.templates
    X, poses, Xref, errs, S = _run(ftk, n, M, Qa, R, eps, images, templates, shifts, case)
    assert errs.max() <= eps
    _check_poses(poses, Xref, errs * S)


def test_align_fp16_input_scale(ftk):
    """The data scales are powers of two taken from the inputs: images x 2^13
    and templates x 2^-9 give exactly 2^4 times the X and pose values and the
    same poses; images x 1e4 stay within eps of 1e4 times the result."""
    n, M, Qa, R, eps = 32, 16, 64, 2.0, 1e-3
    s = synth.workload_set("plain_n32", 2)
    shifts = synth.shift_lattice(R)
    P = ftk.Plan(n, M, Qa, R, eps, precision="fp16")
    P.set_shifts(shifts)
    X0, b0 = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    X1, b1 = P.align(_dev(s.images * 2.0 ** 13), _dev(s.templates * 2.0 ** -9), want_X=True)
    X2, b2 = P.align(_dev(s.images * 1e4), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    X0, X1, X2 = (x.cpu().numpy() for x in (X0, X1, X2))
    p0, p1 = ftk.poses_numpy(b0), ftk.poses_numpy(b1)
    _say(f"[fp16 scale] max |X1 - 16 X0| = {np.max(np.abs(X1 - 16.0 * X0)):.3e}")
    assert np.array_equal(X1, 16.0 * X0)
    assert np.array_equal(p1["shift"], p0["shift"]) and np.array_equal(p1["rot"], p0["rot"])
    assert np.array_equal(p1["value"], 16.0 * p0["value"])
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, eps), shifts)
    a = [O.fb_coefficients(x, plan) for x in s.images]
    b = [O.fb_coefficients(x, plan) for x in s.templates]
    S = np.array([[O.pair_scale(ai, bj, plan) for bj in b] for ai in a])
    rel = np.max(np.abs(X2 - 1e4 * X0), axis=(2, 3)) / (1e4 * S)
    _say(f"  x 1e4: max rel difference {rel.max():.3e}")
    assert rel.max() <= eps


def test_data_scales_unaligned_coefficients(ftk):
    """The per-call data scales (max |a|, max |b| over the coefficients) are
    read with 16-byte loads where the coefficients are 16-byte aligned and
    one by one otherwise: coefficients 8 bytes off that alignment give bitwise
    the same X and poses in both fp16 forms."""
    n, M, Qa, R = 32, 16, 64, 2.0
    st = synth.make_alignment_set(5, n, 7, 3, 20, R, 0.1)
    shifts = synth.shift_lattice(R)

    def offset_copy(t):
        buf = torch.empty(t.numel() + 1, dtype=t.dtype, device=t.device)
        v = buf[1:].view(t.shape)
        v.copy_(t)
        return v

    for prec in ("fp16", "fp16x3"):
        P = ftk.Plan(n, M, Qa, R, 1e-3, precision=prec)
        P.set_shifts(shifts)
        a, b = P.transform(_dev(st.images)), P.transform(_dev(st.templates))
        X0, b0 = P.align_coeffs(a, b, want_X=True)
        a1, b1 = offset_copy(a), offset_copy(b)
        assert a.data_ptr() % 16 == 0 and a1.data_ptr() % 16 == 8 and b1.data_ptr() % 16 == 8
        X1, bb1 = P.align_coeffs(a1, b1, want_X=True)
        torch.cuda.synchronize()
        assert torch.equal(X0.view(torch.int32), X1.view(torch.int32)), prec
        assert torch.equal(b0, bb1), prec


@pytest.mark.parametrize("nshift,nA,nB", [(49, 20, 20), (460, 12, 10)])
def test_persistent_loop_with_idle_slots(ftk, nshift, nA, nB):
    """More (pair, shift block) units than compute units, so the persistent
    Step 3 loops over units, and shift slots without tiles: 49 lattice shifts
    give 4 tiles for 7 compute waves; 460 shifts give three shift blocks, the
    last with one tile, and a workgroup's units change shift block.  A wave
    idle in one unit and busy in the next must multiply the next unit's shift
    panel.  Every pair against the oracle."""
    n, M, Qa, R, eps = 32, 16, 64, 2.0, 1e-3
    rng = np.random.default_rng(11)
    shifts = (synth.shift_lattice(R) if nshift == 49
              else np.array([synth.area_uniform_disk(rng, R) for _ in range(nshift)]))
    assert len(shifts) == nshift
    st = synth.make_alignment_set(17, n, nB, nA, 20, R, 0.1)
    X, poses, Xref, errs, S = _run(ftk, n, M, Qa, R, eps, st.images, st.templates, shifts, f"loop N={nshift}")
    assert errs.max() <= eps
    _check_poses(poses, Xref, errs * S)
    # the best-pose-only kernel (no X written) on the same inputs: bitwise the same poses
    P = ftk.Plan(n, M, Qa, R, eps, precision="fp16")
    P.set_shifts(shifts)
    _, b2 = P.align(_dev(st.images), _dev(st.templates))
    torch.cuda.synchronize()
    p2 = ftk.poses_numpy(b2)
    for k in ("value", "shift", "rot"):
        assert np.array_equal(poses[k], p2[k]), k


@pytest.mark.parametrize("n,M,Qa,R,nshift", [(32, 16, 64, 2.0, 49), (64, 32, 128, 3.0, 0), (128, 64, 256, 4.0, 0),
                                             (128, 64, 256, 8.0, 0), (32, 16, 128, 2.5, 30)])
def test_poses_without_X_equal_poses_with_X(ftk, n, M, Qa, R, nshift):
    """The best-pose-only kernel (argmax per quad of rotations, the winning
    quad recomputed) gives bitwise the poses of the kernel that writes every
    X and compares every element: same values, same (shift, rotation), ties
    to the lowest index.  Blob pairs, white noise against itself and against
    its copy rotated by 90 degrees; 797 shifts (several shift blocks per pair)
    and 30 off-lattice shifts (a partial tile) included."""
    rng = np.random.default_rng(7 + n + Qa)
    shifts = (np.array([synth.area_uniform_disk(rng, R) for _ in range(nshift)]) if nshift
              else synth.shift_lattice(R))
    st = synth.make_alignment_set(9, n, 37, 5, 20, min(R, 2.0), 0.1)
    noise = synth.white_noise_images(33, 3, n)
    images = np.concatenate([st.images, noise, np.rot90(noise, 1, axes=(1, 2))])
    templates = np.concatenate([st.templates, noise])
    P = ftk.Plan(n, M, Qa, R, 1e-3, precision="fp16")
    P.set_shifts(shifts)
    _say(f"[fp16 poses] n={n} Qa={Qa} N={len(shifts)} nA={len(images)} nB={len(templates)}")
    X, b1 = P.align(_dev(images), _dev(templates), want_X=True)
    _, b2 = P.align(_dev(images), _dev(templates))
    torch.cuda.synchronize()
    p1, p2 = ftk.poses_numpy(b1), ftk.poses_numpy(b2)
    for k in ("value", "shift", "rot"):
        assert np.array_equal(p1[k], p2[k]), k
