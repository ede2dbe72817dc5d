"""GPU parity of brute-force rotations (ftk_bfr_align, Section 6.1,
eq. 2dconv) with the oracle's BFR (oracle/bfr.py), element by element over
(shift, rotation), FP32 bar 1e-5 of s_AB; best poses against the oracle's
wherever the margin exceeds twice the pair's error, and equal to the argmax
of the X the call wrote.

Shapes: n = 32 / Qa = 64 over the 2 px lattice; n = 96 / Qa = 192; n = 64 / Qa = 128 with 70
images (two row tiles, ragged), off-lattice and repeated shifts (two passes
of y offsets, a shift listed twice); the benchmark shape n = 128 / Qa = 256
/ 197 shifts on sampled rotations; upsampled rotations (R = 2 Qa); template
chunks bitwise equal to one chunk; refusals.
"""
import math
import sys

import numpy as np
import pytest

import synth
from oracle import bfr as BR
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


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32, device="cuda")


def _run(ftk, n, Qa, R, images, templates, shifts, stage_mib=0, up=1):
    P = ftk.Plan(n, n // 2, Qa, R, 1e-3)
    P.set_shifts(shifts)
    if up > 1:
        P.set_rotations(up)
    if stage_mib:
        P.set_tuning(stage_mib=stage_mib)
    X, best = P.bfr_align(_dev(images), _dev(templates), want_X=True)
    torch.cuda.synchronize()
    return X.cpu().numpy(), ftk.poses_numpy(best)


def _scale(A, B, n):
    # sqrt(X_AA(0, 0) X_BB(0, 0)) of the method itself
    u, v = BR.cartesian_grid(n)
    a = BR.ft_at(A, math.pi * u, math.pi * v)
    b = BR.ft_at(B, math.pi * u, math.pi * v)
    return math.pi ** 2 * math.sqrt(float(np.sum(np.abs(a) ** 2)) * float(np.sum(np.abs(b) ** 2)))


def _check_pairs(X, poses, images, templates, shifts, R, pairs, rots=None, tag=""):
    n = images.shape[1]
    worst, decided = 0.0, 0
    spec = {}
    for i, j in pairs:
        if j not in spec:
            spec[j] = BR.rotated_spectra(templates[j], R, rots)
        u, v = BR.cartesian_grid(n)
        a = BR.ft_at(images[i], math.pi * u, math.pi * v)
        Xr = np.real(BR.bfr_X_spectra(a, spec[j], n, shifts))
        sc = _scale(images[i], templates[j], n)
        got = X[i, j] if rots is None else X[i, j][:, rots]
        err = float(np.max(np.abs(got - Xr))) / sc
        worst = max(worst, err)
        # the pose is the argmax of the X the call wrote (ties to the lower index)
        k = int(np.argmax(X[i, j]))
        assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (k // X.shape[3], k % X.shape[3]), (i, j)
        assert poses[i, j]["value"] == np.float32(X[i, j].reshape(-1)[k])
        if rots is None:
            vbest, si, ri, margin = O.best_pose(Xr)
            if margin > 2 * err * sc:
                assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (si, ri), (i, j)
                decided += 1
    _say(f"[bfr] {tag}: worst rel err {worst:.3e} over {len(pairs)} pairs, poses decided {decided}")
    return worst


def test_bfr_small(ftk):
    n, Qa, R = 32, 64, 2.0
    s = synth.workload_set("plain_n32", 1)
    shifts = synth.shift_lattice(R)
    X, poses = _run(ftk, n, Qa, R, s.images, s.templates, shifts)
    assert X.shape == (len(s.images), len(s.templates), len(shifts), Qa)
    pairs = [(i, j) for i in range(len(s.images)) for j in range(len(s.templates))]
    assert _check_pairs(X, poses, s.images, s.templates, shifts, Qa, pairs, tag="n=32") <= 1e-5


def test_bfr_n96(ftk):
    # n = 96 (fine grid 192, rows of 100 values), Qa = 192 rotations
    n, Qa, R = 96, 192, 2.5
    s = synth.make_alignment_set(8, n, 3, 5, 30, R, 0.1)
    shifts = synth.shift_lattice(R)
    X, poses = _run(ftk, n, Qa, R, s.images, s.templates, shifts)
    pairs = [(0, 0), (3, 2), (4, 1)]
    assert _check_pairs(X, poses, s.images, s.templates, shifts, Qa, pairs, rots=[0, 7, 48, 150], tag="n=96") <= 1e-5


def test_bfr_template_chunks(ftk):
    # 2.3 MB of spectra per template at n = 64, Qa = 128: 16 MiB holds 7 of 9
    n, Qa, R = 64, 128, 2.0
    s = synth.make_alignment_set(5, n, 9, 5, 20, R, 0.1)
    shifts = synth.shift_lattice(R)
    X, poses = _run(ftk, n, Qa, R, s.images, s.templates, shifts)
    X2, poses2 = _run(ftk, n, Qa, R, s.images, s.templates, shifts, stage_mib=16)
    assert np.array_equal(X, X2) and np.array_equal(poses, poses2)


def test_bfr_ragged_rows_and_irregular_shifts(ftk):
    n, Qa, R = 64, 128, 3.0
    rng = np.random.default_rng(4)
    s = synth.make_alignment_set(21, n, 3, 70, 20, R, 0.1)
    lat = synth.shift_lattice(R)
    extra = rng.uniform(-2.0, 2.0, size=(6, 2))  # six more y offsets: 19 > 17, two passes
    shifts = np.concatenate([lat, extra, lat[5:6]])  # and lattice shift 5 listed twice
    X, poses = _run(ftk, n, Qa, R, s.images, s.templates, shifts)
    assert np.array_equal(X[:, :, 5], X[:, :, -1])
    pairs = [(i, 0) for i in (0, 1, 37, 63, 64, 69)] + [(12, 1), (68, 2)]
    assert _check_pairs(X, poses, s.images, s.templates, shifts, Qa, pairs, tag="n=64 ragged") <= 1e-5
    # every pair's pose is its own X's argmax (the duplicate never wins over index 5)
    for i in range(70):
        for j in range(3):
            k = int(np.argmax(X[i, j]))
            assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (k // Qa, k % Qa)


def test_bfr_benchmark_shape_sampled(ftk):
    n, Qa, R = 128, 256, 4.0
    s = synth.make_alignment_set(12, n, 4, 66, 60, R, 0.05)
    shifts = synth.shift_lattice(R)
    X, poses = _run(ftk, n, Qa, R, s.images, s.templates, shifts)
    rots = [0, 37, 128, 201]
    pairs = [(0, 0), (65, 3), (40, 1)]
    assert _check_pairs(X, poses, s.images, s.templates, shifts, Qa, pairs, rots=rots, tag="n=128") <= 1e-5
    # the pose of every pair is its X's argmax
    flat = X.reshape(X.shape[0], X.shape[1], -1)
    k = np.argmax(flat, axis=2)
    assert np.array_equal(poses["shift"], k // Qa) and np.array_equal(poses["rot"], k % Qa)


def test_bfr_upsampled_rotations(ftk):
    n, Qa, R, up = 32, 64, 2.0, 2
    s = synth.workload_set("plain_n32", 1)
    shifts = synth.shift_lattice(R)
    X, poses = _run(ftk, n, Qa, R, s.images[:2], s.templates[:3], shifts, up=up)
    assert X.shape[3] == up * Qa
    pairs = [(0, 0), (1, 2)]
    assert _check_pairs(X, poses, s.images[:2], s.templates[:3], shifts, up * Qa, pairs, tag="R = 2 Qa") <= 1e-5
    # the even rotations are the plain call's
    Xp, _ = _run(ftk, n, Qa, R, s.images[:2], s.templates[:3], shifts)
    assert np.max(np.abs(X[..., ::2] - Xp)) <= 1e-6 * np.max(np.abs(Xp))


def test_bfr_degenerate_inputs(ftk):
    import ctypes
    n, Qa, R = 32, 64, 2.0
    P = ftk.Plan(n, n // 2, Qa, R, 1e-3)
    P.set_shifts(np.array([[0.5, -1.0]]))  # one shift: one x and one y offset
    s = synth.workload_set("plain_n32", 1)
    X, poses = P.bfr_align(_dev(s.images[:3]), _dev(s.templates[:2]), want_X=True)
    torch.cuda.synchronize()
    X, poses = X.cpu().numpy(), ftk.poses_numpy(poses)
    u, v = BR.cartesian_grid(n)
    for i, j in [(0, 0), (2, 1)]:
        a = BR.ft_at(s.images[i], math.pi * u, math.pi * v)
        Xr = np.real(BR.bfr_X_spectra(a, BR.rotated_spectra(s.templates[j], Qa), n, [[0.5, -1.0]]))
        assert np.max(np.abs(X[i, j] - Xr)) <= 1e-5 * _scale(s.images[i], s.templates[j], n)
        assert poses[i, j]["shift"] == 0 and poses[i, j]["rot"] == int(np.argmax(X[i, j, 0]))
    # empty calls do nothing and succeed; both outputs NULL is an error
    L = ftk.lib()
    x = _dev(s.images[:1])
    assert L.ftk_bfr_align(P._h, ctypes.c_void_p(x.data_ptr()), 0, ctypes.c_void_p(x.data_ptr()), 1, None, None,
                           None) == 0
    assert L.ftk_bfr_align(P._h, ctypes.c_void_p(x.data_ptr()), 1, ctypes.c_void_p(x.data_ptr()), 0, None, None,
                           None) == 0
    assert L.ftk_bfr_align(P._h, ctypes.c_void_p(x.data_ptr()), 1, ctypes.c_void_p(x.data_ptr()), 1, None, None,
                           None) != 0


def test_bfr_refusals(ftk):
    P = ftk.Plan(32, 16, 64, 2.0, 1e-3)
    x = torch.zeros((1, 32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(ftk.FTKError):  # no shifts yet
        P.bfr_align(x, x)
    ctf = dict(wavelength_A=0.019687, cs_mm=2.7, amplitude_contrast=0.07, pixel_A=2.0,
               defocus_min_A=14000.0, defocus_max_A=16000.0)
    C = ftk.Plan(32, 16, 64, 2.0, 1e-3, ctf=ctf)
    C.set_poses(synth.shift_lattice(2.0), np.full(49, 15000.0))
    with pytest.raises(ftk.FTKError):
        C.bfr_align(x, x)
