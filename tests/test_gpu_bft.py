"""GPU parity of brute-force translations (ftk_bft_align, Section 6.2 of the
paper) against the oracle's BFT, which equals the direct polar inner product
(no SVD) to rounding.

FP32 bar as everywhere: max |X - X_ref| <= 1e-5 of the pair scale s_AB,
element by element, with the best pose equal to the oracle's wherever its
margin exceeds twice the pair's error.  Cases: the small n = 32 workload;
ragged counts (templates and shifts not multiples of the tiles) at Qa = 128
and 192; the benchmark's shape (n = 128, M = 64, Qa = 256, 197 shifts) on
sampled pairs; Qa = 384; chunked staging bitwise equal; and BFT poses against
the FP32 FTK's where both are decided.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-5


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


def _run(ftk, n, M, Qa, R, images, templates, shifts, stage_mib=0, precision="fp32"):
    P = ftk.Plan(n, M, Qa, R, 1e-3, precision=precision)
    P.set_shifts(shifts)
    if stage_mib:
        P.set_tuning(stage_mib=stage_mib)
    X, best = P.bft_align(_dev(images), _dev(templates), want_X=True)
    torch.cuda.synchronize()
    return X.cpu().numpy(), ftk.poses_numpy(best)


def _check(X, poses, images, templates, pairs, n, M, Qa, R, shifts):
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, 1e-3), shifts)
    Ah = {i: O.polar_ft(images[i], plan.k, Qa) for i in {p[0] for p in pairs}}
    Bh = {j: O.polar_ft(templates[j], plan.k, Qa) for j in {p[1] for p in pairs}}
    worst, decided = 0.0, 0
    for i, j in pairs:
        b = O.ring_coefficients(Bh[j])
        Xr = np.real(O.bft_translations_X(Ah[i], b, plan))
        sc = O.pair_scale(O.ring_coefficients(Ah[i]), b, plan)
        err = float(np.max(np.abs(X[i, j] - Xr))) / sc
        worst = max(worst, err)
        assert err <= TOL, (i, j, err)
        v, si, ri, margin = O.best_pose(Xr)
        got = poses[i, j]
        if margin > 2 * err * sc:
            assert (got["shift"], got["rot"]) == (si, ri), (i, j)
            decided += 1
        else:
            assert Xr[got["shift"], got["rot"]] >= v - 2 * err * sc
    # every pose is the argmax of the X the kernels wrote
    for i, j in pairs:
        v, si, ri, _ = O.best_pose(X[i, j])
        assert (poses[i, j]["shift"], poses[i, j]["rot"]) == (si, ri)
        assert poses[i, j]["value"] == np.float32(v)
    return worst, decided


def test_bft_small_workload(ftk):
    n, M, Qa, R = 32, 16, 64, 2.0
    s = synth.workload_set("plain_n32", 1)
    shifts = synth.shift_lattice(R)
    _say(f"[bft] n={n} M={M} Qa={Qa} N={len(shifts)} pairs={len(s.images)}x{len(s.templates)}")
    X, poses = _run(ftk, n, M, Qa, R, s.images, s.templates, shifts)
    assert X.shape == (len(s.images), len(s.templates), len(shifts), Qa) and np.all(np.isfinite(X))
    pairs = [(i, j) for i in range(len(s.images)) for j in range(len(s.templates))]
    worst, decided = _check(X, poses, s.images, s.templates, pairs, n, M, Qa, R, shifts)
    _say(f"  worst rel err {worst:.3e}, poses decided {decided}/{len(pairs)}")


@pytest.mark.parametrize("Qa,R", [(128, 1.5), (192, 2.5)])
def test_bft_ragged(ftk, Qa, R):
    n, M, nA, nB = 48, 24, 3, 19
    s = synth.make_alignment_set(41, n, nB, nA, 12, R, 0.1)
    shifts = synth.shift_lattice(R)
    _say(f"[bft ragged] n={n} M={M} Qa={Qa} N={len(shifts)} pairs={nA}x{nB}")
    X, poses = _run(ftk, n, M, Qa, R, s.images, s.templates, shifts)
    pairs = [(0, 0), (0, 18), (1, 7), (2, 16), (2, 18)]
    worst, decided = _check(X, poses, s.images, s.templates, pairs, n, M, Qa, R, shifts)
    _say(f"  worst rel err {worst:.3e}, poses decided {decided}/{len(pairs)}")


def test_bft_qa384(ftk):
    n, M, Qa, R = 32, 16, 384, 1.0
    s = synth.workload_set("plain_n32", 2)
    shifts = synth.shift_lattice(R)
    _say(f"[bft] n={n} M={M} Qa={Qa} N={len(shifts)}")
    X, poses = _run(ftk, n, M, Qa, R, s.images[:2], s.templates[:3], shifts)
    worst, _ = _check(X, poses, s.images[:2], s.templates[:3], [(0, 0), (1, 2)], n, M, Qa, R, shifts)
    _say(f"  worst rel err {worst:.3e}")


def test_bft_benchmark_shape_and_chunks(ftk):
    """n = 128, M = 64, Qa = 256, 197 shifts (224 padded): 3 x 100 pairs,
    sampled pairs against the oracle; a 16 MiB staging (one image per
    chunk) gives bitwise the same X and poses."""
    n, M, Qa, R = 128, 64, 256, 4.0
    s = synth.make_alignment_set(12, n, 100, 3, 60, R, 0.05)
    shifts = synth.shift_lattice(R)
    assert len(shifts) == 197
    _say(f"[bft] n={n} M={M} Qa={Qa} N=197 pairs=3x100")
    X, poses = _run(ftk, n, M, Qa, R, s.images, s.templates, shifts)
    worst, decided = _check(X, poses, s.images, s.templates, [(0, 0), (1, 37), (2, 99)], n, M, Qa, R, shifts)
    _say(f"  worst rel err {worst:.3e}, poses decided {decided}/3")
    X2, poses2 = _run(ftk, n, M, Qa, R, s.images, s.templates, shifts, stage_mib=16)
    assert np.array_equal(X.view(np.uint32), X2.view(np.uint32))
    for k in ("value", "shift", "rot"):
        assert np.array_equal(poses[k], poses2[k])


def test_bft_against_ftk_fp32(ftk):
    """Both methods compute the same inner products up to the SVD truncation
    (eps = 1e-3 of the operator) and rounding: poses agree wherever the FTK
    margin exceeds twice the difference of the two X arrays."""
    n, M, Qa, R = 64, 32, 128, 2.0
    s = synth.make_alignment_set(21, n, 24, 4, 20, R, 0.05)
    shifts = synth.shift_lattice(R)
    P = ftk.Plan(n, M, Qa, R, 1e-3)
    P.set_shifts(shifts)
    Xf, bf = P.align(_dev(s.images), _dev(s.templates), want_X=True)
    Xb, bb = P.bft_align(_dev(s.images), _dev(s.templates), want_X=True)
    torch.cuda.synchronize()
    Xf, Xb = Xf.cpu().numpy(), Xb.cpu().numpy()
    pf, pb = ftk.poses_numpy(bf), ftk.poses_numpy(bb)
    same = checked = 0
    for i in range(Xf.shape[0]):
        for j in range(Xf.shape[1]):
            d = float(np.max(np.abs(Xf[i, j] - Xb[i, j])))
            _, _, _, margin = O.best_pose(Xf[i, j])
            if margin > 2 * d:
                checked += 1
                assert (pf[i, j]["shift"], pf[i, j]["rot"]) == (pb[i, j]["shift"], pb[i, j]["rot"]), (i, j)
            same += int((pf[i, j]["shift"], pf[i, j]["rot"]) == (pb[i, j]["shift"], pb[i, j]["rot"]))
    _say(f"[bft vs ftk fp32] same pose {same}/{Xf.shape[0] * Xf.shape[1]}, decided {checked}")
    assert checked > 0
