"""Two-pass alignment (ftk_align_refined): an FP16 pass over every pair, then
the split-bf16 form on each image's k best coarse templates.

The refined pairs must equal the split form's own poses bitwise (list mode
gives the full alignment's values), the other pairs the FP16 poses, and the
per-image best must be the split form's best over the refined list.
"""
import sys

import numpy as np
import pytest

import synth

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


def _topk_host(values, k):
    """k largest values per row, ties to the lower index, NaN last."""
    v = np.where(np.isnan(values), -np.inf, values)
    out = []
    for row in v:
        order = sorted(range(row.size), key=lambda j: (-row[j], j))
        out.append(order[:k])
    return np.array(out)


@pytest.mark.parametrize("k", [1, 4, 17])
def test_refined_matches_both_passes(ftk, k):
    n, M, Qa, R, eps = 64, 32, 128, 2.0, 1e-3
    s = synth.make_alignment_set(21, n, 60, 6, 20, R, 0.05)
    shifts = synth.shift_lattice(R)
    plans = {}
    for f in ("fp16", "bf16x3"):
        P = ftk.Plan(n, M, Qa, R, eps, precision=f)
        P.set_shifts(shifts)
        plans[f] = P
    a = plans["bf16x3"].transform(torch.as_tensor(s.images, dtype=torch.float32, device="cuda"))
    b = plans["bf16x3"].transform(torch.as_tensor(s.templates, dtype=torch.float32, device="cuda"))
    _, coarse = plans["fp16"].align_coeffs(a, b)
    _, fine = plans["bf16x3"].align_coeffs(a, b)
    best, bt, bp = ftk.align_refined(plans["fp16"], plans["bf16x3"], a, b, k)
    torch.cuda.synchronize()
    C, Fn, B = (ftk.poses_numpy(x) for x in (coarse, fine, best))
    bt, bp = bt.cpu().numpy(), bp.cpu().numpy()
    L = _topk_host(C["value"], k)
    same_best = 0
    for i in range(6):
        listed = set(L[i].tolist())
        for j in range(60):
            ref = Fn[i, j] if j in listed else C[i, j]
            assert (B[i, j]["value"], B[i, j]["shift"], B[i, j]["rot"]) == \
                (ref["value"], ref["shift"], ref["rot"]), (k, i, j, j in listed)
        # best over the refined list, ties to the lower template number
        jb = min(L[i], key=lambda j: (-float(Fn[i, j]["value"]), j))
        assert bt[i] == jb
        assert bp[i].view(np.float32)[0] == Fn[i, jb]["value"] and tuple(bp[i][1:]) == (Fn[i, jb]["shift"], Fn[i, jb]["rot"])
        same_best += int(jb == int(np.argmax(Fn[i]["value"])))
    _say(f"[refine k={k}] per-image best equal to the split form's full search on {same_best}/6 images")
    if k >= 4:
        assert same_best == 6


def test_refined_rejects_mismatched_plans(ftk):
    A = ftk.Plan(32, 16, 64, 2.0, 1e-3, precision="fp16")
    B = ftk.Plan(32, 16, 128, 2.0, 1e-3, precision="bf16x3")
    for P in (A, B):
        P.set_shifts(synth.shift_lattice(2.0))
    a = torch.zeros((2, 64, 16), dtype=torch.complex64, device="cuda")
    with pytest.raises(ftk.FTKError):
        ftk.align_refined(A, B, a, a, 1)  # Q differs
    D = ftk.Plan(32, 16, 64, 2.0, 1e-3, precision="bf16x3")
    D.set_shifts(synth.shift_lattice(1.5))
    with pytest.raises(ftk.FTKError):
        ftk.align_refined(A, D, a, a, 1)  # the shift lists differ in length
    C = ftk.Plan(32, 16, 64, 2.0, 1e-3, precision="bf16x3")
    C.set_shifts(synth.shift_lattice(2.0))
    with pytest.raises(ftk.FTKError):
        ftk.align_refined(A, C, a, a, 3)  # k > nB


def test_refined_weighted_coarse_pass(ftk):
    """Coarse pass on a plan with a power-spectrum weighted SVD and a looser
    eps (fewer terms), refinement on the paper's weight: the plans differ in
    H, which the two-pass call allows; the refined pairs still equal the fine
    plan's own poses bitwise and the others the coarse plan's."""
    n, M, Qa, R, k = 64, 32, 128, 2.0, 4
    s = synth.make_alignment_set(23, n, 40, 4, 20, R, 0.05)
    shifts = synth.shift_lattice(R)
    Pc = ftk.Plan(n, M, Qa, R, 5e-3, precision="fp16", weight=synth.blob_power_spectrum())
    Pf = ftk.Plan(n, M, Qa, R, 1e-3, precision="bf16x3")
    for P in (Pc, Pf):
        P.set_shifts(shifts)
    assert Pc.info()["H"] < Pf.info()["H"]
    a = Pf.transform(torch.as_tensor(s.images, dtype=torch.float32, device="cuda"))
    b = Pf.transform(torch.as_tensor(s.templates, dtype=torch.float32, device="cuda"))
    _, coarse = Pc.align_coeffs(a, b)
    _, fine = Pf.align_coeffs(a, b)
    best, bt, bp = ftk.align_refined(Pc, Pf, a, b, k)
    torch.cuda.synchronize()
    C, Fn, B = (ftk.poses_numpy(x) for x in (coarse, fine, best))
    bt = bt.cpu().numpy()
    L = _topk_host(C["value"], k)
    for i in range(4):
        listed = set(L[i].tolist())
        for j in range(40):
            ref = Fn[i, j] if j in listed else C[i, j]
            assert (B[i, j]["value"], B[i, j]["shift"], B[i, j]["rot"]) == \
                (ref["value"], ref["shift"], ref["rot"]), (i, j, j in listed)
        assert bt[i] == min(L[i], key=lambda j: (-float(Fn[i, j]["value"]), j))
    _say(f"[refine weighted] H coarse {Pc.info()['H']} fine {Pf.info()['H']}: "
         f"per-image best equal to the full split search on "
         f"{sum(int(bt[i] == int(np.argmax(Fn[i]['value']))) for i in range(4))}/4 images")
