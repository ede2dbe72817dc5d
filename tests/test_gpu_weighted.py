"""GPU parity of plans with a k-side weighted operator SVD (Section 4.5,
the remark on alternative weight functions; ftk_plan_create_weighted)
against the oracle's FTK with the same weighted factorisation.

The kernels are those of every plan; only the factor tables change (and H
drops).  Bars as everywhere: FP32 1e-5, reduced precision eps, of the pair
scale s_AB, element by element, with the best pose equal wherever the
oracle's margin exceeds twice the pair's error.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

WEIGHT = synth.blob_power_spectrum()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ftk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_12317_amd import ftk as F
    F.lib()
    return F


@pytest.mark.parametrize("shape,form,bar", [("n32", "fp32", 1e-5), ("n32", "fp16x3", 1e-5), ("n128", "fp32", 1e-5),
                                            ("n128", "fp16", 1e-3)])
def test_weighted_plan_against_oracle(ftk, shape, form, bar):
    if shape == "n32":
        n, M, Qa, R, eps, nA, nB, snr, nb = 32, 16, 64, 2.0, 1e-3, 4, 8, 0.1, 20
    else:
        n, M, Qa, R, eps, nA, nB, snr, nb = 128, 64, 256, 4.0, 1e-3, 2, 3, 0.05, 60
    s = synth.make_alignment_set(31, n, nB, nA, nb, R, snr)
    shifts = synth.shift_lattice(R)
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, eps, weight=WEIGHT), shifts)
    a = [O.fb_coefficients(x, plan) for x in s.images]
    b = [O.fb_coefficients(x, plan) for x in s.templates]
    P = ftk.Plan(n, M, Qa, R, eps, precision=form, weight=WEIGHT)
    P.set_shifts(shifts)
    inf = P.info()
    assert inf["weighted"] == 1 and inf["H"] == plan.H
    _say(f"[weighted] {shape} form={form} H={plan.H} (paper weight: {O.make_plan(n, M, Qa, R, eps).H})")
    dev = torch.device("cuda:0")
    X, best = P.align(torch.as_tensor(s.images, dtype=torch.float32, device=dev),
                      torch.as_tensor(s.templates, dtype=torch.float32, device=dev), want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    poses = ftk.poses_numpy(best)
    worst = 0.0
    for i in range(nA):
        for j in range(nB):
            Xr = np.real(O.ftk_X(a[i], b[j], plan))
            sc = O.pair_scale(a[i], b[j], plan)
            err = float(np.max(np.abs(X[i, j] - Xr))) / sc
            worst = max(worst, err)
            v, si, ri, margin = O.best_pose(Xr)
            got = poses[i, j]
            if margin > 2 * err * sc:
                assert (got["shift"], got["rot"]) == (si, ri), (i, j)
            else:
                assert Xr[got["shift"], got["rot"]] >= v - 2 * err * sc
    _say(f"  worst rel err {worst:.3e} (bar {bar:g})")
    assert worst <= bar
