"""GPU: the proposal's restricted search over a shift window (an annulus of
the predicted shift radius; ftk_plan_set_shift_windows + ftk_align_proposed)
equals the full search on its own pairs.

For every image at or above the confidence threshold the returned template
and pose must be the best, over its proposed templates and the shifts of its
window only, of the full alignment's X (bitwise: in the split-bf16 form each
shift's value does not depend on which other shifts share its tile); images
below the threshold must get the full search's best over all templates and
shifts.  The network is untrained (its proposals are arbitrary, which is all
this equality needs).
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
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_12317_amd import ftk as F
    from paper_1905_12317_amd import proposal as PR
    F.lib()
    return F, PR


def test_window_search_equals_full_search_on_its_pairs(lib):
    F, PR = lib
    n, M, Qa, R, topk = 64, 32, 128, 2.0, 4
    n_t, nA = 24, 40
    s = synth.make_alignment_set(33, n, n_t, nA, 20, R, 0.1)
    shifts = synth.shift_lattice(R)
    bins = PR.shift_bins(shifts)
    n_s = int(bins.max()) + 1
    centers = 0.5 * np.arange(n_s)
    plan = F.Plan(n, M, Qa, R, 1e-3, "bf16x3")
    plan.set_shifts(shifts)
    plan.set_shift_windows(centers, 0.5)
    imgs = torch.as_tensor(s.images, dtype=torch.float32, device="cuda")
    tc = plan.transform(torch.as_tensor(s.templates, dtype=torch.float32, device="cuda"))
    ic = plan.transform(imgs)
    kind, n_r, n_q = "power", 16, 8
    dims = [F.feature_count(kind, n_r, n_q), 64, n_t + n_s]
    net = F.MLP(dims, n_t, n_s, "bf16", max_batch=64)
    net.set_params(synth.mlp_init(9, dims))
    feats = F.features(plan, ic, n_r, n_q, kind=kind)
    top, mass, sbin = net.propose(feats, topk)
    top, mass, sbin = top.cpu().numpy(), mass.cpu().numpy(), sbin.cpu().numpy()
    tau = float(np.median(mass))
    bt, bp, fb, nfb = F.align_proposed(plan, net, imgs, tc, n_r, n_q, topk, tau, kind=kind)
    X, _ = plan.align_coeffs(ic, tc, want_X=True)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    bt, bp, fb = bt.cpu().numpy(), bp.cpu().numpy(), fb.cpu().numpy()
    radius = np.hypot(shifts[:, 0], shifts[:, 1])
    restricted = 0
    for i in range(nA):
        if mass[i] < tau:
            cand_t, cand_d = np.arange(n_t), np.arange(len(shifts))
            assert fb[i] == 1
        else:
            cand_t = top[i]
            cand_d = np.where(np.abs(radius - centers[sbin[i]]) <= 0.5 * (1 + 1e-12))[0]
            assert fb[i] == 0
            restricted += 1
        # best over the candidates: per template the first maximum over
        # (shift, rotation) in plan order, then the largest value, ties to the
        # lower template number
        best = None
        for t in sorted(cand_t):
            sub = X[i, t][cand_d]
            k = int(np.argmax(sub))
            v = sub.reshape(-1)[k]
            d, r = int(cand_d[k // Qa]), k % Qa
            if best is None or v > best[0]:
                best = (v, t, d, r)
        v, t, d, r = best
        assert bt[i] == t, (i, bt[i], t)
        assert (bp[i][1], bp[i][2]) == (d, r), (i, tuple(bp[i][1:]), (d, r))
        assert bp[i].view(np.float32)[0] == np.float32(v)
    _say(f"[shift window] {restricted}/{nA} images searched over their window, {nfb} in full")
    assert 0 < restricted < nA


def test_window_arguments(lib):
    F, _ = lib
    plan = F.Plan(32, 16, 64, 2.0, 1e-3)
    with pytest.raises(F.FTKError):  # no shifts yet
        plan.set_shift_windows([0.0, 0.5], 0.5)
    plan.set_shifts(synth.shift_lattice(2.0))
    with pytest.raises(F.FTKError):  # a window with no shift in it
        plan.set_shift_windows([0.0, 7.0], 0.25)
    plan.set_shift_windows([0.0, 0.5, 1.0], 0.5)
    plan.set_shift_windows([], 0.5)
