"""GPU: the learned proposal end to end, scaled down.

Training images are noise-free moved templates re-noised every epoch; the
full FTK search labels each epoch's images; the network is trained on the
GPU by the library's own kernels; the confidence threshold is chosen on a
held-out validation split; on a separate test split the proposal search
must recover the full search's best template and pose on >= 99 % of images
while evaluating fewer image-template pairs than the full search.  The
network's outputs and recall are learned quantities (parity unpinned);
only the kernels are pinned (test_gpu_mlp.py).
"""
import sys
import time

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


def test_proposal_recall_and_gain(lib):
    F, PR = lib
    n, M, Qa, R, eps = 64, 32, 128, 2.0, 1e-3
    n_t, n_clean, n_val, n_test = 128, 24576, 1024, 512
    n_r, n_q, topk, kind = 16, 8, 32, "cross"
    t0 = time.perf_counter()
    s = synth.make_alignment_set(21, n, n_t, n_clean + n_val + n_test, 30, R, 0.1, keep_clean=True)
    shifts = synth.shift_lattice(R)
    bins = PR.shift_bins(shifts)
    n_s = int(bins.max()) + 1
    _say(f"[proposal] data {time.perf_counter() - t0:.1f} s: {n_t} templates, {s.images.shape[0]} images, n={n}")
    plan = F.Plan(n, M, Qa, R, eps, "bf16x3")
    plan.set_shifts(shifts)
    tmps = torch.as_tensor(s.templates, dtype=torch.float32, device="cuda")
    tc = plan.transform(tmps)
    clean = torch.as_tensor(s.clean[:n_clean], dtype=torch.float32, device="cuda")
    sig = s.noise_sigma[:n_clean]
    dims = [F.feature_count(kind, n_r, n_q), 1024, 1024, n_t + n_s]
    net = F.MLP(dims, n_t, n_s, "bf16", max_batch=1024)
    net.set_params(synth.mlp_init(4, dims))
    perms = [synth.permutation(100 + e, n_clean) for e in range(60)]
    t0 = time.perf_counter()
    losses = PR.train_online(net, plan, clean, tc, bins, lambda e: synth.gaussian_noise(1000 + e, sig, n), perms,
                             kind, n_r, n_q, batch=256, lr=2e-3, wd=1e-2)
    _say(f"  trained {len(perms)} epochs in {time.perf_counter() - t0:.1f} s; loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert losses[-1] < 0.7 * losses[0]
    # threshold from the validation split (its own fixed noise)
    vi = torch.as_tensor(s.images[n_clean:n_clean + n_val], dtype=torch.float32, device="cuda")
    vlab, _, _ = PR.ftk_labels(plan, vi, tmps, bins)
    vf = F.features(plan, plan.transform(vi), n_r, n_q, kind=kind)
    top, mass, _ = net.propose(vf, topk)
    hit = (top.cpu().numpy() == vlab.cpu().numpy()[:, None]).any(axis=1)
    tau = PR.choose_tau(mass.cpu().numpy(), hit, max_miss=0.003)
    _say(f"  validation: top-{topk} hit rate {hit.mean():.3f}; tau = {tau:.4f}")
    # test split: proposal search against the full search
    ti = torch.as_tensor(s.images[n_clean + n_val:], dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bt, bp, fb, nfb = F.align_proposed(plan, net, ti, tc, n_r, n_q, topk, tau, kind=kind)
    torch.cuda.synchronize()
    t_prop = time.perf_counter() - t1
    t1 = time.perf_counter()
    _, full = plan.align(ti, tmps)
    fbt, fbp = F.best_template(full)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t1
    bt, bp, fb = bt.cpu().numpy(), bp.cpu().numpy(), fb.cpu().numpy()
    fbt, fbp = fbt.cpu().numpy(), fbp.cpu().numpy()
    same = (bt == fbt) & np.all(bp == fbp, axis=1)
    pairs_prop = n_test * topk + nfb * n_t
    _say(f"  test: recall of the full search's best pose {same.mean():.4f}; fallback {nfb}/{n_test}; "
         f"pairs evaluated {pairs_prop} vs {n_test * n_t} ({n_test * n_t / pairs_prop:.2f}x fewer); "
         f"time {t_prop * 1e3:.1f} ms vs {t_full * 1e3:.1f} ms")
    assert int(np.count_nonzero(fb)) == nfb
    assert np.all(same[fb == 1])  # the fallback is the full search
    assert same.mean() >= 0.99
    assert pairs_prop < 0.8 * n_test * n_t
