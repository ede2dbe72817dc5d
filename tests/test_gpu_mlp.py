"""GPU: the template-proposal kernels through the C-ABI against the FP64
oracle (oracle/mlp.py), and the per-image-list alignment against the full
alignment.

Bars: FP32 mode gradients and logits within 1e-5 of the oracle (relative to
each tensor's largest entry); bf16 mode within 1e-2 (bf16 operands, FP32
accumulation; the oracle uses the same bf16-rounded weights and inputs);
top-k decided on the same FP32 logits on both sides, so indices must be
equal; list alignment bitwise equal to the full alignment's pairs.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O
from oracle import mlp as ML

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
    F.lib()
    return F


def _dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / max(np.max(np.abs(b)), 1e-300))


def _net_case(seed, dims, n_t, n_s, B, n_rows):
    rng = np.random.default_rng(seed)
    params = synth.mlp_init(seed, dims)
    for l in range(len(params)):  # non-zero biases exercise the bias path
        params[l] = (params[l][0], (0.1 * rng.standard_normal(dims[l + 1])).astype(np.float32))
    x_all = (rng.standard_normal((n_rows, dims[0])) * 2.0 + 0.5).astype(np.float32)
    mu = rng.standard_normal(dims[0]).astype(np.float32) * 0.3
    isg = (0.5 + rng.random(dims[0])).astype(np.float32)
    lab_t = rng.integers(0, n_t, n_rows).astype(np.int32)
    lab_s = rng.integers(0, max(n_s, 1), n_rows).astype(np.int32)
    idx = rng.choice(n_rows, B, replace=False).astype(np.int32)
    return params, x_all, mu, isg, lab_t, lab_s, idx


def _oracle_inputs(x_all, mu, isg, idx, bf16):
    xs = ((x_all[idx] - mu) * isg).astype(np.float32)  # the FP32 standardisation the kernel does
    return ML.bf16_round(xs) if bf16 else xs.astype(np.float64)


@pytest.mark.parametrize("prec,tol,dims,B", [
    ("fp32", 1e-5, [37, 29, 23, 15], 19),
    ("bf16", 1e-2, [37, 29, 23, 15], 19),
    ("fp32", 1e-5, [130, 70, 66, 97], 65),
    ("bf16", 1e-2, [2048, 1024, 1024, 1024, 8201], 64),
])
def test_gradients_and_logits_match_oracle(ftk, prec, tol, dims, B):
    n_s = 9 if dims[-1] > 1000 else 5
    n_t = dims[-1] - n_s
    params, x_all, mu, isg, lab_t, lab_s, idx = _net_case(3, dims, n_t, n_s, B, 3 * B)
    _say(f"[mlp grads] {prec} dims={dims} B={B}")
    net = ftk.MLP(dims, n_t, n_s, prec, max_batch=128)
    net.set_params(params)
    net.set_input_norm(mu, isg)
    loss = net.gradients(_dev(x_all), _dev(lab_t, torch.int32), _dev(lab_s, torch.int32), _dev(idx, torch.int32))
    torch.cuda.synchronize()
    bf = prec == "bf16"
    oparams = [((ML.bf16_round(W) if bf else W.astype(np.float64)), b.astype(np.float64)) for W, b in params]
    xo = _oracle_inputs(x_all, mu, isg, idx, bf)
    # the bf16 form rounds every product operand (weights, activations,
    # gradients) to bf16; the oracle rounds the same operands, so the ReLU
    # decisions (z > 0) are taken on the same numbers on both sides
    rnd = ML.bf16_round if bf else None
    oloss, ograds = ML.loss_and_grads(oparams, xo, lab_t[idx], lab_s[idx], n_t, n_s, rnd=rnd)
    gl = float(loss.cpu().numpy()[0])
    _say(f"  loss gpu {gl:.7f} oracle {oloss:.7f}")
    assert abs(gl - oloss) <= tol * abs(oloss)
    if bf:  # for the record: against FP64 activations and gradients
        _, ugrads = ML.loss_and_grads(oparams, xo, lab_t[idx], lab_s[idx], n_t, n_s)
    for l in range(len(params)):
        dW, db = net.grad(l)
        eW, eb = _rel(dW, ograds[l][0]), _rel(db, ograds[l][1])
        extra = f" (unrounded oracle: dW {_rel(dW, ugrads[l][0]):.2e})" if bf else ""
        _say(f"  layer {l}: dW rel {eW:.2e} db rel {eb:.2e}{extra}")
        assert eW <= tol and eb <= tol
    # logits of the same rows through the forward entry point; the forward
    # pass is continuous in every rounding, so it also meets the bar against
    # the oracle without activation rounding
    logits = net.forward(_dev(x_all[idx])).cpu().numpy()
    _, _, ologits = ML.forward(oparams, xo, act_round=rnd)
    _, _, ulogits = ML.forward(oparams, xo)
    el, eu = _rel(logits, ologits), _rel(logits, ulogits)
    _say(f"  logits rel {el:.2e} (unrounded oracle {eu:.2e})")
    assert el <= tol and eu <= tol


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_adamw_steps_match_oracle(ftk, prec):
    dims, n_t, n_s, B = [40, 33, 12], 8, 4, 16
    params, x_all, mu, isg, lab_t, lab_s, idx = _net_case(5, dims, n_t, n_s, B, 64)
    net = ftk.MLP(dims, n_t, n_s, prec, max_batch=32)
    net.set_params(params)
    net.set_input_norm(mu, isg)
    hp = dict(lr=3e-3, beta1=0.9, beta2=0.99, eps=1e-6, wd=0.05)
    w = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    mom = [((np.zeros_like(W), np.zeros_like(W)), (np.zeros_like(b), np.zeros_like(b))) for W, b in w]
    xa, lt, ls = _dev(x_all), _dev(lab_t, torch.int32), _dev(lab_s, torch.int32)
    for t in range(1, 4):
        bidx = _dev(np.roll(idx, t), torch.int32)
        net.train_step(xa, lt, ls, bidx, **hp)
        torch.cuda.synchronize()
        for l in range(len(dims) - 1):
            dW, db = net.grad(l)  # the gradients this step used
            (mW, vW), (mb, vb) = mom[l]
            W, mW, vW = ML.adamw(w[l][0], dW, mW, vW, t, hp["lr"], hp["beta1"], hp["beta2"], hp["eps"], hp["wd"])
            b, mb, vb = ML.adamw(w[l][1], db, mb, vb, t, hp["lr"], hp["beta1"], hp["beta2"], hp["eps"], 0.0)
            w[l], mom[l] = (W, b), ((mW, vW), (mb, vb))
            gW, gb = net.get_layer(l)
            assert np.max(np.abs(gW - W)) <= 1e-6 * max(1.0, np.max(np.abs(W))), (t, l)
            assert np.max(np.abs(gb - b)) <= 1e-6 * max(1.0, np.max(np.abs(b))), (t, l)
    assert net.info()["step"] == 3


def test_features_and_proposal_match_oracle(ftk):
    n, M, Qa = 64, 32, 128
    s = synth.make_alignment_set(8, n, 3, 10, 20, 2.0, 0.1)
    P = ftk.Plan(n, M, Qa, 2.0, 1e-3)
    coeffs = P.transform(_dev(s.images))
    F = ftk.features(P, coeffs, 32, 32).cpu().numpy()
    Fx = ftk.features(P, coeffs, 13, 7, kind="cross").cpu().numpy()
    assert Fx.shape == (10, 7 * 13 * 13)
    Fi = ftk.features(P, coeffs, 32, 24, kind="invariant").cpu().numpy()
    assert Fi.shape == (10, 32 * 24)
    c = coeffs.cpu().numpy()
    for a in range(c.shape[0]):
        # shift- and rotation-invariant features: compare |P| = F^2
        refi = ML.invariant_features(c[a].T.astype(np.complex128), 32, 24)
        assert _rel(Fi[a].astype(np.float64) ** 2, refi ** 2) <= 1e-5
        ref = ML.features(c[a].T.astype(np.complex128), 32, 32)
        assert _rel(F[a], ref) <= 1e-6
        # cross features: compare the products (the square root magnifies
        # rounding of products near zero)
        refx = ML.cross_features(c[a].T.astype(np.complex128), 13, 7)
        gx = np.sign(Fx[a]).astype(np.float64) * Fx[a].astype(np.float64) ** 2
        assert _rel(gx, np.sign(refx) * refx ** 2) <= 1e-6
    # proposals from FP32 logits: both sides rank the same numbers
    dims, n_t, n_s = [1024, 96, 300 + 7], 300, 7
    net = ftk.MLP(dims, n_t, n_s, "bf16", max_batch=4)  # 10 rows: slices of 4
    net.set_params(synth.mlp_init(2, dims))
    mu = F.mean(axis=0)
    isg = 1.0 / (F.std(axis=0) + 1e-12)
    net.set_input_norm(mu, isg)
    Fd = _dev(F)
    top, mass, sb = net.propose(Fd, 20)
    logits = np.concatenate([net.forward(Fd[i:i + 4]).cpu().numpy() for i in range(0, 10, 4)])
    idx, omass, osb = ML.propose(logits, n_t, 20)
    assert np.array_equal(top.cpu().numpy(), idx)
    assert np.array_equal(sb.cpu().numpy(), osb)
    assert _rel(mass.cpu().numpy(), omass) <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16"])
def test_list_alignment_equals_full_alignment(ftk, prec):
    n, M, Qa, R = 64, 32, 128, 2.0
    s = synth.make_alignment_set(12, n, 45, 9, 20, R, 0.1)
    P = ftk.Plan(n, M, Qa, R, 1e-3, prec)
    P.set_shifts(synth.shift_lattice(R))
    a = P.transform(_dev(s.images))
    b = P.transform(_dev(s.templates))
    _, full = P.align_coeffs(a, b)
    full = full.cpu().numpy()
    rng = np.random.default_rng(1)
    K = 21  # off the 16-template tiles; duplicates allowed
    lists = rng.integers(0, 45, (9, K)).astype(np.int32)
    lists[0, :3] = 44
    for stage in (0, 16):  # default staging, then one image per chunk
        P.set_tuning(stage_mib=stage)
        got = ftk.align_lists(P, a, b, _dev(lists, torch.int32)).cpu().numpy()
        for i in range(9):
            assert np.array_equal(got[i], full[i, lists[i]]), (stage, i)
    # best template over the list vs brute force on the host
    bt, bp = ftk.best_template(_dev(got, torch.int32), _dev(lists, torch.int32))
    bt, bp = bt.cpu().numpy(), bp.cpu().numpy()
    v = got[:, :, 0].view(np.float32)
    for i in range(9):
        order = sorted(range(K), key=lambda j: (-float(v[i, j]), int(lists[i, j])))
        assert bt[i] == lists[i, order[0]]
        assert np.array_equal(bp[i], got[i, order[0]])
