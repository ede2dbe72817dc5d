"""Pins of the FP64 proposal oracle (oracle/mlp.py) against what the
mathematics fixes: central finite differences of the loss, closed forms of
softmax cross-entropy and AdamW, exact rotation invariance of the features,
the bfloat16 format, and brute-force top-k.  Planted mistakes must fail.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ftk as O
from oracle import mlp as ML


def _tiny_net(rng, dims):
    return [(rng.standard_normal((dims[i + 1], dims[i])) / math.sqrt(dims[i]),
             0.1 * rng.standard_normal(dims[i + 1])) for i in range(len(dims) - 1)]


def _fd_grads(params, x, lt, ls, n_t, n_s, h=1e-6):
    out = []
    for l, (W, b) in enumerate(params):
        gW = np.zeros_like(W)
        gb = np.zeros_like(b)
        for arr, g in ((W, gW), (b, gb)):
            for idx in np.ndindex(arr.shape):
                keep = arr[idx]
                arr[idx] = keep + h
                fp, _ = ML.loss_and_grads(params, x, lt, ls, n_t, n_s)
                arr[idx] = keep - h
                fm, _ = ML.loss_and_grads(params, x, lt, ls, n_t, n_s)
                arr[idx] = keep
                g[idx] = (fp - fm) / (2 * h)
        out.append((gW, gb))
    return out


def _max_rel(a, b):
    return max(np.max(np.abs(x - y)) / max(np.max(np.abs(y)), 1e-300) for (x, y) in zip(a, b))


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    n_t, n_s = 5, 3
    params = _tiny_net(rng, [6, 7, 5, n_t + n_s])
    x = rng.standard_normal((4, 6))
    lt = rng.integers(0, n_t, 4)
    ls = rng.integers(0, n_s, 4)
    _, grads = ML.loss_and_grads(params, x, lt, ls, n_t, n_s)
    fd = _fd_grads(params, x, lt, ls, n_t, n_s)
    for (gW, gb), (fW, fb) in zip(grads, fd):
        assert _max_rel([gW, gb], [fW, fb]) < 1e-6


def test_planted_mistakes_fail_the_difference_check():
    rng = np.random.default_rng(1)
    n_t, n_s = 4, 2
    params = _tiny_net(rng, [5, 6, n_t + n_s])
    x = rng.standard_normal((3, 5))
    lt = rng.integers(0, n_t, 3)
    ls = rng.integers(0, n_s, 3)
    fd = _fd_grads(params, x, lt, ls, n_t, n_s)
    hs, zs, logits = ML.forward(params, x)
    _, d = ML.loss_and_dlogits(logits, lt, ls, n_t, n_s)

    def bad_backward_no_relu_mask(params, hs, zs, dl):
        grads = [None] * len(params)
        g = dl
        for l in range(len(params) - 1, -1, -1):
            grads[l] = (g.T @ hs[l], np.sum(g, axis=0))
            if l > 0:
                g = g @ params[l][0]
        return grads

    def bad_backward_transposed(params, hs, zs, dl):
        grads = [None] * len(params)
        g = dl
        for l in range(len(params) - 1, -1, -1):
            grads[l] = (g.T @ hs[l], np.sum(g, axis=0))
            if l > 0:
                W = params[l][0]
                g = (g @ W) * (zs[l - 1] > 0)
        grads[0] = (grads[0][0], np.zeros_like(grads[0][1]))  # bias gradient dropped
        return grads

    for bad in (bad_backward_no_relu_mask, bad_backward_transposed):
        g = bad(params, hs, zs, d)
        worst = max(_max_rel([gW, gb], [fW, fb]) for (gW, gb), (fW, fb) in zip(g, fd))
        assert worst > 1e-3


def test_cross_entropy_closed_forms():
    # equal logits: CE = log n_t + log n_s, gradient (1/n - onehot)/B per head
    B, n_t, n_s = 3, 7, 4
    z = np.full((B, n_t + n_s), 0.25)
    lt = np.array([0, 3, 6])
    ls = np.array([1, 1, 3])
    loss, d = ML.loss_and_dlogits(z, lt, ls, n_t, n_s)
    assert loss == pytest.approx(math.log(n_t) + math.log(n_s), rel=1e-14)
    want = np.zeros_like(z)
    want[:, :n_t] = 1.0 / n_t
    want[:, n_t:] = 1.0 / n_s
    want[np.arange(B), lt] -= 1.0
    want[np.arange(B), n_t + ls] -= 1.0
    assert np.allclose(d, want / B, rtol=0, atol=1e-15)
    # a dominant correct logit: CE -> exp(-gap) (1 + ...) on that head
    z = np.zeros((1, 3))
    z[0, 1] = 30.0
    loss, _ = ML.loss_and_dlogits(z, np.array([1]), np.array([0]), 3, 0)
    assert loss == pytest.approx(2 * math.exp(-30.0), rel=1e-9)


def test_adamw_closed_forms():
    # first step, no decay: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3])
    w0 = np.array([1.0, 2.0, -1.0])
    w, m, v = ML.adamw(w0, g, np.zeros(3), np.zeros(3), 1, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0)
    assert np.allclose(w, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # zero gradient: pure decoupled decay w (1 - lr wd)
    w, _, _ = ML.adamw(w0, np.zeros(3), np.zeros(3), np.zeros(3), 5, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8,
                       wd=0.01)
    assert np.allclose(w, w0 * (1 - 0.1 * 0.01), rtol=0, atol=1e-15)
    # constant gradient: after t steps m_hat = g and v_hat = g^2 exactly
    w, m, v = w0.copy(), np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        w, m, v = ML.adamw(w, g, m, v, t, lr=0.01, beta1=0.9, beta2=0.99, eps=0.0, wd=0.0)
    assert np.allclose(w, w0 - 5 * 0.01 * np.sign(g), rtol=0, atol=1e-12)


def test_bf16_round_matches_the_format():
    # exactly representable values stay; halfway cases go to even; 1 + 2^-8 -> 1
    vals = np.array([1.0, -2.5, 0.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65280.0, 1e-40], np.float32)
    got = ML.bf16_round(vals)
    want = [1.0, -2.5, 0.0, 1.0, 1.0 + 4 * 2.0 ** -8, 65280.0, None]
    for g, w in zip(got[:6], want[:6]):
        assert g == w
    # relative error bound: unit roundoff 2^-8 of an 8-bit significand
    x = np.random.default_rng(3).standard_normal(10000).astype(np.float32)
    r = ML.bf16_round(x)
    assert np.max(np.abs(r - x) / np.abs(x)) <= 2.0 ** -8
    # the stored value has 8 significant bits: its low 16 bits of float32 are zero
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_features_are_rotation_invariant():
    """A 90 degree pixel rotation about pixel (n/2, n/2) is exact on the
    grid; with Qa a multiple of 4 it maps polar samples to polar samples, so
    |a(k; q)|^2 must be unchanged to rounding."""
    n, M, Qa = 32, 16, 64
    img = synth.make_alignment_set(9, n, 1, 1, 20, 2.0, 0.1).images[0].copy()
    # pixels of index 0 (x = -1 or y = -1) have no rotated partner on the grid
    img[0, :] = 0.0
    img[:, 0] = 0.0
    rot = np.roll(np.rot90(img), 1, axis=0)
    # np.rot90 maps index (i, j) -> (n-1-j, i); rolling the first axis by one
    # makes that (n-j, i) mod n: a rotation about (n/2, n/2)
    i, j = 5, 9
    assert rot[(n - j) % n, i] == img[i, j]
    plan = O.make_plan(n, M, Qa, 2.0, 1e-3)
    f0 = ML.features(O.fb_coefficients(img, plan), M, 32)
    f1 = ML.features(O.fb_coefficients(rot, plan), M, 32)
    assert np.max(np.abs(f1 - f0)) <= 1e-12 * np.max(np.abs(f0))
    # and they do change under a shift (the features are not shift invariant)
    sh = np.roll(img, 2, axis=0)
    f2 = ML.features(O.fb_coefficients(sh, plan), M, 32)
    assert np.max(np.abs(f2 - f0)) > 1e-3 * np.max(np.abs(f0))


def test_cross_features_rotation_invariant_and_laid_out():
    n, M, Qa = 32, 16, 64
    img = synth.make_alignment_set(9, n, 1, 1, 20, 2.0, 0.1).images[0].copy()
    img[0, :] = 0.0
    img[:, 0] = 0.0
    rot = np.roll(np.rot90(img), 1, axis=0)
    plan = O.make_plan(n, M, Qa, 2.0, 1e-3)
    a0 = O.fb_coefficients(img, plan)
    a1 = O.fb_coefficients(rot, plan)
    f0 = ML.cross_features(a0, 6, 5)
    f1 = ML.cross_features(a1, 6, 5)
    assert f0.shape == (5 * 36,)
    # compare the products themselves: the square root magnifies rounding near 0
    p0, p1 = np.sign(f0) * f0 ** 2, np.sign(f1) * f1 ** 2
    assert np.max(np.abs(p1 - p0)) <= 1e-12 * np.max(np.abs(p0))
    # without the conjugate the product is not invariant: a planted mistake fails
    # (mode 1: a quarter turn multiplies each factor by -i, the product by -1)
    bad0 = a0[1, 1] * a0[3, 1]
    bad1 = a1[1, 1] * a1[3, 1]
    assert abs(bad1 - bad0) > 1e-3 * abs(bad0)
    # the layout, entry by entry, for mode q = 2 (block offset 2 * 36)
    s = lambda x: np.sign(x) * np.sqrt(abs(x))
    c = a0[1, 2] * np.conj(a0[3, 2])
    re_idx = [(k1, k2) for k1 in range(6) for k2 in range(k1, 6)].index((1, 3))
    im_idx = 21 + [(k1, k2) for k1 in range(6) for k2 in range(k1 + 1, 6)].index((1, 3))
    assert f0[72 + re_idx] == pytest.approx(s(c.real), rel=1e-12)
    assert f0[72 + im_idx] == pytest.approx(s(c.imag), rel=1e-12)
    # diagonal products are real and equal the power features
    assert f0[72 + 0] == pytest.approx(math.sqrt(abs(a0[0, 2]) ** 2), rel=1e-12)


def _bordered_blob_image(n, seed):
    # blobs well inside the frame, the outer 4 pixels exactly zero: a cyclic
    # roll by up to 4 pixels is then an exact shift of the image
    img = synth.render(synth.random_blobs(np.random.default_rng(seed), 10, disk_px=4.0, sigma_px=(1.0, 2.0)), n)
    img[:4, :] = 0.0
    img[-4:, :] = 0.0
    img[:, :4] = 0.0
    img[:, -4:] = 0.0
    img[0, :] = 0.0
    img[:, 0] = 0.0
    return img


def test_invariant_features_definition():
    """sqrt|P(k; 2j)| computed from the ring samples (the inverse ring DFT of
    the coefficients, then the DFT of their power) equals the cyclic
    autocorrelation of the coefficients; the odd harmonics of the power of a
    real image vanish."""
    n, M, Qa = 32, 16, 64
    img = synth.white_noise_images(4, 1, n)[0]
    a = O.fb_coefficients(img, O.make_plan(n, M, Qa, 2.0, 1e-3))
    f = ML.invariant_features(a, M, 20)
    samples = Qa * np.fft.ifft(a, axis=1)  # Ahat(k_m, psi_p) = sum_q a(k_m; q) e^{i q psi_p}
    P = np.fft.fft(np.abs(samples) ** 2, axis=1) / Qa
    ref = np.abs(P[:, 0:40:2]).reshape(-1)
    # compare |P| itself (the square root magnifies rounding near zero)
    assert np.max(np.abs(f ** 2 - ref)) <= 1e-12 * np.max(ref)
    assert np.max(np.abs(P[:, 1::2])) <= 1e-12 * np.max(np.abs(P))


def test_invariant_features_shift_and_rotation_invariant(monkeypatch):
    n, M, Qa = 32, 16, 64
    plan = O.make_plan(n, M, Qa, 2.0, 1e-3)
    img = _bordered_blob_image(n, 12)
    f0 = ML.invariant_features(O.fb_coefficients(img, plan), M, 16)
    # exact pixel shifts (the frame's zero border absorbs the roll)
    for d in [(3, -2), (-4, 1), (1, 4)]:
        f1 = ML.invariant_features(O.fb_coefficients(np.roll(img, d, axis=(0, 1)), plan), M, 16)
        # |P| = F^2 (the square root magnifies rounding near zero)
        assert np.max(np.abs(f1 ** 2 - f0 ** 2)) <= 1e-12 * np.max(f0 ** 2), d
    # an exact quarter turn about pixel (n/2, n/2)
    rot = np.roll(np.rot90(img), 1, axis=0)
    f2 = ML.invariant_features(O.fb_coefficients(rot, plan), M, 16)
    assert np.max(np.abs(f2 ** 2 - f0 ** 2)) <= 1e-12 * np.max(f0 ** 2)
    # both at once, with the shift off the pixel grid: the image is rendered
    # with its blobs moved, so agreement is to the sampling of the blobs
    rng = np.random.default_rng(12)
    blobs = synth.random_blobs(rng, 10, disk_px=4.0, sigma_px=(2.0, 3.0))
    g0 = ML.invariant_features(O.fb_coefficients(synth.render(blobs, n), plan), M, 16)
    moved = synth.render(blobs.moved(0.7, (1.3, -0.6)), n)
    g1 = ML.invariant_features(O.fb_coefficients(moved, plan), M, 16)
    assert np.max(np.abs(g1 ** 2 - g0 ** 2)) <= 1e-5 * np.max(g0 ** 2)  # measured 6e-7
    # planted: without the conjugate the product is not shift invariant
    def bad(c, n_r, n_q):
        a = np.asarray(c)
        return np.array([math.sqrt(abs(np.sum(a[m] * a[m, (np.arange(Qa) - 2 * j) % Qa])))
                         for m in range(n_r) for j in range(n_q)])
    monkeypatch.setattr(ML, "invariant_features", bad)
    b0 = ML.invariant_features(O.fb_coefficients(img, plan), M, 16)
    b1 = ML.invariant_features(O.fb_coefficients(np.roll(img, (3, -2), axis=(0, 1)), plan), M, 16)
    assert np.max(np.abs(b1 ** 2 - b0 ** 2)) > 1e-2 * np.max(b0 ** 2)


def test_features_of_real_image_are_symmetric_in_q():
    n, M, Qa = 32, 16, 64
    img = synth.white_noise_images(2, 1, n)[0]
    a = O.fb_coefficients(img, O.make_plan(n, M, Qa, 2.0, 1e-3))
    for q in range(1, Qa // 2):
        assert np.allclose(np.abs(a[:, q]), np.abs(a[:, Qa - q]), rtol=1e-12, atol=1e-14)


def test_propose_matches_brute_force():
    rng = np.random.default_rng(4)
    n_t, n_s, k = 50, 6, 7
    z = rng.standard_normal((9, n_t + n_s)).astype(np.float32)
    z[0, 8] = z[0, 3] = 10.0  # a tie at the top: the lower index comes first
    idx, mass, sb = ML.propose(z, n_t, k)
    for r in range(z.shape[0]):
        order = sorted(range(n_t), key=lambda t: (-float(z[r, t]), t))[:k]
        assert list(idx[r]) == order
        p = np.exp(z[r, :n_t].astype(np.float64))
        p /= p.sum()
        assert mass[r] == pytest.approx(p[order].sum(), rel=1e-12)
        assert sb[r] == int(np.argmax(z[r, n_t:]))
    assert list(idx[0][:2]) == [3, 8]
