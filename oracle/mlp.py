"""FP64 oracle of the learned template proposal (features, MLP, loss,
gradients, AdamW, top-k proposal).

TEST INFRASTRUCTURE ONLY -- the product path never imports this module.

The paper has no learned part; this module defines, plainly, what the
proposal computes so the GPU kernels can be checked against it:

  * features: F[m, q] = |a(k_m; q)|^2 for the first n_r radial nodes and
    modes q = 0 .. n_q - 1.  A rotation of the image multiplies a(k; q) by a
    phase (the rotation property of Fourier-Bessel coefficients, Section 3),
    so F is rotation invariant; for a real image |a(k; -q)| = |a(k; q)|, so
    non-negative q carry all of it.  Flattened index f = m * n_q + q.
  * input standardisation x = (F - mu) * inv_sigma (per feature).
  * MLP: h_0 = x; h_{l+1} = relu(h_l W_l^T + b_l) for hidden layers, the last
    layer linear; W_l has shape [out, in].
  * two softmax heads on the logits: templates [0, n_t) and shift-radius
    bins [n_t, n_t + n_s); loss = mean over the batch of CE_t + CE_s.
  * AdamW (Loshchilov and Hutter, decoupled weight decay) on FP32 master
    parameters; decay applies to weights, not biases.
  * proposal: the top-k templates by softmax probability (ties: lower index
    first) and their probability mass as the confidence.

Everything is FP64 unless a function says otherwise.  `bf16_round` is the
round-to-nearest-even of a float32 to bfloat16, written from the format's
definition (8 exponent bits, 7 stored mantissa bits).
"""
from __future__ import annotations

import math

import numpy as np


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def features(coeffs_rings_modes: np.ndarray, n_r: int, n_q: int) -> np.ndarray:
    """F[m * n_q + q] = |a(k_m; q)|^2 from coefficients laid out [M][Qa] (ring
    m, mode q in storage order 0..Qa/2-1, -Qa/2..-1)."""
    a = np.asarray(coeffs_rings_modes)
    return (np.abs(a[:n_r, :n_q]) ** 2).reshape(-1)


def cross_features(coeffs_rings_modes: np.ndarray, n_r: int, n_q: int) -> np.ndarray:
    """Rotation-invariant products of two rings at one mode,
    c(k1, k2; q) = a(k1; q) conj a(k2; q) (a rotation multiplies both by
    the same phase, which cancels), for rings k1 <= k2 < n_r and modes
    0 <= q < n_q, each taken through the signed square root
    s(x) = sign(x) sqrt|x| (homogeneous of degree one in the image).
    Per mode q a block of n_r^2 numbers: the real parts for k1 <= k2, then
    the imaginary parts for k1 < k2, pairs in row-major (k1, then k2) order."""
    a = np.asarray(coeffs_rings_modes)
    out = []
    for q in range(n_q):
        re, im = [], []
        for k1 in range(n_r):
            for k2 in range(k1, n_r):
                c = a[k1, q] * np.conj(a[k2, q])
                re.append(c.real)
                if k2 > k1:
                    im.append(c.imag)
        out.extend(re)
        out.extend(im)
    v = np.asarray(out, dtype=np.float64)
    return np.sign(v) * np.sqrt(np.abs(v))


def invariant_features(coeffs_rings_modes: np.ndarray, n_r: int, n_q: int) -> np.ndarray:
    """Features invariant to both the rotation and the shift of the image.
    A shift multiplies Ahat(k) by a phase (eq. Fdk), so the power |Ahat(k_m,
    psi)|^2 on ring m does not change; a rotation turns it in psi, so the
    moduli of its angular Fourier coefficients do not change.  With the ring
    samples Ahat(k_m, psi_p) = sum_q a(k_m; q) exp(i q psi_p) (eq. aqkcalc
    inverted) the coefficient of exp(i s psi) in the power is the cyclic
    autocorrelation P(k_m; s) = sum_q a(k_m; q) conj a(k_m; q - s) (indices
    mod Qa); for real images the power is pi-periodic in psi, so only even s
    carry information.  F[m * n_q + j] = sqrt|P(k_m; 2 j)| (homogeneous of
    degree one in the image), m < n_r, j < n_q."""
    a = np.asarray(coeffs_rings_modes, dtype=np.complex128)
    Qa = a.shape[1]
    out = np.zeros((n_r, n_q))
    for m in range(n_r):
        for j in range(n_q):
            s = 2 * j
            out[m, j] = math.sqrt(abs(np.sum(a[m] * np.conj(a[m, (np.arange(Qa) - s) % Qa]))))
    return out.reshape(-1)


def standardise(F: np.ndarray, mu: np.ndarray, inv_sigma: np.ndarray) -> np.ndarray:
    return (np.asarray(F, dtype=np.float64) - mu) * inv_sigma


def forward(params, x, act_round=None):
    """params: list of (W [out, in], b [out]); x [B, in].  Returns the list of
    layer inputs h_0..h_L-1, the pre-activations z_0..z_L-1 and the logits.
    act_round (e.g. bf16_round) is applied to every hidden activation, the
    operands a reduced-precision form feeds to the next product."""
    h = np.asarray(x, dtype=np.float64)
    hs, zs = [], []
    L = len(params)
    for l, (W, b) in enumerate(params):
        hs.append(h)
        z = h @ np.asarray(W, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
        zs.append(z)
        h = np.maximum(z, 0.0) if l < L - 1 else z
        if act_round is not None and l < L - 1:
            h = act_round(h)
    return hs, zs, h


def _log_softmax(z):
    zmax = np.max(z, axis=1, keepdims=True)
    s = z - zmax
    return s - np.log(np.sum(np.exp(s), axis=1, keepdims=True))


def loss_and_dlogits(logits, lab_t, lab_s, n_t: int, n_s: int):
    """Mean over the batch of CE on the template head plus CE on the shift
    head; returns (loss, d loss / d logits)."""
    z = np.asarray(logits, dtype=np.float64)
    B = z.shape[0]
    d = np.zeros_like(z)
    loss = 0.0
    for lo, width, lab in ((0, n_t, lab_t), (n_t, n_s, lab_s)):
        if width == 0:
            continue
        ls = _log_softmax(z[:, lo:lo + width])
        loss += -np.sum(ls[np.arange(B), lab]) / B
        p = np.exp(ls)
        p[np.arange(B), lab] -= 1.0
        d[:, lo:lo + width] = p / B
    return loss, d


def backward(params, hs, zs, dlogits, grad_round=None):
    """Gradients [(dW, db)] by the chain rule through the linear layers and
    the ReLUs of the hidden layers.  grad_round (e.g. bf16_round) is applied
    to the gradient where it enters a product (dW and the gradient of the
    layer input), not to the bias gradient, which is a plain sum."""
    grads = [None] * len(params)
    g = np.asarray(dlogits, dtype=np.float64)
    for l in range(len(params) - 1, -1, -1):
        W = np.asarray(params[l][0], dtype=np.float64)
        gr = grad_round(g) if grad_round is not None else g
        grads[l] = (gr.T @ hs[l], np.sum(g, axis=0))
        if l > 0:
            g = (gr @ W) * (zs[l - 1] > 0.0)
    return grads


def loss_and_grads(params, x, lab_t, lab_s, n_t, n_s, rnd=None):
    """Loss and gradients; rnd (e.g. bf16_round) rounds every product operand
    that a reduced-precision form rounds: hidden activations and gradients."""
    hs, zs, logits = forward(params, x, act_round=rnd)
    loss, d = loss_and_dlogits(logits, lab_t, lab_s, n_t, n_s)
    return loss, backward(params, hs, zs, d, grad_round=rnd)


def adamw(w, g, m, v, t: int, lr, beta1, beta2, eps, wd):
    """One AdamW step (t counts from 1); returns the new (w, m, v)."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v


def softmax(z):
    return np.exp(_log_softmax(np.asarray(z, dtype=np.float64)))


def propose(logits, n_t: int, k: int):
    """Top-k templates per row by probability (ties to the lower index), the
    probability mass they hold, and the most probable shift bin."""
    z = np.asarray(logits, dtype=np.float64)
    p = softmax(z[:, :n_t])
    # softmax is increasing in the logit, so ranking logits ranks probabilities
    idx = np.argsort(-z[:, :n_t], axis=1, kind="stable")[:, :k]
    mass = np.take_along_axis(p, idx, axis=1).sum(axis=1)
    sbin = np.argmax(z[:, n_t:], axis=1) if z.shape[1] > n_t else np.zeros(z.shape[0], np.int64)
    return idx, mass, sbin
