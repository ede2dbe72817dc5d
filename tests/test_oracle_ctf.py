"""Pins of the oracle's joint translation-CTF factorisation (Section 7.1;
readings in oracle/ctf.py).

Pinned by: the frequency convention of the CTF against filtering the pixel
image with a 2D DFT on a zero-padded grid; a constant CTF reducing the
factorisation to the plain translation SVD (same singular values) and the
FTK result to -1 times the plain one; the total and per-mode Hilbert-Schmidt
norms against independent quadrature (sum_l J_l^2 = 1); reconstruction of
the kernel in the operator's norm (eq. efrob); the truncation bound of
eq. Xmserr over shifts, defocus and rotations; planted mistakes.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import jv

import synth
from oracle import ctf as C
from oracle import ftk as O

# 300 kV electrons, Cs 2.7 mm, 7 % amplitude contrast, 2 A pixels
CTF = C.CtfModel(0.019687, 2.7, 0.07, 2.0)
T0, T1 = 14000.0, 16000.0


@pytest.fixture(scope="module")
def plan32():
    return C.make_ctf_plan(32, 16, 64, 2.0, 1e-3, CTF, T0, T1)


def _polar_ft_grid(img, k, Qa, origin):
    """dx^2 sum A_ij exp(-i k . x_ij) for a grid of pixel size 2/n0 whose
    pixel `origin` is the image origin (n0 = the unpadded side)."""
    n0 = 2 * origin[1]
    dx = 2.0 / n0
    N = img.shape[0]
    xs = (np.arange(N) - origin[0]) * dx
    psi = O.polar_angles(Qa)
    Ex = np.exp(-1j * np.multiply.outer(np.multiply.outer(k, np.cos(psi)), xs))
    Ey = np.exp(-1j * np.multiply.outer(np.multiply.outer(k, np.sin(psi)), xs))
    return dx * dx * np.sum(Ex * (Ey @ img.T), axis=-1)


def _filter_error(scale):
    # a blob image filtered in pixel space with the CTF on the DFT grid of a
    # 4x zero-padded frame (frequencies in 1/Angstrom from the pixel size);
    # its polar transform must equal the unfiltered one times C(k / Kmax)
    n, pad, tau = 32, 4, 2500.0
    rng = np.random.default_rng(2)
    img = synth.render(synth.random_blobs(rng, 5, disk_px=5.0, sigma_px=(2.0, 3.0)), n)
    N = pad * n
    big = np.zeros((N, N))
    o = N // 2 - n // 2
    big[o:o + n, o:o + n] = img
    f = np.fft.fftfreq(N, d=CTF.pixel_A)
    s = np.hypot(f[:, None], f[None, :])
    flt = np.real(np.fft.ifft2(np.fft.fft2(big) * CTF(scale * 2.0 * CTF.pixel_A * s, tau)))
    kmax = 0.5 * math.pi * n
    k, _ = O.radial_quadrature(12, kmax)
    want = O.polar_ft(img, k, 48) * CTF(k / kmax, tau)[:, None]
    got = _polar_ft_grid(flt, k, 48, (N // 2, n // 2))
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def test_ctf_frequency_convention():
    assert _filter_error(1.0) < 1e-6


def test_constant_ctf_is_the_translation_svd():
    flat = C.CtfModel(0.0, 0.0, 1.0, 2.0)  # chi = 0, A = 1: C = -1
    X = math.pi * 2.0
    for ell in (0, 3):
        s = C.ctf_modal_svd(ell, X, flat, T0, T1)
        ref = O.modal_svd(ell, X).sigma
        h = int(np.sum(ref > 1e-12))
        assert np.allclose(s.sigma[:h], ref[:h], rtol=1e-10, atol=1e-14)
    img = synth.white_noise_images(5, 2, 32)
    pc = C.set_poses(C.make_ctf_plan(32, 16, 64, 2.0, 1e-3, flat, T0, T1), synth.shift_lattice(2.0),
                     np.full(49, 15000.0))
    pp = O.set_shifts(O.make_plan(32, 16, 64, 2.0, 1e-3), synth.shift_lattice(2.0))
    a, b = (O.fb_coefficients(x, pp) for x in img)
    Xc, Xp = O.ftk_X(a, b, pc), O.ftk_X(a, b, pp)
    assert pc.H == pp.H
    assert np.max(np.abs(Xc + Xp)) < 1e-10 * np.max(np.abs(Xp))


def _mean_c2(y):
    # defocus average of C^2 by an independent composite rule
    t = np.linspace(T0, T1, 4001)
    v = CTF(y, t) ** 2
    return float(np.sum((v[1:] + v[:-1]) * 0.5) / (t.size - 1))


def test_total_hilbert_schmidt_norm(plan32):
    X = math.pi * 2.0
    want = 0.5 * X * X * quad(lambda y: y * _mean_c2(y), 0.0, 1.0, limit=400)[0]
    total = 0.0
    for ell in range(0, 40):
        s = C.ctf_modal_svd(ell, X, CTF, T0, T1)
        part = float(np.sum(s.sigma ** 2))
        total += part if ell == 0 else 2.0 * part
        if part < 1e-20:
            break
    assert math.isclose(total, want, rel_tol=1e-8)


@pytest.mark.parametrize("ell", [0, 4])
def test_modal_hilbert_schmidt_norm(ell):
    X = math.pi * 2.0
    s = C.ctf_modal_svd(ell, X, CTF, T0, T1)

    def inner(x):
        return x * quad(lambda y: jv(ell, x * y) ** 2 * _mean_c2(y) * y, 0.0, 1.0, limit=400)[0]

    want = quad(inner, 0.0, X, limit=200)[0]
    assert math.isclose(float(np.sum(s.sigma ** 2)), want, rel_tol=1e-6)


def test_reconstruction_in_operator_norm(plan32):
    # || K_l - sum_{eta <= h} u sigma v ||^2 = sum_{eta > h} sigma^2 on a grid
    # of nodes independent of the SVD's
    ell = 2
    sv = plan32.svds[ell]
    h = int(np.sum(plan32.ell == ell))
    xq, xw = O.radial_quadrature(80, sv.X)
    tq, tw = C.legendre_rule(30, T0, T1)
    yq, yw = O.radial_quadrature(260, 1.0)
    # Sigma v_eta(y) on the grid, every eta at once (Nystrom through the shift side)
    Ky = jv(ell, np.multiply.outer(yq, sv.xn)) * CTF(yq[:, None], sv.tn[None, :])
    SV = Ky @ (np.sqrt(sv.rw)[:, None] * sv.Umat[:, :h])  # (y, eta)
    resid = 0.0
    for t, wt in zip(tq, tw):
        Kx = jv(ell, np.multiply.outer(xq, sv.yn)) * CTF(sv.yn, t)[None, :]
        Ux = (Kx @ (np.sqrt(sv.yw)[:, None] * sv.Vt[:h].T)) / sv.sigma[:h]  # (x, eta)
        K = jv(ell, np.multiply.outer(xq, yq)) * CTF(yq, t)[None, :]
        resid += wt * float(np.sum(xw[:, None] * yw[None, :] * (K - Ux @ SV.T) ** 2))
    tail = float(np.sum(sv.sigma[h:] ** 2))
    assert math.isclose(resid, tail, rel_tol=2e-2, abs_tol=1e-12)


def test_truncation_bound(plan32):
    # eq. Xmserr with the defocus as one more pose variable (uniform measure
    # of mass 1): || X - X_direct ||^2 over (delta, tau, gamma) <=
    # (2 pi Sigma_{H+1})^2 (2 pi)^2 int P_A P_B k dk
    n, Qa = 32, 64
    img = synth.white_noise_images(6, 2, n)
    r, wr = O.radial_quadrature(10, 2.0)
    om = 2 * math.pi * np.arange(20) / 20
    tq, tw = C.legendre_rule(8, T0, T1)
    pts, wts, taus = [], [], []
    for ri, wi in zip(r, wr):
        for o in om:
            for t, wt in zip(tq, tw):
                pts.append([ri * math.cos(o), ri * math.sin(o)])
                wts.append(wi * 2 * math.pi / 20 * wt * (2.0 / n) ** 2)
                taus.append(t)
    pts, wts, taus = np.array(pts), np.array(wts), np.array(taus)
    plan = C.set_poses(plan32, pts, taus)
    Ah, Bh = O.polar_ft(img[0], plan.k, Qa), O.polar_ft(img[1], plan.k, Qa)
    a, b = O.ring_coefficients(Ah), O.ring_coefficients(Bh)
    Xf = O.ftk_X(a, b, plan)
    Xd = C.direct_X_ctf(Ah, Bh, plan.k, plan.w, pts, taus, n, CTF, plan.kmax)
    err2 = float(np.sum(wts[:, None] * np.abs(Xf - Xd) ** 2) * 2 * math.pi / Qa)
    PA, PB = np.sum(np.abs(a) ** 2, axis=1), np.sum(np.abs(b) ** 2, axis=1)
    bound = (2 * math.pi * plan.sigma_next) ** 2 * (2 * math.pi) ** 2 * float(np.sum(plan.w * PA * PB))
    assert 0.0 < err2 <= bound


def test_planted_mistakes_fail(monkeypatch):
    # the frequency of pixel p taken as y / p instead of y / (2 p)
    assert _filter_error(2.0) > 1e-2
    # the defocus rule with weights of mass tmax - tmin instead of 1, planted
    # in the oracle's discretisation: the modal norm no longer matches
    rule = C.legendre_rule
    monkeypatch.setattr(C, "legendre_rule", lambda P, lo, hi: (rule(P, lo, hi)[0], rule(P, lo, hi)[1] * (hi - lo)))
    X = math.pi * 2.0
    s = C.ctf_modal_svd(0, X, CTF, T0, T1)
    want = quad(lambda x: x * quad(lambda y: jv(0, x * y) ** 2 * _mean_c2(y) * y, 0, 1, limit=400)[0], 0, X,
                limit=200)[0]
    assert not math.isclose(float(np.sum(s.sigma ** 2)), want, rel_tol=1e-2)
