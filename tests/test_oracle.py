"""Pins of the FP64 oracle against facts the paper and mathematics fix.

Every function of oracle.ftk is checked here against something other than
itself: printed values of the paper, closed forms (Gaussian Fourier
transforms and inner products, Lommel's integral, Jacobi-Anger), exact
identities (Parseval, Hermitian symmetry), the paper's bounds, and brute
force on tiny inputs.  A few tests plant a mistake in a copy of the oracle's
arithmetic and show that the pins catch it.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import jv

import synth
from oracle import ftk as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# --------------------------------------------------------------- quadrature

@pytest.mark.parametrize("M", [4, 16, 64])
def test_radial_quadrature_exact_for_polynomials(M):
    K = 0.5 * math.pi * 2 * M
    k, w = O.radial_quadrature(M, K)
    assert np.all((k > 0) & (k < K)) and np.all(w > 0)
    assert math.isclose(w.sum(), K * K / 2, rel_tol=1e-13)
    # int_0^K k^j k dk = K^(j+2)/(j+2), exact up to degree 2M-1
    for j in (1, M, 2 * M - 1):
        exact = K ** (j + 2) / (j + 2)
        assert math.isclose(np.sum(w * k ** j), exact, rel_tol=1e-10)


# ---------------------------------------------------------------- modal SVD

def test_paper_worked_example_ranks():
    g = _gold("paper_worked_example.json")
    keep, _, _ = O.truncation(g["R_px"], g["eps"])
    per_l = {}
    for l, e, s in keep:
        per_l[l] = per_l.get(l, 0) + 1
    for l, h in g["H_ell"].items():
        assert per_l[int(l)] == h
        assert per_l[-int(l)] == h
    capped, _, _ = O.truncation(g["R_px"], g["eps"], lmax=8)
    assert len(capped) == g["H_total"]
    assert len(keep) == 36  # every Sigma > eps kept (the reading used throughout)


@pytest.mark.parametrize("R", [2.0, 4.0])
def test_total_hs_norm_closed_form(R):
    # sum_l int int J_l(xy)^2 x dx y dy = (X^2/2)(1/2) since sum_l J_l^2 = 1
    X = math.pi * R
    tot = sum(float(np.sum(O.singular_values(l, X) ** 2)) for l in range(-60, 61))
    W = R / 2
    assert math.isclose(tot, math.pi ** 2 * W ** 2, rel_tol=1e-11)


@pytest.mark.parametrize("ell", [0, 1, 4, 9])
def test_modal_hs_norm_lommel(ell):
    X = math.pi * 4.0
    s = O.singular_values(ell, X)
    assert math.isclose(float(np.sum(s ** 2)), O.hs_norm_sq_modal(ell, X), rel_tol=1e-10)


def test_svd_converged_and_symmetric():
    X = math.pi * 4.0
    for ell in (0, 5, 13):
        a = O.singular_values(ell, X)
        b = O.singular_values(ell, X, P=2 * O.svd_nodes(X))
        assert np.max(np.abs(a[:20] - b[:20])) < 1e-12
        c = O.singular_values(-ell, X)
        assert np.max(np.abs(a - c)) < 1e-13
    # singular values depend on W only (Section 4.5): the Kmax, D scaling is
    # absorbed into x = Kmax delta, so the same X gives the same Sigma


@pytest.mark.parametrize("R,eps", [(2.0, 1e-2), (2.0, 1e-5), (4.0, 1e-3), (8.0, 1e-3)])
def test_rank_lemma_bound(R, eps):
    keep, _, dropped = O.truncation(R, eps)
    assert dropped <= eps
    per_l = {}
    for l, e, s in keep:
        per_l[l] = per_l.get(l, 0) + 1
    for l, h in per_l.items():
        assert h <= O.rank_lemma_bound(l, R / 2, eps) + 1e-12
    # Theorem t:rank: H <= 2 cH^2 with cH = max(pi e^2 W, log(2 pi W/eps)) + 3/2
    cH = max(math.pi * math.e ** 2 * R / 2, math.log(2 * math.pi * (R / 2) / eps)) + 1.5
    assert len(keep) <= 2 * cH * cH


def test_empirical_rank_fit_loose():
    # Remark after Lemma l:rank: H_l ~ 2.0 (W - |l|/(2 pi)) + 0.5 log(1/eps);
    # the log base is unstated, so only a +-30% agreement of H_0 is asked.
    for R, eps in [(4.0, 1e-3), (8.0, 1e-3), (4.0, 1e-6)]:
        keep, _, _ = O.truncation(R, eps)
        h0 = sum(1 for l, e, s in keep if l == 0)
        fit = 2.0 * (R / 2) + 0.5 * math.log(1 / eps)
        assert 0.7 * fit <= h0 <= 1.3 * fit + 1


def test_truncated_factors_reconstruct_kernel():
    # eq. efrob per l: || J_l - sum_{eta<=H} u sigma v ||_HS^2 = sum_{eta>H} sigma^2,
    # measured on an independent fine grid with the Nystrom-evaluated factors.
    R, eps = 4.0, 1e-3
    X = math.pi * R
    plan = O.make_plan(128, 64, 256, R, eps)
    xq, xw = O.radial_quadrature(120, X)
    yq, yw = O.radial_quadrature(120, 1.0)
    for ell in (0, 3, -7):
        sv = plan.svds[ell]
        zs = [z for z in range(plan.H) if plan.ell[z] == ell]
        approx = np.zeros((xq.size, yq.size))
        for z in zs:
            e = int(plan.eta[z])
            approx += np.outer(sv.u(e, xq), sv.sigma_v(e, yq))
        resid = jv(ell, np.outer(xq, yq)) - approx
        hs2 = float(np.sum(xw[:, None] * yw[None, :] * resid ** 2))
        tail = float(np.sum(sv.sigma[len(zs):] ** 2))
        assert math.isclose(hs2, tail, rel_tol=1e-3, abs_tol=1e-14)
        assert sv.sigma[len(zs)] <= eps < sv.sigma[len(zs) - 1]


def test_g_rows_match_nystrom_and_negative_l_sign():
    # J_{-l} = (-1)^l J_l, so the (-l) factorisation reproduces the same kernel
    plan = O.make_plan(32, 16, 64, 2.0, 1e-3)
    plan = O.set_shifts(plan, synth.shift_lattice(2.0))
    y = plan.k / plan.kmax
    x = math.pi * np.hypot(plan.shifts[:, 0], plan.shifts[:, 1])
    om = np.arctan2(plan.shifts[:, 1], plan.shifts[:, 0])
    # f(delta, k_m; l) = J_l(delta k_m) exp(-i l (omega + pi/2)), eq. fdef
    for ell in (-3, 0, 2, 5):
        zs = [z for z in range(plan.H) if plan.ell[z] == ell]
        approx = plan.Y[:, zs] @ plan.g[zs, :]
        exact = jv(ell, np.outer(x, y)) * np.exp(-1j * ell * (om + math.pi / 2))[:, None]
        assert np.max(np.abs(approx - exact)) < 30 * plan.eps


# --------------------------------------------------------------- transform

def _blob_ft(bs, k, psi, n):
    dx = 2.0 / n
    kx = np.multiply.outer(k, np.cos(psi))
    ky = np.multiply.outer(k, np.sin(psi))
    out = 0
    for c, s, a in zip(bs.centers, bs.sigmas, bs.amps):
        s, c = s * dx, c * dx
        out = out + a * 2 * math.pi * s * s * np.exp(-(kx ** 2 + ky ** 2) * s * s / 2) \
            * np.exp(-1j * (kx * c[0] + ky * c[1]))
    return out


def test_polar_ft_matches_gaussian_fourier_transform():
    rng = np.random.default_rng(11)
    n = 64
    bs = synth.random_blobs(rng, 6, 8.0, (2.0, 3.0))
    img = synth.render(bs, n)
    k, w = O.radial_quadrature(32, math.pi * n / 2)
    Ah = O.polar_ft(img, k, 128)
    ref = _blob_ft(bs, k, O.polar_angles(128), n)
    assert np.max(np.abs(Ah - ref)) < 1e-9 * np.max(np.abs(ref))
    # DC term: Ahat(0) = dx^2 sum A
    Ah0 = O.polar_ft(img, np.array([0.0]), 8)
    assert np.allclose(Ah0, (2 / n) ** 2 * img.sum(), rtol=1e-14)


def test_fb_coefficients_jacobi_anger_closed_form():
    # one blob: a(k;q) = 2 pi s^2 exp(-k^2 s^2/2) J_q(k|c|) exp(-i q (phi_c + pi/2))
    n = 64
    bs = synth.BlobSet(np.array([[5.0, -3.0]]), np.array([2.5]), np.array([1.0]))
    img = synth.render(bs, n)
    k, _ = O.radial_quadrature(16, math.pi * n / 2)
    a = O.ring_coefficients(O.polar_ft(img, k, 128))
    dx = 2 / n
    s, c = 2.5 * dx, np.array([5.0, -3.0]) * dx
    q = O.signed_modes(128)
    ref = (2 * math.pi * s * s * np.exp(-k ** 2 * s * s / 2))[:, None] \
        * jv(q[None, :], np.outer(k, np.hypot(*c)) * np.ones((1, q.size))) \
        * np.exp(-1j * q * (math.atan2(c[1], c[0]) + math.pi / 2))[None, :]
    assert np.max(np.abs(a - ref)) < 1e-9 * np.max(np.abs(ref))


def test_ring_coefficients_invert_by_fourier_series():
    rng = np.random.default_rng(2)
    Ah = rng.standard_normal((5, 32)) + 1j * rng.standard_normal((5, 32))
    a = O.ring_coefficients(Ah)
    psi = O.polar_angles(32)
    back = a @ np.exp(1j * np.multiply.outer(O.signed_modes(32), psi))
    assert np.allclose(back, Ah, atol=1e-13)


def test_real_image_coefficients_are_hermitian():
    # a(k;-q) = (-1)^q conj a(k;q) for real images
    img = synth.white_noise_images(5, 1, 32)[0]
    k, _ = O.radial_quadrature(16, math.pi * 16)
    a = O.ring_coefficients(O.polar_ft(img, k, 64))
    q = O.signed_modes(64)
    for qi in range(1, 31):
        neg = np.where(q == -q[qi])[0][0]
        assert np.allclose(a[:, neg], (-1) ** q[qi] * np.conj(a[:, qi]), atol=1e-13)


# ------------------------------------------------------------ inner products

def _blob_pair(seed, n=64, nb=5):
    rng = np.random.default_rng(seed)
    A = synth.random_blobs(rng, nb, 6.0, (2.0, 2.5))
    B = synth.random_blobs(rng, nb, 6.0, (2.0, 2.5))
    return A, B, synth.render(A, n), synth.render(B, n)


def _closed_form_ip(bsA, bsB, d_px, gamma, n):
    """(2 pi)^2 <R_gamma T_delta A, B> for continuous blob sums."""
    dx = 2.0 / n
    c, s_ = math.cos(gamma), math.sin(gamma)
    rot = np.array([[c, -s_], [s_, c]])
    tot = 0.0
    for ca, sa, aa in zip(bsA.centers, bsA.sigmas, bsA.amps):
        cp = rot @ ((ca + d_px) * dx)
        sa = sa * dx
        for cb, sb, ab in zip(bsB.centers, bsB.sigmas, bsB.amps):
            sb, cb = sb * dx, cb * dx
            v = sa * sa + sb * sb
            tot += aa * ab * 2 * math.pi * sa * sa * sb * sb / v * math.exp(-np.sum((cp - cb) ** 2) / (2 * v))
    return (2 * math.pi) ** 2 * tot


@pytest.fixture(scope="module")
def blob_case():
    n = 64
    A, B, Ai, Bi = _blob_pair(3, n)
    plan = O.make_plan(n, 32, 128, 2.0, 1e-8)
    shifts = synth.shift_lattice(2.0)
    plan = O.set_shifts(plan, shifts)
    Ah = O.polar_ft(Ai, plan.k, plan.Qa)
    Bh = O.polar_ft(Bi, plan.k, plan.Qa)
    Xd = O.direct_X(Ah, Bh, plan.k, plan.w, shifts, n)
    return dict(n=n, A=A, B=B, Ai=Ai, Bi=Bi, plan=plan, shifts=shifts, Ah=Ah, Bh=Bh, Xd=Xd)


def test_parseval_at_zero_pose(blob_case):
    c = blob_case
    i0 = int(np.where((c["shifts"] == 0).all(1))[0][0])
    dx = 2 / c["n"]
    ref = (2 * math.pi) ** 2 * dx * dx * float(np.sum(c["Ai"] * c["Bi"]))
    assert math.isclose(c["Xd"][i0, 0].real, ref, rel_tol=1e-11)


def test_direct_matches_closed_form_gaussian_inner_product(blob_case):
    c = blob_case
    scale = np.max(np.abs(c["Xd"]))
    for s in (0, 7, 24, 48):
        for r in (0, 9, 64, 127):
            ref = _closed_form_ip(c["A"], c["B"], c["shifts"][s], 2 * math.pi * r / 128, c["n"])
            assert abs(c["Xd"][s, r].real - ref) < 1e-11 * scale


def test_direct_matches_pixel_brute_force():
    # (2 pi)^2 dx^2 sum_ij (R_g T_d A)(x_ij) B(x_ij), A moved analytically
    n = 32
    A, B, Ai, Bi = _blob_pair(8, n, 3)
    # polar rule fine enough that the discretisation error is at rounding level
    k, w = O.radial_quadrature(32, math.pi * n / 2)
    shifts = np.array([[0.5, -1.0], [1.5, 0.0], [0.0, 0.0]])
    Xd = O.direct_X(O.polar_ft(Ai, k, 128), O.polar_ft(Bi, k, 128), k, w, shifts, n)
    dx = 2 / n
    for s in range(3):
        for r in (0, 13, 40, 101):
            g = 2 * math.pi * r / 128
            moved = synth.BlobSet(A.centers + shifts[s], A.sigmas, A.amps).moved(g, (0, 0))
            ref = (2 * math.pi) ** 2 * dx * dx * float(np.sum(synth.render(moved, n) * Bi))
            assert abs(Xd[s, r].real - ref) < 1e-12 * abs(Xd).max()


def test_direct_is_real_and_equivariant():
    n = 32
    img = synth.white_noise_images(21, 2, n)
    k, w = O.radial_quadrature(16, math.pi * n / 2)
    Ah, Bh = O.polar_ft(img[0], k, 64), O.polar_ft(img[1], k, 64)
    sh = synth.shift_lattice(1.0)
    X = O.direct_X(Ah, Bh, k, w, sh, n)
    assert np.max(np.abs(X.imag)) < 1e-12 * np.max(np.abs(X))
    # rotation: Bhat(psi) -> Bhat(psi - 2 pi r1/Qa) moves r -> r + r1
    r1 = 5
    X2 = O.direct_X(Ah, np.roll(Bh, r1, axis=1), k, w, sh, n)
    assert np.allclose(X2, np.roll(X, r1, axis=1), atol=1e-12 * np.abs(X).max())
    # translation: Ahat * exp(-i k . d1) gives X(delta + d1)
    d1 = np.array([0.5, 0.0])
    psi = O.polar_angles(64)
    ph = np.exp(-1j * (2 / n) * (np.outer(k, np.cos(psi)) * d1[0] + np.outer(k, np.sin(psi)) * d1[1]))
    X3 = O.direct_X(Ah * ph, Bh, k, w, np.array([[0.0, 0.0]]), n)
    i1 = int(np.where(np.all(np.isclose(sh, d1), axis=1))[0][0])
    assert np.allclose(X3[0], X[i1], atol=1e-12 * np.abs(X).max())


def test_ftk_untruncated_kernel_equals_direct_exactly():
    # with the exact Bessel kernel (eq. fastrots) and cyclic q - l the FB
    # formula is the polar-grid product itself
    n = 32
    img = synth.white_noise_images(4, 2, n)
    plan = O.make_plan(n, 16, 64, 2.0, 1e-3)
    plan = O.set_shifts(plan, synth.shift_lattice(2.0))
    Ah, Bh = O.polar_ft(img[0], plan.k, 64), O.polar_ft(img[1], plan.k, 64)
    a, b = O.ring_coefficients(Ah), O.ring_coefficients(Bh)
    Xb = O.bft_X(a, b, plan, 31)
    Xd = O.direct_X(Ah, Bh, plan.k, plan.w, plan.shifts, n)
    assert np.max(np.abs(Xb - Xd)) < 1e-12 * np.max(np.abs(Xd))


def _delta_rms_quadrature(R, n, nr=12, nw=24):
    """Polar Gauss x trapezoid rule on the shift disk (pixels): points and
    area weights in the paper's units (dx^2 per px^2)."""
    r, wr = O.radial_quadrature(nr, R)
    om = 2 * math.pi * np.arange(nw) / nw
    pts = np.array([[ri * math.cos(o), ri * math.sin(o)] for ri in r for o in om])
    wts = np.array([wi * 2 * math.pi / nw for wi in wr for o in om]) * (2.0 / n) ** 2
    return pts, wts


@pytest.mark.parametrize("kind", ["blobs", "noise"])
def test_ftk_error_within_truncation_bound(kind):
    # Section 5.2 eq. Xmserr with the 2D operator norm 2 pi Sigma_{H+1} and the
    # last factor (2 pi)^2 int P_A P_B k dk, P_A(k) = sum_q |a(k;q)|^2
    n, R = 32, 2.0
    if kind == "blobs":
        s = synth.workload_set("plain_n32", 7, n_images=1, n_templates=1)
        A, B = s.images[0], s.templates[0]
    else:
        A, B = synth.white_noise_images(9, 2, n)
    errs = []
    for eps in (1e-2, 1e-3, 1e-5):
        plan = O.make_plan(n, 16, 64, R, eps)
        pts, wts = _delta_rms_quadrature(R, n)
        plan = O.set_shifts(plan, pts)
        Ah, Bh = O.polar_ft(A, plan.k, 64), O.polar_ft(B, plan.k, 64)
        a, b = O.ring_coefficients(Ah), O.ring_coefficients(Bh)
        Xf = O.ftk_X(a, b, plan)
        Xd = O.direct_X(Ah, Bh, plan.k, plan.w, pts, n)
        # L2 over Omega_D x [0, 2 pi)
        err2 = float(np.sum(wts[:, None] * np.abs(Xf - Xd) ** 2) * 2 * math.pi / 64)
        PA = np.sum(np.abs(a) ** 2, axis=1)
        PB = np.sum(np.abs(b) ** 2, axis=1)
        last = (2 * math.pi) ** 2 * float(np.sum(plan.w * PA * PB))
        bound = (2 * math.pi * plan.sigma_next) ** 2 * last
        assert err2 <= bound
        errs.append(math.sqrt(err2))
    assert errs[0] > errs[1] > errs[2]


def test_ftk_matches_direct_to_eps_scale():
    n = 32
    s = synth.workload_set("plain_n32", 1, n_images=2, n_templates=2)
    plan = O.make_plan(n, 16, 64, 2.0, 1e-3)
    plan = O.set_shifts(plan, synth.shift_lattice(2.0))
    for A in s.images:
        for B in s.templates:
            Ah, Bh = O.polar_ft(A, plan.k, 64), O.polar_ft(B, plan.k, 64)
            a, b = O.ring_coefficients(Ah), O.ring_coefficients(Bh)
            Xf = O.ftk_X(a, b, plan)
            Xd = O.direct_X(Ah, Bh, plan.k, plan.w, plan.shifts, n)
            sc = O.pair_scale(a, b, plan)
            assert O.rel_err(Xf, Xd, sc) < 2 * plan.eps
            assert np.max(np.abs(Xf.imag)) < 1e-12 * sc
            assert np.max(np.abs(Xd)) <= sc * (1 + 1e-9)  # Cauchy-Schwarz


def test_pose_recovery_noise_free():
    # the paper's consistency check: the maximum sits at the true template
    # and next to the generating pose (delta, gamma) = (-s, -theta)
    n, Qa = 32, 64
    s = synth.make_alignment_set(5, n, 3, 4, 20, 2.0, None, sigma_px=(1.5, 3.0))
    plan = O.make_plan(n, 16, Qa, 2.0, 1e-3)
    plan = O.set_shifts(plan, synth.shift_lattice(2.0))
    bcoef = [O.fb_coefficients(t, plan) for t in s.templates]
    for ia, A in enumerate(s.images):
        a = O.fb_coefficients(A, plan)
        best = None
        for ib, b in enumerate(bcoef):
            v, si, ri, _ = O.best_pose(O.ftk_X(a, b, plan))
            if best is None or v > best[0]:
                best = (v, ib, si, ri)
        _, ib, si, ri = best
        assert ib == s.true_template[ia]
        d = plan.shifts[si] - (-s.true_shift[ia])
        assert np.hypot(*d) <= 0.5 * math.sqrt(2) + 1e-9
        g = (-s.true_theta[ia]) % (2 * math.pi)
        dg = abs((2 * math.pi * ri / Qa - g + math.pi) % (2 * math.pi) - math.pi)
        assert dg <= 2 * math.pi / Qa + 1e-9


def test_best_pose_tie_rule():
    X = np.zeros((3, 4))
    X[1, 2] = X[2, 0] = X[1, 3] = 5.0
    v, si, ri, margin = O.best_pose(X)
    assert (v, si, ri, margin) == (5.0, 1, 2, 0.0)


# ------------------------------------------------- planted mistakes are caught

def test_planted_mistakes_fail_the_pins():
    n = 32
    img = synth.white_noise_images(4, 2, n)
    plan = O.make_plan(n, 16, 64, 2.0, 1e-5)
    plan = O.set_shifts(plan, synth.shift_lattice(2.0))
    Ah, Bh = O.polar_ft(img[0], plan.k, 64), O.polar_ft(img[1], plan.k, 64)
    a, b = O.ring_coefficients(Ah), O.ring_coefficients(Bh)
    Xd = O.direct_X(Ah, Bh, plan.k, plan.w, plan.shifts, n)
    sc = O.pair_scale(a, b, plan)
    assert O.rel_err(O.ftk_X(a, b, plan), Xd, sc) < 1e-4
    import copy
    # (1) wrong sign of the shift phase omega in Y
    bad = copy.copy(plan)
    bad.Y = np.conj(plan.Y) * np.exp(-1j * plan.ell * math.pi)[None, :]
    assert O.rel_err(O.ftk_X(a, b, bad), Xd, sc) > 1e-2
    # (2) q + l instead of q - l
    bad = copy.copy(plan)
    bad.ell = -plan.ell
    assert O.rel_err(O.ftk_X(a, b, bad), Xd, sc) > 1e-2
    # (3) dropped radial weight
    bad = copy.copy(plan)
    bad.w = np.ones_like(plan.w) * plan.w.mean()
    assert O.rel_err(O.ftk_X(a, b, bad), Xd, sc) > 1e-2


def test_lattice_counts_golden():
    g = _gold("lattice_counts.json")
    for R, cnt in g["counts"].items():
        assert len(synth.shift_lattice(float(R))) == cnt


# ------------------------------------------ error scale and pose margin, exact

def _scale_pin_devs(scale_fn, c):
    """Relative deviations of a pair-scale function from what fixes it
    exactly: s_AA = Re X_dir,AA(0, 0) (the direct polar inner product of
    eq. Xdg at zero shift and rotation, with no Fourier-Bessel step),
    s_AB^2 = X_AA(0, 0) X_BB(0, 0), and, for band-limited blobs, Parseval's
    (2 pi)^2 dx^2 sum_ij A_ij^2 (eq. planch)."""
    plan, n = c["plan"], c["n"]
    a, b = O.ring_coefficients(c["Ah"]), O.ring_coefficients(c["Bh"])
    zero = np.zeros((1, 2))
    xaa = float(O.direct_X(c["Ah"], c["Ah"], plan.k, plan.w, zero, n)[0, 0].real)
    xbb = float(O.direct_X(c["Bh"], c["Bh"], plan.k, plan.w, zero, n)[0, 0].real)
    dx = 2.0 / n
    pars = (2 * math.pi) ** 2 * dx * dx * float(np.sum(c["Ai"] ** 2))
    return [abs(scale_fn(a, a, plan) - xaa) / xaa,
            abs(scale_fn(b, b, plan) - xbb) / xbb,
            abs(scale_fn(a, b, plan) ** 2 - xaa * xbb) / (xaa * xbb),
            abs(scale_fn(a, a, plan) - pars) / pars]


def test_pair_scale_exact(blob_case):
    devs = _scale_pin_devs(O.pair_scale, blob_case)
    assert max(devs[:3]) < 1e-12, devs
    assert devs[3] < 1e-10, devs


def test_pair_scale_planted_mistakes_fail():
    # an extra 2 pi, a missing square root, a dropped radial weight: each must
    # break the exact pins (an overestimate would loosen every parity bar)
    n = 64
    A, B, Ai, Bi = _blob_pair(3, n)
    plan = O.make_plan(n, 32, 128, 2.0, 1e-8)
    c = dict(n=n, plan=plan, Ai=Ai, Ah=O.polar_ft(Ai, plan.k, 128), Bh=O.polar_ft(Bi, plan.k, 128))
    assert max(_scale_pin_devs(O.pair_scale, c)) < 1e-10
    bad = [lambda a, b, p: 2 * math.pi * O.pair_scale(a, b, p),
           lambda a, b, p: O.pair_scale(a, b, p) ** 2,
           lambda a, b, p: O.pair_scale(a, b, _replaced(p, w=np.full_like(p.w, p.w.mean())))]
    for f in bad:
        assert max(_scale_pin_devs(f, c)) > 1e-2


def _replaced(plan, **kw):
    import copy
    q = copy.copy(plan)
    for k, v in kw.items():
        setattr(q, k, v)
    return q


def _margin_pin(pose_fn):
    """Distinct values with a known best, position and margin; a large
    imaginary part that must not count (argmax of Re X)."""
    rng = np.random.default_rng(31)
    vals = rng.permutation(35).astype(np.float64) * 1.5 + 0.25  # 0.25, 1.75, ..., 51.25
    X = vals.reshape(5, 7) + 1j * rng.uniform(-200, 200, (5, 7))
    where = int(np.argmax(vals))
    v, si, ri, margin = pose_fn(X)
    return (v, si, ri, margin) == (51.25, where // 7, where % 7, 1.5)


def test_best_pose_margin_exact():
    assert _margin_pin(O.best_pose)
    # a single pose has no second best: infinite margin
    assert O.best_pose(np.array([[3.0]]))[3] == np.inf


def test_best_pose_planted_mistakes_fail():
    def second_equals_best(X):
        v, si, ri, _ = O.best_pose(X)
        return v, si, ri, 0.0

    def magnitude(X):
        return O.best_pose(np.abs(X))

    def swapped_indices(X):
        v, si, ri, m = O.best_pose(X)
        return v, ri, si, m

    for f in (second_equals_best, magnitude, swapped_indices):
        assert not _margin_pin(f)
