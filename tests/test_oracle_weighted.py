"""Pins of the oracle's weighted operator SVD (Section 4.5, the remark on
alternative weight functions: the k-side measure k dk becomes p(k) k dk).

The weight is a sum of Gaussians in k / Kmax, scaled to mean 1 over the
disk; the workload's is the expected power spectrum of its blob templates.  Pinned by: a constant weight giving the
paper's SVD; the closed form of the total Hilbert-Schmidt norm (pi^2 W^2 for
every weight, since sum_l J_l^2 = 1); the per-mode norm by independent
quadrature; the truncation bound of eq. Xmserr with the weighted operator
norm (last factor (2 pi)^2 int P_A P_B / p k dk); and planted mistakes.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import jv

import synth
from oracle import ftk as O

WEIGHT = synth.blob_power_spectrum()


def test_constant_weight_is_the_papers_svd():
    for R, eps in ((2.0, 1e-3), (4.0, 1e-5)):
        a = O.make_plan(32, 16, 64, R, eps)
        b = O.make_plan(32, 16, 64, R, eps, weight=([2.5, 0.5], [0.0, 0.0]))
        assert a.H == b.H and np.array_equal(a.ell, b.ell)
        assert np.max(np.abs(a.sigma - b.sigma) / a.sigma) < 1e-12
        assert np.max(np.abs(a.g - b.g)) < 1e-10 * np.max(np.abs(a.g))


def test_weight_normalised_to_disk_mean_one():
    p = O.weight_function(*WEIGHT)
    val, _ = quad(lambda y: p(y) * y, 0.0, 1.0, limit=200, epsabs=1e-15, epsrel=1e-13)
    assert math.isclose(val, 0.5, rel_tol=1e-12)
    with pytest.raises(ValueError):
        O.weight_function([1.0, -1.0], [0.0, 1.0])
    with pytest.raises(ValueError):
        O.weight_function([0.0], [1.0])


@pytest.mark.parametrize("R", [2.0, 4.0])
def test_weighted_total_hs_norm_closed_form(R):
    # sum_l int int J_l(xy)^2 x dx p(y) y dy = (X^2/2) int p y dy = X^2/4 = pi^2 W^2
    X = math.pi * R
    p = O.weight_function(*WEIGHT)
    tot = sum(float(np.sum(O.singular_values(l, X, weight=p) ** 2)) for l in range(-60, 61))
    assert math.isclose(tot, math.pi ** 2 * (R / 2) ** 2, rel_tol=1e-9)


@pytest.mark.parametrize("ell", [0, 2, 7])
def test_weighted_modal_hs_norm_by_quadrature(ell):
    X = math.pi * 4.0
    p = O.weight_function(*WEIGHT)
    s = O.singular_values(ell, X, weight=p)

    def inner(x):
        v, _ = quad(lambda y: jv(ell, x * y) ** 2 * p(y) * y, 0.0, 1.0, limit=200, epsabs=1e-15, epsrel=1e-12)
        return v * x

    ref, _ = quad(inner, 0.0, X, limit=200, epsabs=1e-13, epsrel=1e-11)
    assert math.isclose(float(np.sum(s ** 2)), ref, rel_tol=1e-8)


def test_weighted_rank_is_smaller():
    for R, eps in ((4.0, 1e-3), (4.0, 1e-5), (8.0, 1e-3)):
        a = O.make_plan(128, 64, 256, R, eps)
        b = O.make_plan(128, 64, 256, R, eps, weight=WEIGHT)
        assert b.H < a.H, (R, eps, a.H, b.H)


def _quad_disk(R, n, nr=24, nw=48):
    r, wr = O.radial_quadrature(nr, R)
    om = 2 * math.pi * np.arange(nw) / nw
    pts = np.array([[ri * math.cos(o), ri * math.sin(o)] for ri in r for o in om])
    wts = np.array([wi * 2 * math.pi / nw for wi in wr for o in om]) * (2.0 / n) ** 2
    return pts, wts


def _error_and_bound(plan, A, B, n, Qa, p):
    pts, wts = _quad_disk(plan.R, n)
    plan = O.set_shifts(plan, pts)
    Ah, Bh = O.polar_ft(A, plan.k, Qa), O.polar_ft(B, plan.k, Qa)
    a, b = O.ring_coefficients(Ah), O.ring_coefficients(Bh)
    Xf = O.ftk_X(a, b, plan)
    Xd = O.direct_X(Ah, Bh, plan.k, plan.w, pts, n)
    err2 = float(np.sum(wts[:, None] * np.abs(Xf - Xd) ** 2) * 2 * math.pi / Qa)
    PA = np.sum(np.abs(a) ** 2, axis=1)
    PB = np.sum(np.abs(b) ** 2, axis=1)
    last = (2 * math.pi) ** 2 * float(np.sum(plan.w * PA * PB / p(plan.k / plan.kmax)))
    return err2, (2 * math.pi * plan.sigma_next) ** 2 * last


@pytest.mark.parametrize("kind", ["blobs", "noise"])
def test_weighted_ftk_error_within_truncation_bound(kind):
    # eq. Xmserr with the weighted operator: the error kernel maps L2(p k dk)
    # to L2(delta d delta) with norm Sigma_{H+1}, so the last factor becomes
    # (2 pi)^2 int P_A P_B / p k dk
    n, R, Qa = 32, 2.0, 64
    if kind == "blobs":
        s = synth.workload_set("plain_n32", 7, n_images=1, n_templates=1)
        A, B = s.images[0], s.templates[0]
    else:
        A, B = synth.white_noise_images(9, 2, n)
    p = O.weight_function(*WEIGHT)
    errs = []
    for eps in (1e-2, 1e-3, 1e-5):
        plan = O.make_plan(n, 16, Qa, R, eps, weight=WEIGHT)
        err2, bound = _error_and_bound(plan, A, B, n, Qa, p)
        assert err2 <= bound
        errs.append(math.sqrt(err2))
    assert errs[0] > errs[1] > errs[2]


def _weighted_residual(sv, h, p, ell):
    """|| J_l - sum_{eta < h} u sigma v ||^2 in the k-weighted norm
    (x dx, p(y) y dy) on a fine grid independent of the SVD's nodes."""
    xq, xw = O.radial_quadrature(120, sv.X)
    yq, yw = O.radial_quadrature(120, 1.0)
    approx = np.zeros((xq.size, yq.size))
    for e in range(h):
        approx += np.outer(sv.u(e, xq), sv.sigma_v(e, yq))
    resid = jv(ell, np.outer(xq, yq)) - approx
    return float(np.sum(xw[:, None] * (yw * p(yq))[None, :] * resid ** 2))


def test_weighted_factors_reconstruct_kernel():
    # eq. efrob in the weighted norm: || J_l - sum_{eta<=H} ||^2 = sum_{eta>H} Sigma^2
    R, eps = 4.0, 1e-3
    p = O.weight_function(*WEIGHT)
    plan = O.make_plan(128, 64, 256, R, eps, weight=WEIGHT)
    for ell in (0, 3, -5):
        sv = plan.svds[ell]
        h = int(np.sum(plan.ell == ell))
        tail = float(np.sum(sv.sigma[h:] ** 2))
        assert math.isclose(_weighted_residual(sv, h, p, ell), tail, rel_tol=1e-3, abs_tol=1e-14)


def test_weighted_planted_mistakes_fail():
    X, ell = math.pi * 4.0, 2
    p = O.weight_function(*WEIGHT)
    P = O.svd_nodes(X)
    xn, xw = O.radial_quadrature(P, X)
    yn, yw = O.radial_quadrature(P, 1.0)
    J = jv(ell, np.multiply.outer(xn, yn))
    # (1) the weight on the shift side: the Hilbert-Schmidt norm is the same
    # (swap x and y), but its truncation no longer reconstructs the kernel in
    # the k-weighted norm
    wx = xw * p(xn / X)
    U, sg, Vt = np.linalg.svd(np.sqrt(wx)[:, None] * J * np.sqrt(yw)[None, :])
    bad = O.ModalSVD(ell, X, sg, U, Vt, xn, wx, yn, yw)
    h = int(np.sum(sg > 1e-3))
    tail = float(np.sum(sg[h:] ** 2))
    assert not math.isclose(_weighted_residual(bad, h, p, ell), tail, rel_tol=0.5)
    # (2) the weight without its square root in the matrix breaks the norm

    def inner(x):
        v, _ = quad(lambda y: jv(ell, x * y) ** 2 * p(y) * y, 0.0, 1.0, limit=200)
        return v * x

    ref, _ = quad(inner, 0.0, X, limit=200)
    s2 = np.linalg.svd(np.sqrt(xw)[:, None] * J * (yw * p(yn))[None, :], compute_uv=False)
    assert not math.isclose(float(np.sum(s2 ** 2)), ref, rel_tol=1e-3)
