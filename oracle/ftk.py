"""FP64 oracle of the FTK hot path (plain, slow, written from the paper).

TEST INFRASTRUCTURE ONLY -- the product path never imports this module.

Paper: Rangan, Spivak, Anden, Barnett, "Factorization of the translation
kernel for fast rigid image alignment" (arXiv 1905.12317).

Everything is FP64.  Library primitives used as single steps: SciPy's
Gauss-Jacobi nodes (`roots_jacobi`), Bessel J (`jv`) and NumPy's dense SVD
and matrix products.  No blocking, fusion or reordering beyond what the
formulas state.

Units.  Images live on [-1,1]^2 with dx = 2/n; pixel (i,j) is at
(i dx - 1, j dx - 1) (Section 2.1, the pixel grid); Kmax = pi n / 2 is the
Nyquist frequency (Remark on Nyquist, Section 2).  Shifts are passed in
pixels; a shift of d pixels is d*dx in the paper's units, so
Kmax * |delta| = pi * |d|.  The maximum shift radius R (pixels) is 2W in the
paper's wavelength units.

Readings of the paper taken here (where it is silent, ambiguous or garbled):
  * pixel indices run 0..n-1 (Section 2.1 grid definition, not the 1..n of
    the trapezoid sum);
  * modes q run over -Qa/2..Qa/2-1 with Qa = 2Q angular samples
    (eq. aqkcalc), and a(k; q - l) is taken cyclically mod Qa: this makes
    eq. Xtrunc equal to the polar-grid product exactly;
  * rotations are gamma_r = 2 pi r / Qa, r = 0..Qa-1 (Step 2 of eq. fbk2);
  * X(delta, gamma) = <R_gamma T_delta A, B> with B conjugated (eq. Xtrunc);
  * every (l, eta) with Sigma_eta(l) > eps is kept, scanning |l| upward until
    Sigma_1(l) <= eps (Section 4.5 relabelling; Theorem t:rank).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import jv, roots_jacobi

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# Radial quadrature (Section 3.1, Gauss-Jacobi alpha=0, beta=1 for k dk)
# ---------------------------------------------------------------------------

def radial_quadrature(M: int, kmax: float):
    """Nodes k_m in [0, kmax] and weights w_m with int_0^kmax g k dk ~ sum w g.

    Gauss-Jacobi(alpha=0, beta=1) on t in [-1,1] integrates (1+t) h(t) dt;
    with k = kmax (1+t)/2 one has k dk = (kmax/2)^2 (1+t) dt.
    """
    t, wt = roots_jacobi(M, 0.0, 1.0)
    k = 0.5 * kmax * (1.0 + t)
    w = (0.5 * kmax) ** 2 * wt
    return k, w


# ---------------------------------------------------------------------------
# Operator SVD of the modal translation kernel (Section 4.5, eq. Jsvd and the
# remark on approximating it)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class ModalSVD:
    """SVD of J_l(x y) on x in [0, X] (weight x dx), y in [0, 1] (y dy).

    The discretisation is a Gauss-Jacobi(0,1) Nystrom matrix
    K_ij = sqrt(wx_i) J_l(x_i y_j) sqrt(wy_j); its singular values
    approximate the operator's and its singular vectors, divided by the
    square-root weights, sample the singular functions.
    """

    ell: int
    X: float
    sigma: np.ndarray  # (P,)
    Umat: np.ndarray  # (P, P) left vectors (x side), columns
    Vt: np.ndarray  # (P, P) right vectors (y side), rows
    xn: np.ndarray
    xw: np.ndarray
    yn: np.ndarray
    yw: np.ndarray  # y-side quadrature weights times the weight function p(y_j)

    def sigma_v(self, eta: int, y) -> np.ndarray:
        """Sigma_eta * v_eta(y) at any y in [0,1] (Nystrom, no division)."""
        y = np.asarray(y, dtype=np.float64)
        J = jv(self.ell, np.multiply.outer(y, self.xn))  # (..., P)
        return J @ (np.sqrt(self.xw) * self.Umat[:, eta])

    def u(self, eta: int, x) -> np.ndarray:
        """u_eta(x) at any x in [0, X] (Nystrom through the y side; the y-side
        measure p(y) y dy is in yw)."""
        x = np.asarray(x, dtype=np.float64)
        J = jv(self.ell, np.multiply.outer(x, self.yn))  # (..., P)
        return (J @ (np.sqrt(self.yw) * self.Vt[eta, :])) / self.sigma[eta]


def svd_nodes(X: float) -> int:
    """Nystrom size used by the oracle: generous, then checked by doubling."""
    return int(math.ceil(2.0 * X)) + 48


def weight_function(alpha, beta=None):
    """The k-side weight p(y), y = k / Kmax in [0, 1], of the remark on
    alternative weight functions (Section 4.5): a sum of Gaussians
    p(y) = c sum_j alpha_j exp(-beta_j y^2) (alpha_j >= 0 and not all zero,
    beta_j >= 0), with c such that its mean over the unit disk is 1,
    int_0^1 p(y) y dy = 1/2 (each term integrates to
    alpha (1 - exp(-beta)) / (2 beta), alpha / 2 at beta = 0).  alpha None:
    p = 1, the paper's weight (the L2 norm over the disk).  With this scaling
    the sum of every Sigma^2 stays pi^2 W^2 for any weight."""
    if alpha is None:
        return None
    a = np.asarray(alpha, dtype=np.float64).ravel()
    b = np.asarray(beta, dtype=np.float64).ravel()
    if a.size < 1 or a.size != b.size or not (np.all(np.isfinite(a)) and np.all(np.isfinite(b))):
        raise ValueError("weight: alpha and beta of equal length, finite")
    if np.any(a < 0) or np.any(b < 0) or not np.any(a > 0):
        raise ValueError("weight: alpha >= 0 (not all 0), beta >= 0")
    total = float(sum(aj * ((1.0 - math.exp(-bj)) / (2.0 * bj) if bj > 0 else 0.5) for aj, bj in zip(a, b)))
    c = 0.5 / total
    def p(y):
        y = np.asarray(y, dtype=np.float64)
        t = a[:, None] * np.exp(-np.multiply.outer(b, y.ravel() ** 2))
        return c * np.sum(t, axis=0).reshape(y.shape)

    return p


def modal_svd(ell: int, X: float, P: int | None = None, weight=None) -> ModalSVD:
    """weight: None (p = 1) or a function p(y) from weight_function.  The SVD
    is that of J_l(x y) on x in [0, X] (x dx), y in [0, 1] (p(y) y dy)."""
    P = svd_nodes(X) if P is None else P
    xn, xw = radial_quadrature(P, X)
    yn, yw = radial_quadrature(P, 1.0)
    if weight is not None:
        yw = yw * weight(yn)
    K = np.sqrt(xw)[:, None] * jv(ell, np.multiply.outer(xn, yn)) * np.sqrt(yw)[None, :]
    U, s, Vt = np.linalg.svd(K)
    return ModalSVD(ell, X, s, U, Vt, xn, xw, yn, yw)


def singular_values(ell: int, X: float, P: int | None = None, weight=None) -> np.ndarray:
    return modal_svd(ell, X, P, weight).sigma


@dataclasses.dataclass
class Plan:
    """Truncated kernel factorisation plus the radial quadrature."""

    n: int
    M: int
    Qa: int
    R: float  # max shift radius in pixels
    eps: float
    kmax: float
    k: np.ndarray  # (M,)
    w: np.ndarray  # (M,)
    ell: np.ndarray  # (H,) int
    eta: np.ndarray  # (H,) int
    sigma: np.ndarray  # (H,)
    g: np.ndarray  # (H, M) Sigma_zeta v_zeta(k_m / kmax)
    svds: dict  # ell -> ModalSVD
    sigma_next: float  # largest discarded singular value
    weight: object = None  # the k-side weight function p(y), or None (p = 1)
    shifts: np.ndarray | None = None  # (N, 2) px
    Y: np.ndarray | None = None  # (N, H) complex

    @property
    def H(self) -> int:
        return int(self.ell.size)


def truncation(R: float, eps: float, lmax: int | None = None, P: int | None = None, weight=None):
    """(l, eta, sigma) of every kept term, the svds, and the first dropped value.

    Keeps Sigma_eta(l) > eps for l = 0, +-1, +-2, ... until Sigma_1(l) <= eps
    (or |l| > lmax when a cap is given).  weight: the k-side weight function
    (weight_function), or None.
    """
    X = math.pi * R
    svds, keep = {}, []
    dropped = 0.0
    ell = 0
    while True:
        if lmax is not None and ell > lmax:
            break
        sv = modal_svd(ell, X, P, weight)
        if sv.sigma[0] <= eps:
            dropped = max(dropped, sv.sigma[0])
            break
        signs = [ell] if ell == 0 else [ell, -ell]
        for l in signs:
            s = sv if l == ell else modal_svd(l, X, P, weight)
            svds[l] = s
            h = int(np.sum(s.sigma > eps))
            keep += [(l, e, s.sigma[e]) for e in range(h)]
            dropped = max(dropped, s.sigma[h] if h < s.sigma.size else 0.0)
        ell += 1
    if lmax is not None:
        sv = modal_svd(lmax + 1, X, P, weight)
        dropped = max(dropped, sv.sigma[0])
    return keep, svds, dropped


def make_plan(n: int, M: int, Qa: int, R: float, eps: float,
              lmax: int | None = None, P: int | None = None, weight=None) -> Plan:
    """weight: None (the paper's weight), or (alpha, beta) of the k-side
    weight sum_j alpha_j exp(-beta_j (k / Kmax)^2) (see weight_function)."""
    kmax = 0.5 * math.pi * n
    k, w = radial_quadrature(M, kmax)
    weight = None if weight is None else weight_function(*weight)
    keep, svds, dropped = truncation(R, eps, lmax, P, weight)
    keep.sort(key=lambda t: (t[0], t[1]))
    ell = np.array([t[0] for t in keep], dtype=np.int64)
    eta = np.array([t[1] for t in keep], dtype=np.int64)
    sig = np.array([t[2] for t in keep])
    y = k / kmax
    g = np.zeros((ell.size, M))
    for z, (l, e) in enumerate(zip(ell, eta)):
        g[z] = svds[int(l)].sigma_v(int(e), y)
    return Plan(n, M, Qa, R, eps, kmax, k, w, ell, eta, sig, g, svds, dropped, weight)


def set_shifts(plan: Plan, shifts_px: np.ndarray) -> Plan:
    """Y[delta, zeta] = u_zeta(Kmax |delta|) exp(-i l_zeta (omega + pi/2)).

    Section 4.5, the construction of Y^svd from the left singular functions.
    """
    shifts_px = np.asarray(shifts_px, dtype=np.float64).reshape(-1, 2)
    r = np.hypot(shifts_px[:, 0], shifts_px[:, 1])
    if np.any(r > plan.R * (1 + 1e-12)):
        raise ValueError("shift outside the planned disk")
    om = np.arctan2(shifts_px[:, 1], shifts_px[:, 0])
    x = math.pi * r  # Kmax * delta
    Y = np.zeros((shifts_px.shape[0], plan.H), dtype=np.complex128)
    for z, (l, e) in enumerate(zip(plan.ell, plan.eta)):
        u = plan.svds[int(l)].u(int(e), x)
        Y[:, z] = u * np.exp(-1j * l * (om + 0.5 * math.pi))
    plan.shifts = shifts_px
    plan.Y = Y
    return plan


# ---------------------------------------------------------------------------
# Transform: pixels -> polar Fourier samples -> Fourier-Bessel coefficients
# (Section 2.1 eq. Ahattrap; Section 3.2 eq. aqkcalc)
# ---------------------------------------------------------------------------

def polar_angles(Qa: int) -> np.ndarray:
    return TWO_PI * np.arange(Qa) / Qa


def polar_ft(img: np.ndarray, k: np.ndarray, Qa: int) -> np.ndarray:
    """Ahat(k_m, psi_p) = dx^2 sum_ij A_ij exp(-i k . x_ij), direct sum.

    img is (n, n) with the first index along x.  Returns (M, Qa) complex.
    """
    n = img.shape[0]
    dx = 2.0 / n
    xs = np.arange(n) * dx - 1.0
    psi = polar_angles(Qa)
    kx = np.multiply.outer(k, np.cos(psi))  # (M, Qa)
    ky = np.multiply.outer(k, np.sin(psi))
    Ex = np.exp(-1j * np.multiply.outer(kx, xs))  # (M, Qa, n_i)
    Ey = np.exp(-1j * np.multiply.outer(ky, xs))  # (M, Qa, n_j)
    # inner sum over j for every (m, p, i), then over i
    T = Ey @ img.T  # (M, Qa, n_i): sum_j Ey[m,p,j] A[i,j]
    return dx * dx * np.sum(Ex * T, axis=-1)


def signed_modes(Qa: int) -> np.ndarray:
    """Mode numbers in storage order: 0..Qa/2-1, then -Qa/2..-1."""
    q = np.arange(Qa)
    return np.where(q < Qa // 2, q, q - Qa)


def ring_coefficients(Ahat: np.ndarray) -> np.ndarray:
    """a(k_m; q) = (1/Qa) sum_p Ahat(k_m, psi_p) exp(-i q psi_p), eq. aqkcalc.

    Written as the explicit DFT sum; storage order of q is signed_modes().
    """
    Qa = Ahat.shape[1]
    q = signed_modes(Qa)
    psi = polar_angles(Qa)
    D = np.exp(-1j * np.multiply.outer(psi, q))  # (p, q)
    return (Ahat @ D) / Qa


def fb_coefficients(img: np.ndarray, plan: Plan) -> np.ndarray:
    return ring_coefficients(polar_ft(img, plan.k, plan.Qa))


# ---------------------------------------------------------------------------
# Inner products
# ---------------------------------------------------------------------------

def direct_X(Ahat: np.ndarray, Bhat: np.ndarray, k, w, shifts_px, n: int) -> np.ndarray:
    """Direct band-limited inner product on the polar quadrature (eq. Xdg).

    X(delta, r) = (2 pi / Qa) sum_m w_m sum_p F(delta, k_m, psi_p)
                  Ahat(k_m, psi_p) conj(Bhat(k_m, psi_{p+r})),
    F(delta, k) = exp(-i delta . k) (eq. Fdk), gamma_r = 2 pi r / Qa.
    No Fourier-Bessel expansion and no SVD.  Returns (N, Qa) complex.
    """
    M, Qa = Ahat.shape
    dx = 2.0 / n
    psi = polar_angles(Qa)
    d = np.asarray(shifts_px, dtype=np.float64).reshape(-1, 2) * dx
    N = d.shape[0]
    X = np.zeros((N, Qa), dtype=np.complex128)
    p = np.arange(Qa)
    for m in range(M):
        kx = k[m] * np.cos(psi)
        ky = k[m] * np.sin(psi)
        F = np.exp(-1j * (np.multiply.outer(d[:, 0], kx) + np.multiply.outer(d[:, 1], ky)))
        P = F * Ahat[m][None, :]  # (N, Qa) over p
        C = np.conj(Bhat[m][(p[:, None] + p[None, :]) % Qa])  # C[p, r] = conj B(p + r)
        X += w[m] * (P @ C)
    return X * (TWO_PI / Qa)


def ftk_zhat(a: np.ndarray, b: np.ndarray, plan: Plan) -> np.ndarray:
    """Step 1 of eq. fbk3 for every q (storage order):

    Zhat[zeta, q] = 2 pi sum_m w_m G_zeta(k_m) a(k_m; q - l_zeta) conj b(k_m; q)
    with q - l taken mod Qa.
    """
    M, Qa = a.shape
    Z = np.zeros((plan.H, Qa), dtype=np.complex128)
    idx = np.arange(Qa)
    for z in range(plan.H):
        l = int(plan.ell[z])
        ash = a[:, (idx - l) % Qa]  # a(k_m; q - l) in storage order (cyclic)
        Z[z] = TWO_PI * np.sum((plan.w * plan.g[z])[:, None] * ash * np.conj(b), axis=0)
    return Z


def ftk_X(a: np.ndarray, b: np.ndarray, plan: Plan) -> np.ndarray:
    """FP64 FTK (eq. fbk3): Step 1, then Step 3 (shift contraction), then the
    rotation sum X(delta, r) = sum_q exp(-i q gamma_r) Xhat(delta, q).

    Step 3 is applied before the rotation sum; both are linear so the order
    does not change the result.  Returns (N, Qa) complex.
    """
    Zh = ftk_zhat(a, b, plan)  # (H, Qa)
    Xh = plan.Y @ Zh  # (N, Qa)
    Qa = a.shape[1]
    q = signed_modes(Qa)
    gam = polar_angles(Qa)
    E = np.exp(-1j * np.multiply.outer(q, gam))  # (q, r)
    return Xh @ E


def ftk_xhat(a: np.ndarray, b: np.ndarray, plan: Plan) -> np.ndarray:
    """Xhat(delta, q) of eq. fbk3 (Step 1, then Step 3): (N, Qa), q in
    signed_modes() order."""
    return plan.Y @ ftk_zhat(a, b, plan)


def rotation_sum_upsampled(Xh: np.ndarray, U: int) -> np.ndarray:
    """Step 2 (eq. 1dfft) on a U times finer rotation grid, gamma_r =
    2 pi r / (U Qa), r = 0 .. U Qa - 1: the zero-padded angular sum of the
    remark after eq. 1dfft.  The Nyquist mode -Qa/2 enters as its cosine (half
    of it at each of +-Qa/2), so X stays real and, at every U-th angle, equals
    the sum on the Qa-point grid.  Xh: (N, Qa) in signed_modes() order."""
    N, Qa = Xh.shape
    q = signed_modes(Qa)
    gam = TWO_PI * np.arange(U * Qa) / (U * Qa)
    inner = q != -(Qa // 2)
    E = np.exp(-1j * np.multiply.outer(q[inner], gam))
    return Xh[:, inner] @ E + Xh[:, ~inner] * np.cos(0.5 * Qa * gam)[None, :]


def ftk_X_upsampled(a: np.ndarray, b: np.ndarray, plan: Plan, U: int) -> np.ndarray:
    """FP64 FTK with U Qa rotations: (N, U Qa) complex."""
    return rotation_sum_upsampled(ftk_xhat(a, b, plan), U)


def bft_X_upsampled(Ahat: np.ndarray, b: np.ndarray, plan: Plan, U: int) -> np.ndarray:
    """Brute-force translations with U Qa rotations: (N, U Qa) complex."""
    Ta = bft_translated_coefficients(Ahat, plan)
    Xh = TWO_PI * np.einsum("m,dmq,mq->dq", plan.w, Ta, np.conj(b))
    return rotation_sum_upsampled(Xh, U)


def bft_X(a: np.ndarray, b: np.ndarray, plan: Plan, lmax: int) -> np.ndarray:
    """FTK Steps 1-2 with the exact Bessel kernel (eq. fastrots), one shift at a
    time: the untruncated reference of the same cyclic discretisation."""
    M, Qa = a.shape
    idx = np.arange(Qa)
    q = signed_modes(Qa)
    gam = polar_angles(Qa)
    E = np.exp(-1j * np.multiply.outer(q, gam))
    dx = 2.0 / plan.n
    out = np.zeros((plan.shifts.shape[0], Qa), dtype=np.complex128)
    for s, (sx, sy) in enumerate(plan.shifts):
        delta = math.hypot(sx, sy) * dx
        om = math.atan2(sy, sx)
        Ta = np.zeros_like(a)
        for l in range(-lmax, lmax + 1):
            f = jv(l, delta * plan.k) * np.exp(-1j * l * (om + 0.5 * math.pi))
            Ta += f[:, None] * a[:, (idx - l) % Qa]
        Xh = TWO_PI * np.sum(plan.w[:, None] * Ta * np.conj(b), axis=0)
        out[s] = Xh @ E
    return out


def bft_translated_coefficients(Ahat: np.ndarray, plan: Plan) -> np.ndarray:
    """Brute-force translations, precomputation (Section 6.2): for every
    shift, the Fourier-Bessel coefficients of the translated image, T_delta
    a(k_m; q) = (1/Qa) sum_p Ahat(k_m, psi_p) exp(-i k_m . delta)
    exp(-i q psi_p): the ring samples times the translation phase (eq. Fdk)
    before the ring DFT of eq. aqkcalc.  Returns (N, M, Qa), q in
    signed_modes() order."""
    M, Qa = Ahat.shape
    dx = 2.0 / plan.n
    psi = polar_angles(Qa)
    q = signed_modes(Qa)
    D = np.exp(-1j * np.multiply.outer(psi, q)) / Qa  # (p, q)
    out = np.zeros((plan.shifts.shape[0], M, Qa), dtype=np.complex128)
    for s, (sx, sy) in enumerate(plan.shifts):
        kd = np.multiply.outer(plan.k, sx * dx * np.cos(psi) + sy * dx * np.sin(psi))  # (M, p)
        out[s] = (Ahat * np.exp(-1j * kd)) @ D
    return out


def bft_translations_X(Ahat: np.ndarray, b: np.ndarray, plan: Plan) -> np.ndarray:
    """Brute-force translations (Section 6.2): eq. fbk2 with l_max = 0 on
    the translated coefficients of each shift, then the rotation sum of
    eq. 1dfft: X(delta, r) = sum_q e^{-i q gamma_r} 2 pi sum_m w_m
    T_delta a(k_m; q) conj b(k_m; q).  Returns (N, Qa)."""
    Ta = bft_translated_coefficients(Ahat, plan)
    Qa = b.shape[1]
    E = np.exp(-1j * np.multiply.outer(signed_modes(Qa), polar_angles(Qa)))  # (q, r)
    Xh = TWO_PI * np.einsum("m,dmq,mq->dq", plan.w, Ta, np.conj(b))
    return Xh @ E


# ---------------------------------------------------------------------------
# Poses and error scale
# ---------------------------------------------------------------------------

def best_pose(X: np.ndarray):
    """argmax of Re X over (shift, rotation); ties go to the lowest shift
    index, then the lowest rotation index (row-major first maximum).

    Returns (value, shift_index, rot_index, margin) where margin is the best
    value minus the second best over all grid poses.
    """
    R = np.real(X)
    flat = R.reshape(-1)
    i = int(np.argmax(flat))
    v = float(flat[i])
    if flat.size > 1:
        second = float(np.partition(flat, -2)[-2])
    else:
        second = -np.inf
    return v, i // R.shape[1], i % R.shape[1], v - second


def pair_scale(a: np.ndarray, b: np.ndarray, plan: Plan) -> float:
    """s_AB = sqrt(X_AA(0,0) X_BB(0,0)): by Cauchy-Schwarz it bounds |X|
    on the quadrature (|F| = 1)."""
    def self_ip(c):
        return TWO_PI * float(np.sum(plan.w[:, None] * np.abs(c) ** 2))
    return math.sqrt(self_ip(a) * self_ip(b))


def rel_err(X: np.ndarray, Xref: np.ndarray, scale: float) -> float:
    return float(np.max(np.abs(np.real(X) - np.real(Xref)))) / scale


# ---------------------------------------------------------------------------
# Truncation bound (Section 5.2, eq. Xmserr, with the 2D constant)
# ---------------------------------------------------------------------------

def rank_lemma_bound(ell: int, W: float, eps: float) -> float:
    """H_ell upper bound of Lemma l:rank (eq. rank); W in wavelengths = R/2."""
    return max(0.0, math.pi * math.e ** 2 * W - abs(ell) / 2.0,
               math.log(2 * math.pi * W / eps) + 1.5 - abs(ell) / 2.0)


def hs_norm_sq_modal(ell: int, X: float) -> float:
    """int_0^X int_0^1 J_l(x y)^2 y dy x dx via Lommel's closed form for the
    inner integral: (J_l(x)^2 - J_{l-1}(x) J_{l+1}(x)) / 2."""
    from scipy.integrate import quad

    def inner(x):
        return 0.5 * (jv(ell, x) ** 2 - jv(ell - 1, x) * jv(ell + 1, x)) * x

    val, _ = quad(inner, 0.0, X, limit=400, epsabs=1e-14, epsrel=1e-13)
    return val
