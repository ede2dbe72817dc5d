"""FP64 oracle of the joint factorisation of translation and contrast transfer
function (Section 7.1 of the paper, other 2D kernels).

TEST INFRASTRUCTURE ONLY -- the product path never imports this module.

Translating by delta and filtering by a CTF with defocus tau multiply the
Fourier transform by F(delta, k) C(|k|; tau).  The paper proposes factorising
that product into terms Y_zeta(delta, tau) G_zeta(k) and running the same
algorithm.  Readings taken here (the paper names the idea, not the model):

  * the CTF is the isotropic weak-phase model
        C(s; tau) = -( sqrt(1 - A^2) sin chi(s) + A cos chi(s) ),
        chi(s)    = pi lambda tau s^2 - (pi / 2) Cs lambda^3 s^4,
    s the spatial frequency in 1/Angstrom, lambda the electron wavelength,
    Cs the spherical aberration, A the amplitude contrast, tau the defocus
    (Angstrom, positive = underfocus); no envelope, no astigmatism;
  * with pixels of p Angstrom the image square [-1, 1]^2 is n p Angstrom
    wide, so k = y Kmax (Kmax = pi n / 2) is s = y / (2 p) (Nyquist at
    y = 1);
  * per angular mode l the kernel J_l(x y) C(y; tau) is decomposed by the
    SVD of the operator from L2(y dy) on [0, 1] to L2(x dx dtau / |T|) on
    [0, X] x [tmin, tmax] (the defocus range, uniform measure of mass 1):
    the translation SVD of Section 4.5 with one more variable on the shift
    side, so that Y_zeta(delta, tau) = u_zeta(Kmax |delta|, tau)
    exp(-i l (omega + pi/2)) and G_zeta(k) = Sigma_zeta v_zeta(k / Kmax);
  * terms are kept as in the plain factorisation (Sigma > eps, scanning |l|
    until Sigma_1(l) <= eps).

The filter is applied to the image side: X(delta, tau, gamma) =
<R_gamma T_delta C_tau A, B>, which for a real, isotropic C equals the
alignment of A with the CTF-filtered template C_tau B.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import jv, roots_legendre

from oracle import ftk as O


@dataclasses.dataclass
class CtfModel:
    wavelength_A: float
    cs_mm: float
    amplitude_contrast: float
    pixel_A: float

    def chi(self, y, tau):
        s = np.asarray(y, dtype=np.float64) / (2.0 * self.pixel_A)
        lam = self.wavelength_A
        cs = self.cs_mm * 1e7
        return math.pi * lam * np.asarray(tau) * s ** 2 - 0.5 * math.pi * cs * lam ** 3 * s ** 4

    def __call__(self, y, tau):
        """C at k = y Kmax and defocus tau (broadcasting)."""
        a = self.amplitude_contrast
        c = self.chi(y, tau)
        return -(math.sqrt(1.0 - a * a) * np.sin(c) + a * np.cos(c))


def legendre_rule(P: int, lo: float, hi: float):
    """Gauss-Legendre nodes on [lo, hi], weights of total mass 1."""
    x, w = roots_legendre(P)
    return lo + 0.5 * (x + 1.0) * (hi - lo), 0.5 * w


def ctf_nodes(X: float, ctf: CtfModel, tmin: float, tmax: float):
    """(P_delta, P_tau, P_k) of the oracle's discretisation: the plain
    factorisation's node count on the shift side, plus enough defocus nodes
    for the phase range pi lambda (tmax - tmin) / (4 p^2) of chi at Nyquist
    and enough k nodes for the oscillation of C along k."""
    pd = O.svd_nodes(X)
    dchi = math.pi * ctf.wavelength_A * (tmax - tmin) / (4.0 * ctf.pixel_A ** 2)
    chimax = float(np.max(np.abs(ctf.chi(np.linspace(0.0, 1.0, 257)[:, None], np.array([tmin, tmax])[None, :]))))
    return pd, int(math.ceil(dchi)) + 16, pd + int(math.ceil(2.0 * chimax)) + 32


@dataclasses.dataclass
class CtfSVD:
    """SVD of J_l(x y) C(y; tau); rows are the shift-side nodes (x_i, tau_t)
    in the order i P_tau + t, columns the k-side nodes y_j."""

    ell: int
    X: float
    ctf: CtfModel
    sigma: np.ndarray
    Umat: np.ndarray
    Vt: np.ndarray
    xn: np.ndarray  # rows: x of each row node
    tn: np.ndarray  # rows: tau of each row node
    rw: np.ndarray  # rows: x-weight times tau-weight
    yn: np.ndarray
    yw: np.ndarray

    def sigma_v(self, eta: int, y) -> np.ndarray:
        """Sigma_eta v_eta(y) (Nystrom through the shift side)."""
        y = np.asarray(y, dtype=np.float64)
        K = jv(self.ell, np.multiply.outer(y, self.xn)) * self.ctf(y[..., None], self.tn)
        return K @ (np.sqrt(self.rw) * self.Umat[:, eta])

    def u(self, eta: int, x, tau) -> np.ndarray:
        """u_eta(x, tau) (Nystrom through the k side)."""
        x = np.asarray(x, dtype=np.float64)
        tau = np.asarray(tau, dtype=np.float64)
        K = jv(self.ell, np.multiply.outer(x, self.yn)) * self.ctf(self.yn, tau[..., None])
        return (K @ (np.sqrt(self.yw) * self.Vt[eta, :])) / self.sigma[eta]


def ctf_modal_svd(ell: int, X: float, ctf: CtfModel, tmin: float, tmax: float, nodes=None) -> CtfSVD:
    pd, pt, py = ctf_nodes(X, ctf, tmin, tmax) if nodes is None else nodes
    xn, xw = O.radial_quadrature(pd, X)
    tn, tw = legendre_rule(pt, tmin, tmax)
    yn, yw = O.radial_quadrature(py, 1.0)
    rx = np.repeat(xn, pt)
    rt = np.tile(tn, pd)
    rw = np.repeat(xw, pt) * np.tile(tw, pd)
    K = jv(ell, np.multiply.outer(rx, yn)) * ctf(yn[None, :], rt[:, None])
    A = np.sqrt(rw)[:, None] * K * np.sqrt(yw)[None, :]
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    return CtfSVD(ell, X, ctf, s, U, Vt, rx, rt, rw, yn, yw)


def make_ctf_plan(n: int, M: int, Qa: int, R: float, eps: float, ctf: CtfModel, tmin: float, tmax: float,
                  nodes=None) -> O.Plan:
    """The plan of the joint factorisation (same fields as the translation
    plan; its svds are CtfSVD).  Attributes ctf, tmin, tmax are added."""
    kmax = 0.5 * math.pi * n
    k, w = O.radial_quadrature(M, kmax)
    X = math.pi * R
    svds, keep, dropped = {}, [], 0.0
    ell = 0
    while True:
        sv = ctf_modal_svd(ell, X, ctf, tmin, tmax, nodes)
        if sv.sigma[0] <= eps:
            dropped = max(dropped, sv.sigma[0])
            break
        for l in ([0] if ell == 0 else [ell, -ell]):
            s = sv if l == ell else ctf_modal_svd(l, X, ctf, tmin, tmax, nodes)
            svds[l] = s
            h = int(np.sum(s.sigma > eps))
            keep += [(l, e, s.sigma[e]) for e in range(h)]
            dropped = max(dropped, s.sigma[h] if h < s.sigma.size else 0.0)
        ell += 1
    keep.sort(key=lambda t: (t[0], t[1]))
    ells = np.array([t[0] for t in keep], dtype=np.int64)
    etas = np.array([t[1] for t in keep], dtype=np.int64)
    sig = np.array([t[2] for t in keep])
    g = np.zeros((ells.size, M))
    for z, (l, e) in enumerate(zip(ells, etas)):
        g[z] = svds[int(l)].sigma_v(int(e), k / kmax)
    plan = O.Plan(n, M, Qa, R, eps, kmax, k, w, ells, etas, sig, g, svds, dropped)
    plan.ctf, plan.tmin, plan.tmax = ctf, tmin, tmax
    return plan


def set_poses(plan: O.Plan, shifts_px: np.ndarray, defocus_A: np.ndarray) -> O.Plan:
    """Y[i, zeta] = u_zeta(Kmax |delta_i|, tau_i) exp(-i l (omega_i + pi/2))
    for the poses i = (shift_i, defocus_i)."""
    shifts_px = np.asarray(shifts_px, dtype=np.float64).reshape(-1, 2)
    tau = np.asarray(defocus_A, dtype=np.float64).reshape(-1)
    if tau.size != shifts_px.shape[0]:
        raise ValueError("one defocus per shift")
    r = np.hypot(shifts_px[:, 0], shifts_px[:, 1])
    if np.any(r > plan.R * (1 + 1e-12)) or np.any(tau < plan.tmin) or np.any(tau > plan.tmax):
        raise ValueError("pose outside the planned domain")
    om = np.arctan2(shifts_px[:, 1], shifts_px[:, 0])
    Y = np.zeros((shifts_px.shape[0], plan.H), dtype=np.complex128)
    for z, (l, e) in enumerate(zip(plan.ell, plan.eta)):
        Y[:, z] = plan.svds[int(l)].u(int(e), math.pi * r, tau) * np.exp(-1j * l * (om + 0.5 * math.pi))
    plan.shifts, plan.defocus, plan.Y = shifts_px, tau, Y
    return plan


def direct_X_ctf(Ahat: np.ndarray, Bhat: np.ndarray, k, w, shifts_px, defocus_A, n: int, ctf: CtfModel,
                 kmax: float) -> np.ndarray:
    """Direct polar inner product with the multiplier F(delta, k) C(|k|; tau)
    for every pose (shift_i, defocus_i): eq. Xdg discretised as in
    ftk.direct_X, the image's samples multiplied by C."""
    tau = np.asarray(defocus_A, dtype=np.float64).reshape(-1)
    sh = np.asarray(shifts_px, dtype=np.float64).reshape(-1, 2)
    out = np.zeros((sh.shape[0], Ahat.shape[1]), dtype=np.complex128)
    for i in range(sh.shape[0]):
        c = ctf(np.asarray(k) / kmax, tau[i])  # (M,)
        out[i] = O.direct_X(Ahat * c[:, None], Bhat, k, w, sh[i:i + 1], n)[0]
    return out
