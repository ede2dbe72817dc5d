"""FP64 oracle of brute-force rotations (BFR, Section 6.1 of the paper), the
comparison method that correlates over a Cartesian grid of translations by
the 2D convolution theorem (eq. 2dconv), once per rotation.

TEST INFRASTRUCTURE ONLY -- the product path never imports this module.

Eq. 2dconv writes the inner product as an integral over the disk |k| <= Kmax
of Ahat(k) conj(R_gamma Bhat(k)) exp(-i k . delta); BFR discretises it on a
Cartesian grid in k and obtains every delta of a Cartesian grid at once with
one inverse 2D FFT per rotation (zero padding refines the delta spacing).
Readings taken here:

  * the k grid is the one of the pixel DFT: k = pi (u, v) (spacing
    2 Kmax / n, Kmax = pi n / 2) with integer u, v, restricted to the closed
    disk u^2 + v^2 <= (n/2)^2, a point set symmetric under k -> -k and under
    quarter turns; weight (pi)^2 per point;
  * the rotated template is sampled at the rotated grid points,
    (R_gamma Bhat)(k) = Bhat(R_gamma k) with R_gamma the rotation by
    +gamma, the convention of the polar inner product (eq. Xdg as
    discretised in ftk.direct_X), gamma_r = 2 pi r / Qa;
  * the normalisation is that of ftk.direct_X (no 1 / (2 pi)^2: the
    integral of Ahat conj Bhat over the plane is (2 pi)^2 <A, B>);
  * a zero-padded inverse FFT evaluates the same trigonometric sum at a finer
    delta grid, so the method's output at any requested shift is the sum
    itself, written out below.

X_BFR(delta, r) = pi^2 sum_{(u, v) in disk} exp(-i k_uv . delta)
                  Ahat(k_uv) conj(Bhat(R_{gamma_r} k_uv)).

It is real for real images (the point set is symmetric under k -> -k).
"""
from __future__ import annotations

import math

import numpy as np


def cartesian_grid(n: int, square: bool = False):
    """Integer (u, v) of the grid k = pi (u, v): the closed disk
    u^2 + v^2 <= (n/2)^2 (the method's set), or with square=True the n x n
    grid of the pixel DFT, u, v in [-n/2, n/2) (used by a pin)."""
    h = n // 2
    u, v = np.meshgrid(np.arange(-h, h + 1), np.arange(-h, h + 1), indexing="ij")
    u, v = u.ravel(), v.ravel()
    keep = (u < h) & (v < h) if square else (u * u + v * v <= h * h)
    return u[keep], v[keep]


def ft_at(img: np.ndarray, kx, ky) -> np.ndarray:
    """Ahat(k) = dx^2 sum_ij A_ij exp(-i k . x_ij) at arbitrary points
    (eq. Ahattrap), pixel (i, j) at ((i - n/2) dx, (j - n/2) dx), dx = 2/n."""
    n = img.shape[0]
    dx = 2.0 / n
    x = (np.arange(n) - n // 2) * dx
    kx = np.asarray(kx, dtype=np.float64)
    ky = np.asarray(ky, dtype=np.float64)
    Ex = np.exp(-1j * np.multiply.outer(kx, x))  # over i
    Ey = np.exp(-1j * np.multiply.outer(ky, x))  # over j
    return dx * dx * np.sum((Ex @ img) * Ey, axis=-1)


def rotated_spectra(img: np.ndarray, Qa: int, rots=None, square: bool = False) -> np.ndarray:
    """Bhat(R_{gamma_r} k_uv) for the rotations r in rots (default all Qa),
    shape (len(rots), P) over the grid points of cartesian_grid."""
    n = img.shape[0]
    u, v = cartesian_grid(n, square)
    kx, ky = math.pi * u, math.pi * v
    rots = range(Qa) if rots is None else rots
    out = []
    for r in rots:
        g = 2.0 * math.pi * r / Qa
        c, s = math.cos(g), math.sin(g)
        out.append(ft_at(img, c * kx - s * ky, s * kx + c * ky))
    return np.array(out)


def bfr_X_spectra(Ahat0: np.ndarray, Bhat_rot: np.ndarray, n: int, shifts_px, square: bool = False) -> np.ndarray:
    """X_BFR(delta_i, r) from Ahat on the grid (P,) and the rotated template
    spectra (R, P); returns (N, R) complex."""
    u, v = cartesian_grid(n, square)
    kx, ky = math.pi * u, math.pi * v
    d = np.asarray(shifts_px, dtype=np.float64).reshape(-1, 2) * (2.0 / n)
    F = np.exp(-1j * (np.multiply.outer(d[:, 0], kx) + np.multiply.outer(d[:, 1], ky)))  # (N, P)
    return math.pi ** 2 * (F @ (Ahat0[:, None] * np.conj(Bhat_rot.T)))


def bfr_X(A: np.ndarray, B: np.ndarray, shifts_px, Qa: int, rots=None, square: bool = False) -> np.ndarray:
    """X_BFR(delta_i, r) for images A, B (n x n), the shifts (N, 2) in
    pixels and the rotations r in rots (default all Qa); (N, R) complex."""
    n = A.shape[0]
    u, v = cartesian_grid(n, square)
    Ah = ft_at(A, math.pi * u, math.pi * v)
    return bfr_X_spectra(Ah, rotated_spectra(B, Qa, rots, square), n, shifts_px, square)
