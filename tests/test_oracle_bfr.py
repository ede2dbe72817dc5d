"""Pins of the oracle's brute-force rotations (BFR, Section 6.1, eq. 2dconv;
readings in oracle/bfr.py).

Pinned by: on the full n x n DFT grid, at rotation 0 and integer shifts, the
sum is the cyclic cross-correlation of the pixel arrays times (2 pi)^2 dx^2
(Parseval for the DFT), brute force over pixels; on the disk, quarter and
half turns of the template equal the same pixel array turned by index
permutation (the disk grid maps onto itself); the result is real; for smooth
central blobs it equals the polar-quadrature inner product of eq. Xdg
(ftk.direct_X, pinned elsewhere) at half-pixel shifts and off-axis rotations;
planted mistakes (the phase's sign, the rotation's direction) fail.
"""
import math

import numpy as np
import pytest

import synth
from oracle import bfr as B
from oracle import ftk as O


def _cyclic_correlation(A, Bm, d):
    n = A.shape[0]
    dx = 2.0 / n
    return (2 * math.pi) ** 2 * dx * dx * float(np.sum(A * np.roll(Bm, (-d[0], -d[1]), axis=(0, 1))))


def test_square_grid_is_the_pixel_cross_correlation():
    n = 16
    A, Bm = synth.white_noise_images(3, 2, n)
    shifts = np.array([[0, 0], [3, -1], [-2, 5], [7, 7], [-8, 1]], dtype=np.float64)
    X = B.bfr_X(A, Bm, shifts, 8, rots=[0], square=True)[:, 0]
    want = np.array([_cyclic_correlation(A, Bm, d.astype(int)) for d in shifts])
    assert np.max(np.abs(X - want)) < 1e-12 * np.max(np.abs(want))


def _bordered_blobs(seed, n):
    img = synth.render(synth.random_blobs(np.random.default_rng(seed), 8, disk_px=5.0), n)
    img[0, :] = 0.0
    img[:, 0] = 0.0
    return img


def _quarter_turn(Bm):
    # pixel (i, j) -> (j, n - i): the grid rotated by +pi/2 about pixel (n/2, n/2)
    n = Bm.shape[0]
    out = np.zeros_like(Bm)
    for i in range(1, n):
        out[:, n - i] = Bm[i, :]
    return out


def test_quarter_turns_are_index_permutations():
    n, Qa = 16, 16
    A = _bordered_blobs(5, n)
    Bm = _bordered_blobs(6, n)
    shifts = synth.shift_lattice(2.0)
    X = B.bfr_X(A, Bm, shifts, Qa, rots=[0, 4, 8, 12])
    turned = Bm
    for t in range(4):
        X0 = B.bfr_X(A, turned, shifts, Qa, rots=[0])[:, 0]
        assert np.max(np.abs(X[:, t] - X0)) < 1e-12 * np.max(np.abs(X0)), t
        turned = _quarter_turn(turned)


def test_real_for_real_images():
    A, Bm = synth.white_noise_images(4, 2, 16)
    X = B.bfr_X(A, Bm, synth.shift_lattice(2.0), 16, rots=[0, 3, 7])
    assert np.max(np.abs(X.imag)) < 1e-12 * np.max(np.abs(X.real))


def _smooth_pair(n):
    rng = np.random.default_rng(11)
    A = synth.render(synth.random_blobs(rng, 6, disk_px=6.0, sigma_px=(2.0, 3.0)), n)
    Bm = synth.render(synth.random_blobs(rng, 6, disk_px=6.0, sigma_px=(2.0, 3.0)), n)
    return A, Bm


def _polar_reference(A, Bm, shifts, Qa, rots):
    n = A.shape[0]
    k, w = O.radial_quadrature(n, 0.5 * math.pi * n)
    Ah, Bh = O.polar_ft(A, k, Qa), O.polar_ft(Bm, k, Qa)
    X = O.direct_X(Ah, Bh, k, w, shifts, n)[:, rots]
    sc = math.sqrt(O.direct_X(Ah, Ah, k, w, [[0.0, 0.0]], n)[0, 0].real *
                   O.direct_X(Bh, Bh, k, w, [[0.0, 0.0]], n)[0, 0].real)
    return X, sc


def test_agrees_with_the_polar_inner_product():
    n, Qa = 64, 128
    A, Bm = _smooth_pair(n)
    shifts = np.array([[0.0, 0.0], [0.5, -1.5], [-2.0, 0.5], [1.5, 1.0]])
    rots = [0, 5, 37, 90]
    X = B.bfr_X(A, Bm, shifts, Qa, rots=rots)
    ref, sc = _polar_reference(A, Bm, shifts, Qa, rots)
    assert np.max(np.abs(X - ref)) < 1e-12 * sc  # measured 2.6e-15


def test_planted_mistakes_fail(monkeypatch):
    n, Qa = 64, 128
    A, Bm = _smooth_pair(n)
    shifts = np.array([[0.5, -1.5], [-2.0, 0.5]])
    rots = [5, 37]
    ref, sc = _polar_reference(A, Bm, shifts, Qa, rots)
    # the rotation's direction reversed
    rs = B.rotated_spectra
    monkeypatch.setattr(B, "rotated_spectra", lambda img, Q, r=None, sq=False: rs(img, Q, [(-x) % Q for x in r], sq))
    assert np.max(np.abs(B.bfr_X(A, Bm, shifts, Qa, rots=rots) - ref)) > 1e-2 * sc
    monkeypatch.undo()
    # the phase's sign flipped (exp(+i k . delta))
    X = B.bfr_X(A, Bm, -shifts, Qa, rots=rots)
    assert np.max(np.abs(X - ref)) > 1e-2 * sc
    # on the pixel grid as well
    A16, B16 = synth.white_noise_images(3, 2, 16)
    d = np.array([[3.0, -1.0]])
    assert abs(B.bfr_X(A16, B16, -d, 8, rots=[0], square=True)[0, 0] -
               _cyclic_correlation(A16, B16, (3, -1))) > 1e-3
