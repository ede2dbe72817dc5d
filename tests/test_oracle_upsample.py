"""Pins of the oracle's rotation upsampling (the remark after eq. 1dfft:
zero-padding the angular sum samples many more rotations): X on the grid
gamma_r = 2 pi r / (U Qa).

Pinned by: U = 1 giving the plain FTK sum; every U-th angle equal to the
Qa-point grid; the values between grid angles equal to the direct inner
product with the template rendered at that (off-grid) rotation, to the
angular band limit of the blob images; X real; a planted mistake (the phase
of the finer grid with the wrong sign) failing the off-grid pin.
"""
import math

import numpy as np

import synth
from oracle import ftk as O


def _blob_case(n=32, Qa=64, R=2.0):
    rng = np.random.default_rng(3)
    A = synth.random_blobs(rng, 6, disk_px=6.0, sigma_px=(2.0, 3.0))
    B = synth.random_blobs(rng, 6, disk_px=6.0, sigma_px=(2.0, 3.0))
    plan = O.set_shifts(O.make_plan(n, 16, Qa, R, 1e-3), synth.shift_lattice(R))
    return plan, A, B


def test_u1_is_the_plain_sum():
    img = synth.white_noise_images(8, 2, 32)
    plan = O.set_shifts(O.make_plan(32, 16, 64, 2.0, 1e-3), synth.shift_lattice(2.0))
    a, b = (O.fb_coefficients(x, plan) for x in img)
    X = O.ftk_X(a, b, plan)
    assert np.max(np.abs(O.ftk_X_upsampled(a, b, plan, 1) - X)) < 1e-12 * np.max(np.abs(X))


def test_coarse_angles_and_reality():
    img = synth.white_noise_images(9, 2, 32)
    plan = O.set_shifts(O.make_plan(32, 16, 64, 2.0, 1e-3), synth.shift_lattice(2.0))
    a, b = (O.fb_coefficients(x, plan) for x in img)
    X = O.ftk_X(a, b, plan)
    for U in (2, 3, 5):
        Xu = O.ftk_X_upsampled(a, b, plan, U)
        assert Xu.shape == (X.shape[0], U * 64)
        assert np.max(np.abs(Xu[:, ::U] - X)) < 1e-12 * np.max(np.abs(X))
        assert np.max(np.abs(Xu.imag)) < 1e-12 * np.max(np.abs(Xu))


def _offgrid_error(sign):
    plan, A, B = _blob_case()
    n, Qa, U = plan.n, plan.Qa, 4
    Ah = O.polar_ft(synth.render(A, n), plan.k, Qa)
    Bh = O.polar_ft(synth.render(B, n), plan.k, Qa)
    Xu = O.bft_X_upsampled(Ah, O.ring_coefficients(Bh), plan, U)
    scale = np.max(np.abs(Xu))
    worst = 0.0
    for rp in (1, 2, 3, 37, 101, 255):
        g = sign * 2 * math.pi * rp / (U * Qa)
        # B rotated so that its transform is Bhat(k, psi + gamma)
        Bg = O.polar_ft(synth.render(B.moved(-g, (0.0, 0.0)), n), plan.k, Qa)
        Xt = O.direct_X(Ah, Bg, plan.k, plan.w, plan.shifts, n)[:, 0]
        worst = max(worst, float(np.max(np.abs(Xu[:, rp] - Xt)) / scale))
    return worst


def test_between_grid_angles_matches_rotated_template():
    assert _offgrid_error(+1.0) < 1e-5


def test_planted_wrong_phase_fails():
    assert _offgrid_error(-1.0) > 1e-2
