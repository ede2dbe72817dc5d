"""Pins of the oracle's brute-force translations (Section 6.2 of the paper):
translated coefficients per shift (ring samples times the phase of eq. Fdk,
then the ring DFT of eq. aqkcalc), the l_max = 0 contraction of eq. fbk2 and
the rotation sum of eq. 1dfft.

Pinned by: the direct polar inner product (O4, written as a circular
correlation over the ring samples, no coefficients at all) to rounding; the
untruncated Bessel-kernel FB formula (eq. fastrots); zero shift giving the
plain coefficients; the translated coefficients of a blob image equal to the
coefficients of the image rendered at the shifted centres (fixes the sign of
the phase and the pixel unit); planted mistakes.
"""
import numpy as np

import synth
from oracle import ftk as O


def _case(n=32, Qa=64, R=2.0):
    img = synth.white_noise_images(4, 2, n)
    plan = O.set_shifts(O.make_plan(n, 16, Qa, R, 1e-3), synth.shift_lattice(R))
    Ah, Bh = O.polar_ft(img[0], plan.k, Qa), O.polar_ft(img[1], plan.k, Qa)
    return plan, Ah, Bh


def test_bft_equals_direct_inner_product():
    plan, Ah, Bh = _case()
    b = O.ring_coefficients(Bh)
    Xb = O.bft_translations_X(Ah, b, plan)
    Xd = O.direct_X(Ah, Bh, plan.k, plan.w, plan.shifts, plan.n)
    assert np.max(np.abs(Xb - Xd)) < 1e-12 * np.max(np.abs(Xd))


def test_bft_equals_untruncated_bessel_kernel():
    plan, Ah, Bh = _case(n=24, Qa=48, R=1.5)
    a, b = O.ring_coefficients(Ah), O.ring_coefficients(Bh)
    Xb = O.bft_translations_X(Ah, b, plan)
    Xk = O.bft_X(a, b, plan, 23)
    assert np.max(np.abs(Xb - Xk)) < 1e-12 * np.max(np.abs(Xk))


def test_zero_shift_gives_plain_coefficients():
    plan, Ah, _ = _case()
    i0 = int(np.where(np.all(plan.shifts == 0.0, axis=1))[0][0])
    Ta = O.bft_translated_coefficients(Ah, plan)
    a = O.ring_coefficients(Ah)
    assert np.max(np.abs(Ta[i0] - a)) < 1e-14 * np.max(np.abs(a))


def _shifted_blob_coefficients(sign):
    n, Qa, R = 48, 96, 2.0
    rng = np.random.default_rng(5)
    blobs = synth.random_blobs(rng, 6, disk_px=6.0, sigma_px=(2.0, 3.0))
    plan = O.make_plan(n, 24, Qa, R, 1e-3)
    shifts = np.array([[1.5, -0.5], [-2.0, 0.0], [0.5, 1.0]])
    plan = O.set_shifts(plan, sign * shifts)
    Ta = O.bft_translated_coefficients(O.polar_ft(synth.render(blobs, n), plan.k, Qa), plan)
    worst = 0.0
    for s, d in enumerate(shifts):
        moved = O.fb_coefficients(synth.render(blobs.moved(0.0, d), n), plan)
        worst = max(worst, float(np.max(np.abs(Ta[s] - moved)) / np.max(np.abs(moved))))
    return worst


def test_translated_coefficients_are_those_of_the_shifted_image():
    # blobs of width >= 2 px are band-limited to ~exp(-pi^2 sigma^2 / 2) at
    # the Nyquist disk, so the pixel images' transforms follow the analytic shift
    assert _shifted_blob_coefficients(+1.0) < 1e-7


def test_planted_mistakes_fail():
    # the phase with the wrong sign moves the image the other way
    assert _shifted_blob_coefficients(-1.0) > 1e-2
    # conjugating the image instead of the template
    plan, Ah, Bh = _case()
    b = O.ring_coefficients(Bh)
    Xd = O.direct_X(Ah, Bh, plan.k, plan.w, plan.shifts, plan.n)
    Ta = O.bft_translated_coefficients(Ah, plan)
    Qa = b.shape[1]
    E = np.exp(-1j * np.multiply.outer(O.signed_modes(Qa), O.polar_angles(Qa)))
    bad = (2 * np.pi * np.einsum("m,dmq,mq->dq", plan.w, np.conj(Ta), b)) @ E
    assert np.max(np.abs(bad - Xd)) > 1e-2 * np.max(np.abs(Xd))
