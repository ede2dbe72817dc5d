"""The library's FP64 planner for plans with a CTF (ftk_plan_tables_ctf,
host only) against the oracle's joint translation-CTF factorisation: the
same kept terms, singular values to 1e-11 and, per angular mode, the same
reconstructed kernel sum_eta Y G on the poses (sign-free: singular vectors
are defined up to sign), at the library's own (smaller) node counts."""
import numpy as np
import pytest

import synth
from oracle import ctf as C

CTFD = dict(wavelength_A=0.019687, cs_mm=2.7, amplitude_contrast=0.07, pixel_A=2.0,
            defocus_min_A=14000.0, defocus_max_A=16000.0)


@pytest.fixture(scope="module")
def F():
    from paper_1905_12317_amd import ftk
    try:
        ftk.lib()
    except ImportError as e:
        pytest.skip(str(e))
    return ftk


def test_ctf_tables_match_oracle(F):
    n, M, R = 32, 16, 2.0
    sh = synth.shift_lattice(R)
    df = np.linspace(14000.0, 16000.0, len(sh))
    T = F.ftk_plan_tables_ctf(n, M, R, 1e-3, CTFD, sh, df)
    cm = C.CtfModel(CTFD["wavelength_A"], CTFD["cs_mm"], CTFD["amplitude_contrast"], CTFD["pixel_A"])
    p = C.set_poses(C.make_ctf_plan(n, M, 64, R, 1e-3, cm, 14000.0, 16000.0), sh, df)
    assert T["H"] == p.H and np.array_equal(T["ell"], p.ell)
    assert np.max(np.abs(T["sigma"] - p.sigma) / p.sigma) < 1e-11
    assert abs(T["sigma_next"] - p.sigma_next) < 1e-11
    for l in np.unique(p.ell):
        zo, zl = np.where(p.ell == l)[0], np.where(T["ell"] == l)[0]
        Ko = p.Y[:, zo] @ p.g[zo]
        Kl = T["Y"][:, zl] @ T["G"][zl]
        assert np.max(np.abs(Ko - Kl)) < 1e-11 * np.max(np.abs(Ko)), l


def test_ctf_argument_checks(F):
    bad = dict(CTFD, amplitude_contrast=1.5)
    with pytest.raises(F.FTKError):
        F.ftk_plan_tables_ctf(32, 16, 2.0, 1e-3, bad)
    rev = dict(CTFD, defocus_min_A=16000.0, defocus_max_A=14000.0)
    with pytest.raises(F.FTKError):
        F.ftk_plan_tables_ctf(32, 16, 2.0, 1e-3, rev)
    with pytest.raises(F.FTKError):  # a defocus outside the planned range
        F.ftk_plan_tables_ctf(32, 16, 2.0, 1e-3, CTFD, np.zeros((1, 2)), np.array([20000.0]))
