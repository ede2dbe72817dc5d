"""The host FP64 planner (quadrature, Bessel recurrence, modal SVD and
truncation, spreading kernel, FFT lengths) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run over the sizes the
library plans for: no sanitizer report, and its numbers equal the FP64
oracle's (Section 3.1 quadrature moments; Section 4.5 truncation: H, L, the
first dropped singular value, factor products)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.special import jv

from oracle import ftk as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_12317_amd", "csrc")


@pytest.fixture(scope="module")
def lines(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "planner_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(ROOT, "tests", "native", "planner_check.cpp"),
           os.path.join(CSRC, "planner.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    out = {}
    for ln in r.stdout.splitlines():
        k, *v = ln.split()
        out.setdefault(k, []).append([float(x) for x in v])
    return out


def test_radial_rule(lines):
    kmax = math.pi * 64.0
    for M, sw, m3, k0, k1 in lines["rule"]:
        M = int(M)
        k, w = O.radial_quadrature(M, kmax)
        assert sw == pytest.approx(kmax ** 2 / 2, rel=1e-12)
        if M >= 2:  # exact for k^3 k dk once 2M - 1 >= 3
            assert m3 == pytest.approx(kmax ** 5 / 5, rel=1e-12)
        assert k0 == pytest.approx(k[0], rel=1e-11) and k1 == pytest.approx(k[-1], rel=1e-12)


def test_bessel(lines):
    for z, j0, j3, s in lines["bessel"]:
        assert j0 == pytest.approx(jv(0, z), abs=1e-14)
        assert j3 == pytest.approx(jv(3, z), abs=1e-14)
        assert s == pytest.approx(1.0, abs=1e-13)  # J_0^2 + 2 sum J_l^2 = 1


def test_truncation(lines):
    rows = lines["trunc"]
    assert len(rows) == 15 * 3
    for R, eps, H, L, nxt, s2, uv in rows:
        if R > 5.0:
            continue  # the oracle's larger SVDs are slow; the sanitizer run covers them
        keep, svds, dropped = O.truncation(R, eps)
        assert int(H) == len(keep), (R, eps)
        assert int(L) == max(abs(t[0]) for t in keep)
        assert nxt == pytest.approx(dropped, rel=1e-9, abs=1e-14)
        assert s2 <= math.pi ** 2 * R ** 2 / 4 * (1 + 1e-12)  # sum of all sigma^2 = pi^2 W^2, W = R/2
        X = math.pi * R
        ref = sum(float(svds[l].u(e, 0.7 * X) * svds[l].sigma_v(e, 0.3)) for l, e, _ in keep if l >= 0)
        assert uv == pytest.approx(ref, rel=1e-9, abs=1e-11), (R, eps)


def test_spread_and_fft(lines):
    for n, nf, f0, f1 in lines["spread"]:
        assert int(nf) >= 2 * n and f0 > f1 > 0
    sizes = {int(L): (int(s), int(ok)) for L, s, ok in lines["fft"]}
    assert sizes[7] == (8, 0) and sizes[100] == (108, 0) and sizes[385] == (432, 0)
    assert sizes[4096] == (4096, 1) and sizes[4097] == (0, 0) and sizes[9000] == (0, 0)


def test_jacobi_svd(lines):
    (s,) = lines["svd"]
    A = np.array([[4, 1, 2], [1, 3, 0], [2, 0, 5], [1, 1, 1]], float)
    assert np.allclose(s, np.linalg.svd(A, compute_uv=False), rtol=1e-13)
