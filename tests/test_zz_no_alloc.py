"""ftk_align_coeffs_noalloc (the entry point for callers that cannot allocate
device memory) against ftk_align_coeffs, through the C-ABI.

Both run the same kernels, so X and the poses must agree bitwise (the
no-allocation staging may hold fewer images per chunk, which changes no
sum).  Two calls in a row on one GPU share the fixed scratch; the second is
smaller and must not see the first's contents.  The plan's device memory
must not grow, and a call that needs more than the scratch is refused on the
host before any work is issued.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ftk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_12317_amd import ftk as F
    F.lib()
    return F


def _coeffs(ftk, n, M, Qa, images, templates):
    T = ftk.Plan(n, M, Qa, 2.0, 1e-3)
    dev = torch.device("cuda:0")
    a = T.transform(torch.as_tensor(images, dtype=torch.float32, device=dev))
    b = T.transform(torch.as_tensor(templates, dtype=torch.float32, device=dev))
    return a, b


def _same(ftk, X0, b0, X1, b1):
    assert np.array_equal(X0.cpu().numpy().view(np.uint32), X1.cpu().numpy().view(np.uint32))
    p0, p1 = ftk.poses_numpy(b0), ftk.poses_numpy(b1)
    for k in ("value", "shift", "rot"):
        assert np.array_equal(p0[k], p1[k])


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp16", "fp16x3"])
def test_noalloc_matches_align_coeffs(ftk, form):
    n, M, Qa, R = 32, 16, 64, 2.0
    s = synth.make_alignment_set(21, n, 11, 5, 20, R, 0.1)
    a, b = _coeffs(ftk, n, M, Qa, s.images, s.templates)
    P = ftk.Plan(n, M, Qa, R, 1e-3, precision=form)
    P.set_shifts(synth.shift_lattice(R))
    held = P.info()["device_bytes"]
    N = P.info()["N"]
    for nA, nB in ((5, 11), (2, 3)):  # the second call smaller
        _say(f"[noalloc] form={form} nA={nA} nB={nB} n={n} N={N}")
        aa, bb = a[:nA].contiguous(), b[:nB].contiguous()
        X1 = torch.full((nA, nB, N, Qa), float("nan"), dtype=torch.float32, device="cuda")
        b1 = torch.full((nA, nB, 3), -1, dtype=torch.int32, device="cuda")
        P.align_coeffs_noalloc(aa, bb, X=X1, best=b1)
        torch.cuda.synchronize()
        assert P.info()["device_bytes"] == held  # nothing allocated by the call
        R0 = ftk.Plan(n, M, Qa, R, 1e-3, precision=form)
        R0.set_shifts(synth.shift_lattice(R))
        X0, b0 = R0.align_coeffs(aa, bb, want_X=True)
        torch.cuda.synchronize()
        _same(ftk, X0, b0, X1, b1)


def test_noalloc_chunks_and_limit(ftk):
    """n = 128, 197 shifts, 300 templates: the scratch holds the staging of
    five images, so six images run in two chunks; the poses equal
    ftk_align_coeffs' (one chunk) bitwise.  6000 templates need more than the
    scratch: FTK_EUNSUPPORTED, outputs untouched."""
    n, M, Qa, R = 128, 64, 256, 4.0
    s = synth.make_alignment_set(22, n, 300, 6, 60, R, 0.05)
    a, b = _coeffs(ftk, n, M, Qa, s.images, s.templates)
    P = ftk.Plan(n, M, Qa, R, 1e-3, precision="fp32")
    P.set_shifts(synth.shift_lattice(R))
    _say("[noalloc] fp32 n=128 nA=6 nB=300 (two chunks)")
    b1 = torch.full((6, 300, 3), -1, dtype=torch.int32, device="cuda")
    P.align_coeffs_noalloc(a, b, best=b1)
    _, b0 = P.align_coeffs(a, b)
    torch.cuda.synchronize()
    p0, p1 = ftk.poses_numpy(b0), ftk.poses_numpy(b1)
    for k in ("value", "shift", "rot"):
        assert np.array_equal(p0[k], p1[k])
    big = b[:1].expand(6000, -1, -1).contiguous()
    out = torch.full((6, 6000, 3), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(ftk.FTKError) as ei:
        P.align_coeffs_noalloc(a, big, best=out)
    assert ei.value.code == -6  # FTK_EUNSUPPORTED
    assert "fixed scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == -7).all())
