"""GPU: ragged batches (ftk_batch_*) and launch-shape tuning (ftk_plan_*_tuning).

A batch only schedules independent alignments, so each stack's outputs must
be bitwise equal to ftk_align on the same plan and inputs, whatever the
lanes, graph capture and autotuned shapes; and the launch shapes must not
change any result (each pair's sums run in the same order for every shape).
The largest stack shape (n = 192, Qa = 384, W = 8 px, 797 shifts) is also
checked against the FP64 oracle, since no other test covers it.
"""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import ftk as O

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


def _dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _bits(t):
    return t.detach().cpu().numpy().view(np.uint32)


def _stack_specs():
    """Scaled-down ragged workload: shapes drawn like the 64-stack batch
    (n in {64, 96, 128, 192}, M = n/2, Qa = 2n, W in 2..8 px) plus the
    largest shape forced in; the four precision forms alternate."""
    specs = synth.ragged_stack_specs(11, count=6, scale=0.03)
    specs.append(dict(n=192, M=96, Qa=384, R=8.0, n_templates=3, n_images=2))
    for i, sp in enumerate(specs):
        sp["precision"] = ("fp32", "bf16x3", "fp16", "fp16x3")[i % 4]
        sp["want_X"] = i % 2 == 0
    return specs


@pytest.fixture(scope="module")
def stacks(ftk):
    out = []
    for i, sp in enumerate(_stack_specs()):
        s = synth.make_alignment_set(100 + i, sp["n"], sp["n_templates"], sp["n_images"], 20,
                                     min(sp["R"], 4.0), 0.1)
        shifts = synth.shift_lattice(sp["R"])
        P = ftk.Plan(sp["n"], sp["M"], sp["Qa"], sp["R"], 1e-3, sp["precision"])
        P.set_shifts(shifts)
        imgs, tmps = _dev(s.images), _dev(s.templates)
        X = (torch.empty((imgs.shape[0], tmps.shape[0], len(shifts), sp["Qa"]), dtype=torch.float32, device="cuda")
             if sp["want_X"] else None)
        best = torch.empty((imgs.shape[0], tmps.shape[0], 3), dtype=torch.int32, device="cuda")
        out.append(dict(plan=P, images=imgs, templates=tmps, X=X, best=best, spec=sp, shifts=shifts, set=s))
        _say(f"[stack {i}] n={sp['n']} Qa={sp['Qa']} W={sp['R']} N={len(shifts)} H={P.info()['H']} "
             f"nA={imgs.shape[0]} nB={tmps.shape[0]} {sp['precision']} X={sp['want_X']}")
    return out


def _reference(st):
    """ftk_align on the stack's own plan, fresh outputs (the null stream)."""
    X, best = st["plan"].align(st["images"], st["templates"], want_X=st["X"] is not None)
    torch.cuda.synchronize()
    return (None if X is None else _bits(X)), _bits(best)


def _poison(stacks_):
    for st in stacks_:
        if st["X"] is not None:
            st["X"].fill_(float("nan"))
        st["best"].fill_(-7)
    torch.cuda.synchronize()


def _compare(stacks_, refs, tag):
    for i, (st, (Xr, br)) in enumerate(zip(stacks_, refs)):
        assert np.array_equal(_bits(st["best"]), br), f"{tag}: stack {i} poses differ"
        if Xr is not None:
            assert np.array_equal(_bits(st["X"]), Xr), f"{tag}: stack {i} X differs"


def test_tuning_does_not_change_results(ftk):
    n, M, Qa, R = 128, 64, 256, 4.0
    s = synth.make_alignment_set(7, n, 40, 5, 30, R, 0.05)
    shifts = synth.shift_lattice(R)
    for prec in ("fp32", "bf16x3", "fp16", "fp16x3"):
        P = ftk.Plan(n, M, Qa, R, 1e-3, prec)
        P.set_shifts(shifts)
        d = P.tuning()
        _say(f"[tuning {prec}] default {d}")
        assert d == {"step3_waves": 16, "step1_zblk": 64 if prec == "fp16" else 128, "step1_wgs": 4096,
                     "stage_mib": 8192} or \
            any(k in os.environ for k in ("FTK_STEP3_WAVES", "FTK_STEP1_ZBLK", "FTK_STEP1_WGS", "FTK_STAGE_MB"))
        imgs, tmps = _dev(s.images), _dev(s.templates)
        X0, b0 = P.align(imgs, tmps, want_X=True)
        torch.cuda.synchronize()
        X0, b0 = _bits(X0), _bits(b0)
        # 16 MiB of staging forces one image per chunk here (40 templates x 516 KiB)
        for t in [dict(step3_waves=4), dict(step3_waves=7, step1_zblk=64), dict(step1_wgs=64),
                  dict(stage_mib=16), dict(step3_waves=1, step1_zblk=64, step1_wgs=65536, stage_mib=16)]:
            P.set_tuning(**t)
            X1, b1 = P.align(imgs, tmps, want_X=True)
            torch.cuda.synchronize()
            _say(f"  {t}: in force {P.tuning()}")
            assert np.array_equal(_bits(b1), b0), t
            assert np.array_equal(_bits(X1), X0), t
        P.set_tuning()
        assert P.tuning() == d
        with pytest.raises(ftk.FTKError):
            P.set_tuning(step3_waves=17)
        with pytest.raises(ftk.FTKError):
            P.set_tuning(step1_zblk=96)
        with pytest.raises(ftk.FTKError):
            P.set_tuning(stage_mib=8)


@pytest.mark.parametrize("n,M,Qa,R,nA,nB", [(64, 32, 128, 6.0, 8, 99), (192, 96, 384, 4.0, 2, 6)])
def test_svd_block_does_not_change_results(ftk, n, M, Qa, R, nA, nB):
    """Step 1 with 64 and 128 SVD terms per workgroup, every precision form:
    bitwise the same X.  At these shapes the fp16 forms' image operand
    conversions once differed between the two kernels (a fused
    product-and-round in one, a product rounded to FP32 and then converted in
    the other), which an autotuned batch then showed as a few pairs differing
    from ftk_align."""
    s = synth.make_alignment_set(103, n, nB, nA, 20, min(R, 4.0), 0.1)
    shifts = synth.shift_lattice(R)
    for prec in ("fp32", "bf16x3", "fp16", "fp16x3"):
        P = ftk.Plan(n, M, Qa, R, 1e-3, prec)
        P.set_shifts(shifts)
        out = []
        for z in (128, 64):
            P.set_tuning(step1_zblk=z)
            X, b = P.align(_dev(s.images), _dev(s.templates), want_X=True)
            torch.cuda.synchronize()
            out.append((_bits(X), _bits(b)))
        nd = int(np.sum(out[0][0] != out[1][0]))
        _say(f"[svd block n={n} {prec}] N={len(shifts)} H={P.info()['H']}: X elements differing {nd}")
        assert nd == 0 and np.array_equal(out[0][1], out[1][1])


def test_batch_graph_two_lanes_autotuned(ftk, stacks, tmp_path):
    refs = [_reference(st) for st in stacks]
    os.environ["FTK_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        stream = torch.cuda.Stream()
        B = ftk.Batch(stacks, lanes=2, graph=True, autotune=True, stream=stream)
    finally:
        del os.environ["FTK_TUNE_CACHE"]
    info = B.info()
    _say(f"[batch graph] {info}")
    lines = (tmp_path / "tune.txt").read_text().strip().splitlines()
    assert len(lines) >= 1
    other = ftk.Plan(32, 16, 64, 2.0, 1e-3)
    other.set_shifts(synth.shift_lattice(2.0))
    small = synth.workload_set("plain_n32", 1)
    for rep in range(3):
        _poison(stacks)
        B.run(stream)
        stream.synchronize()
        if rep == 0:
            assert B.info()["graph_nodes"] > 0
        _compare(stacks, refs, f"replay {rep}")
        # eager work between replays: torch kernels and another plan's alignment
        y = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        _, bo = other.align(_dev(small.images), _dev(small.templates))
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
    # new inputs in the same buffers: the replayed graph must see them
    st = stacks[0]
    st["images"].copy_(torch.flip(st["images"], dims=[0]))
    torch.cuda.synchronize()
    refs[0] = _reference(st)
    _poison(stacks)
    B.run(stream)
    stream.synchronize()
    _compare(stacks, refs, "after input change")
    B.close()


def test_batch_graph_four_lanes(ftk, stacks):
    """Four lanes (one hardware queue each), one graph: bitwise equal to the
    single-stack alignments over replays."""
    refs = [_reference(st) for st in stacks]
    stream = torch.cuda.Stream()
    B = ftk.Batch(stacks, lanes=4, graph=True, stream=stream)
    _say(f"[batch graph 4 lanes] {B.info()}")
    assert B.info()["lanes"] == 4
    for rep in range(2):
        _poison(stacks)
        B.run(stream)
        stream.synchronize()
        _compare(stacks, refs, f"4 lanes, replay {rep}")
        torch.cuda.synchronize()
    B.close()


def test_batch_eager_one_lane(ftk, stacks):
    refs = [_reference(st) for st in stacks]
    B = ftk.Batch(stacks, lanes=1)
    for rep in range(2):
        _poison(stacks)
        B.run()
        torch.cuda.synchronize()
        _compare(stacks, refs, f"eager run {rep}")
    assert B.info()["graph_nodes"] == 0
    B.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-3), ("fp16", 1e-3), ("fp16x3", 1e-5)])
def test_largest_stack_shape_against_oracle(ftk, prec, tol):
    """n = 192, M = 96, Qa = 384, W = 8 px (797 shifts) through a batch,
    against the FP64 oracle element by element (FP32 and split fp16: 1e-5,
    split bf16 and FP16: eps = 1e-3, of the pair scale)."""
    n, M, Qa, R = 192, 96, 384, 8.0
    s = synth.make_alignment_set(41, n, 2, 1, 30, 4.0, 0.1)
    shifts = synth.shift_lattice(R)
    P = ftk.Plan(n, M, Qa, R, 1e-3, prec)
    P.set_shifts(shifts)
    X = torch.full((1, 2, len(shifts), Qa), float("nan"), device="cuda")
    best = torch.full((1, 2, 3), -7, dtype=torch.int32, device="cuda")
    st = dict(plan=P, images=_dev(s.images), templates=_dev(s.templates), X=X, best=best)
    _say(f"[n192 {prec}] N={len(shifts)} H={P.info()['H']}")
    B = ftk.Batch([st], lanes=1)
    B.run()
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    poses = ftk.poses_numpy(best)
    plan = O.set_shifts(O.make_plan(n, M, Qa, R, 1e-3), shifts)
    a = O.fb_coefficients(s.images[0], plan)
    for j in range(2):
        bj = O.fb_coefficients(s.templates[j], plan)
        Xref = np.real(O.ftk_X(a, bj, plan))
        S = O.pair_scale(a, bj, plan)
        err = np.max(np.abs(X[0, j] - Xref)) / S
        v, si, ri, margin = O.best_pose(Xref)
        _say(f"  pair (0,{j}) rel err {err:.3e}; pose {(poses[0, j]['shift'], poses[0, j]['rot'])} "
             f"oracle {(si, ri)} margin/scale {margin / S:.2e}")
        assert err <= tol
        if margin > 2 * err * S:
            assert (poses[0, j]["shift"], poses[0, j]["rot"]) == (si, ri)
    B.close()


def test_batch_errors(ftk, stacks):
    with pytest.raises(ftk.FTKError) as e:
        ftk.Batch(stacks[:1], lanes=5)
    assert e.value.code == -1
    P = ftk.Plan(32, 16, 64, 2.0, 1e-3)  # shifts never set
    imgs = torch.zeros((1, 32, 32), device="cuda")
    best = torch.empty((1, 1, 3), dtype=torch.int32, device="cuda")
    with pytest.raises(ftk.FTKError) as e:
        ftk.Batch([dict(plan=P, images=imgs, templates=imgs, best=best)])
    assert e.value.code == -5
    B = ftk.Batch(stacks[:1], graph=True)
    with pytest.raises(ftk.FTKError) as e:
        B.run(stream=0)  # the null stream cannot be captured
    assert e.value.code == -1
    B.close()
    B = ftk.Batch([])
    B.run()
    assert B.info()["count"] == 0
    B.close()
