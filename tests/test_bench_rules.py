"""CPU: the benchmark's reporting rules (no GPU).

The reported form is chosen by comparing each form's per-image best template
and pose with the FP32 form's, so the helpers that pick them are pinned here:
the best template is the largest pose value, the lower template number on
ties (the tie rule of ftk_best_template and of the oracle's best pose), and
agreement needs template, shift and rotation all equal.  A request for more
than one GPU exits with a message.
"""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1905_12317_amd import ftk  # noqa: E402


def _poses(values, shifts, rots):
    p = np.zeros(np.shape(values), dtype=ftk.POSE_DTYPE)
    p["value"], p["shift"], p["rot"] = values, shifts, rots
    return p


def test_image_best_takes_largest_value_lowest_template_on_ties():
    v = np.array([[0.1, 0.7, 0.7, -1.0], [2.0, 1.0, 3.0, 3.0]], dtype=np.float32)
    sh = np.array([[5, 6, 7, 8], [1, 2, 3, 4]], dtype=np.int32)
    ro = np.array([[9, 10, 11, 12], [13, 14, 15, 16]], dtype=np.int32)
    bt, bs, br = bench.image_best(_poses(v, sh, ro))
    assert bt.tolist() == [1, 2]
    assert bs.tolist() == [6, 3] and br.tolist() == [10, 15]


def test_agreement_needs_template_shift_and_rotation():
    ref = (np.array([0, 1, 2, 3]), np.array([5, 5, 5, 5]), np.array([7, 7, 7, 7]))
    other = (np.array([0, 1, 9, 3]), np.array([5, 4, 5, 5]), np.array([7, 7, 7, 6]))
    # image 0 agrees; 1 differs in shift, 2 in template, 3 in rotation
    assert bench.agreement(other, ref) == 0.25
    assert bench.agreement(ref, ref) == 1.0


def test_recall_counts_generating_template():
    class S:
        true_template = np.array([3, 1, 4, 1])
    assert bench.recall((np.array([3, 1, 0, 0]), None, None), S) == 0.5


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _sha1_of(names):
    import hashlib
    h = hashlib.sha1()
    for name in names:
        with open(os.path.join(ROOT, "paper_1905_12317_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def test_traffic_is_null_once_the_kernel_sources_change(monkeypatch):
    """The recorded HBM bytes of a Step 3 kernel are reported only while the
    sources they were measured on are unchanged (SHA-1 over the listed files)."""
    fresh = dict(bench.TRAFFIC["fp16"])
    fresh["sha1"] = _sha1_of(fresh["sources"])
    monkeypatch.setitem(bench.TRAFFIC, "fp16", fresh)
    assert bench.measured_traffic("fp16") == fresh["bytes_per_launch"]
    stale = dict(bench.TRAFFIC["fp16"], sha1="0" * 40)
    monkeypatch.setitem(bench.TRAFFIC, "fp16", stale)
    assert bench.measured_traffic("fp16") is None
    assert bench.measured_traffic("fp16+bf16x3") is None  # no entry of its own
