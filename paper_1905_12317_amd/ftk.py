"""Thin Python binding of libftk.so (argument marshalling only).

Every computation runs in the HIP library; this module only converts
Python/torch arguments to the C-ABI's plain pointers, sizes and streams.
Device buffers are torch CUDA (HIP) tensors; streams default to torch's
current stream.  If the library is not built, importing the binding's
functions raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libftk.so")

FTK_OK = 0
FTK_FP32 = 0
FTK_BF16X3 = 1
FTK_FP16 = 2
FTK_FP16X3 = 3
PRECISIONS = {"fp32": FTK_FP32, "bf16x3": FTK_BF16X3, "fp16": FTK_FP16, "fp16x3": FTK_FP16X3}


class FTKError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {code})")
        self.code = code


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("M", ctypes.c_int), ("Qa", ctypes.c_int), ("H", ctypes.c_int),
                ("L", ctypes.c_int), ("N", ctypes.c_int), ("precision", ctypes.c_int),
                ("nufft_width", ctypes.c_int), ("nufft_grid", ctypes.c_int),
                ("shift_radius_px", ctypes.c_double), ("eps", ctypes.c_double),
                ("sigma_next", ctypes.c_double), ("kmax", ctypes.c_double),
                ("coeff_bytes_per_image", ctypes.c_size_t), ("device_bytes", ctypes.c_size_t),
                ("weighted", ctypes.c_int), ("rotations", ctypes.c_int), ("ctf", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("step3_waves", ctypes.c_int), ("step1_zblk", ctypes.c_int), ("step1_wgs", ctypes.c_int),
                ("stage_mib", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Stack(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("images", ctypes.c_void_p), ("nA", ctypes.c_int),
                ("templates", ctypes.c_void_p), ("nB", ctypes.c_int), ("X", ctypes.c_void_p),
                ("best", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("lanes", ctypes.c_int), ("graph_nodes", ctypes.c_int),
                ("workspace_bytes", ctypes.c_size_t), ("cost_gflop", ctypes.c_double),
                ("tune_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


FTK_BATCH_GRAPH = 1
FTK_BATCH_AUTOTUNE = 2

POSE_DTYPE = np.dtype([("value", np.float32), ("shift", np.int32), ("rot", np.int32)])

#: every symbol include/ftk.h declares
EXPORTS = ["ftk_plan_create", "ftk_plan_destroy", "ftk_plan_info", "ftk_set_shifts", "ftk_transform",
           "ftk_align_coeffs", "ftk_align_coeffs_noalloc", "ftk_align", "ftk_bft_align", "ftk_bfr_align", "ftk_plan_set_rotations", "ftk_plan_create_ctf", "ftk_set_poses",
           "ftk_plan_tables_ctf", "ftk_plan_set_shift_windows", "ftk_plan_tables", "ftk_plan_create_weighted",
           "ftk_plan_tables_weighted", "ftk_plan_profile", "ftk_plan_stage_times",
           "ftk_plan_set_tuning", "ftk_plan_get_tuning", "ftk_batch_create", "ftk_batch_run", "ftk_batch_info",
           "ftk_batch_destroy", "ftk_strerror", "ftk_last_error_message",
           # include/ftk_mlp.h
           "ftk_mlp_create", "ftk_mlp_destroy", "ftk_mlp_info", "ftk_mlp_set_layer", "ftk_mlp_get_layer",
           "ftk_mlp_set_input_norm", "ftk_features", "ftk_mlp_forward", "ftk_mlp_gradients", "ftk_mlp_get_grad",
           "ftk_mlp_train_step", "ftk_propose", "ftk_align_lists", "ftk_best_template", "ftk_align_proposed",
           "ftk_align_refined"]

FTK_MLP_FP32 = 0
FTK_MLP_BF16 = 1
MLP_PRECISIONS = {"fp32": FTK_MLP_FP32, "bf16": FTK_MLP_BF16}


class Ctf(ctypes.Structure):
    """ftk_ctf_t: weak-phase CTF of ftk_plan_create_ctf."""
    _fields_ = [("wavelength_A", ctypes.c_double), ("cs_mm", ctypes.c_double),
                ("amplitude_contrast", ctypes.c_double), ("pixel_A", ctypes.c_double),
                ("defocus_min_A", ctypes.c_double), ("defocus_max_A", ctypes.c_double)]


class MLPInfo(ctypes.Structure):
    _fields_ = [("nlayers", ctypes.c_int), ("dims", ctypes.c_int * 9), ("n_template", ctypes.c_int),
                ("n_shift", ctypes.c_int), ("precision", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("step", ctypes.c_int64), ("param_count", ctypes.c_size_t), ("device_bytes", ctypes.c_size_t)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["dims"] = list(self.dims)[:self.nlayers + 1]
        return d

_lib = None


def lib() -> ctypes.CDLL:
    """Load libftk.so once; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1905_12317_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.ftk_plan_create.argtypes = [ctypes.POINTER(vp), i, i, i, d, d, i]
    L.ftk_plan_create_weighted.argtypes = [ctypes.POINTER(vp), i, i, i, d, d, i, vp, vp, i]
    L.ftk_plan_tables_weighted.argtypes = [i, i, d, d, vp, vp, i, vp, i, ctypes.POINTER(i), vp, vp, vp, vp, vp, vp,
                                           ctypes.POINTER(d)]
    L.ftk_plan_destroy.argtypes = [vp]
    L.ftk_plan_destroy.restype = None
    L.ftk_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.ftk_set_shifts.argtypes = [vp, vp, i]
    L.ftk_transform.argtypes = [vp, vp, i, vp, vp]
    L.ftk_align_coeffs.argtypes = [vp, vp, i, vp, i, vp, vp, vp]
    L.ftk_align_coeffs_noalloc.argtypes = [vp, vp, i, vp, i, vp, vp, vp]
    L.ftk_align.argtypes = [vp, vp, i, vp, i, vp, vp, vp]
    L.ftk_bft_align.argtypes = [vp, vp, i, vp, i, vp, vp, vp]
    L.ftk_bfr_align.argtypes = [vp, vp, i, vp, i, vp, vp, vp]
    L.ftk_plan_set_rotations.argtypes = [vp, i]
    L.ftk_plan_create_ctf.argtypes = [ctypes.POINTER(vp), i, i, i, d, d, i, ctypes.POINTER(Ctf)]
    L.ftk_set_poses.argtypes = [vp, vp, vp, i]
    L.ftk_plan_set_shift_windows.argtypes = [vp, vp, i, d]
    L.ftk_plan_tables_ctf.argtypes = [i, i, d, d, ctypes.POINTER(Ctf), vp, vp, i, ctypes.POINTER(i), vp, vp, vp, vp,
                                      vp, vp, ctypes.POINTER(d)]
    L.ftk_plan_tables.argtypes = [i, i, d, d, vp, i, ctypes.POINTER(i), vp, vp, vp, vp, vp, vp,
                                  ctypes.POINTER(d)]
    L.ftk_plan_profile.argtypes = [vp, i]
    L.ftk_plan_stage_times.argtypes = [vp, vp, vp, i]
    L.ftk_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.ftk_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.ftk_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Stack), i, i, i, vp]
    L.ftk_batch_run.argtypes = [vp, vp]
    L.ftk_batch_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    L.ftk_batch_destroy.argtypes = [vp]
    L.ftk_batch_destroy.restype = None
    L.ftk_mlp_create.argtypes = [ctypes.POINTER(vp), vp, i, i, i, i, i]
    L.ftk_mlp_destroy.argtypes = [vp]
    L.ftk_mlp_destroy.restype = None
    L.ftk_mlp_info.argtypes = [vp, ctypes.POINTER(MLPInfo)]
    L.ftk_mlp_set_layer.argtypes = [vp, i, vp, vp]
    L.ftk_mlp_get_layer.argtypes = [vp, i, vp, vp]
    L.ftk_mlp_set_input_norm.argtypes = [vp, vp, vp]
    L.ftk_features.argtypes = [vp, vp, i, i, i, i, vp, vp]
    L.ftk_mlp_forward.argtypes = [vp, vp, i, vp, vp]
    L.ftk_mlp_gradients.argtypes = [vp, vp, vp, vp, vp, i, vp, vp]
    L.ftk_mlp_get_grad.argtypes = [vp, i, vp, vp]
    f = ctypes.c_float
    L.ftk_mlp_train_step.argtypes = [vp, vp, vp, vp, vp, i, f, f, f, f, f, vp, vp]
    L.ftk_propose.argtypes = [vp, vp, i, i, vp, vp, vp, vp]
    L.ftk_align_lists.argtypes = [vp, vp, i, vp, i, vp, i, vp, vp]
    L.ftk_align_refined.argtypes = [vp, vp, vp, i, vp, i, i, vp, vp, vp, vp]
    L.ftk_best_template.argtypes = [vp, vp, i, i, vp, vp, vp]
    L.ftk_align_proposed.argtypes = [vp, vp, vp, i, vp, i, i, i, i, i, f, vp, vp, vp, ctypes.POINTER(i), vp]
    L.ftk_strerror.restype = ctypes.c_char_p
    L.ftk_strerror.argtypes = [i]
    L.ftk_last_error_message.restype = ctypes.c_char_p
    L.ftk_last_error_message.argtypes = []
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != FTK_OK:
        L = lib()
        raise FTKError(rc, where, L.ftk_last_error_message().decode() or L.ftk_strerror(rc).decode())


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _require_cuda(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _weight_arrays(weight):
    if weight is None:
        return None, None, 0
    a = np.ascontiguousarray(weight[0], dtype=np.float64).ravel()
    b = np.ascontiguousarray(weight[1], dtype=np.float64).ravel()
    if a.size != b.size:
        raise ValueError("weight: alpha and beta differ in length")
    return a, b, a.size


def ftk_plan_tables(n: int, K: int, W: float, eps: float, shifts_px=None, weight=None):
    """Host-only FP64 tables of the planner (no device work); weight =
    (alpha, beta) of the k-side weight, or None."""
    L = lib()
    H = ctypes.c_int(0)
    sn = ctypes.c_double(0)
    a, b, nt = _weight_arrays(weight)
    ap, bp = (a.ctypes.data, b.ctypes.data) if nt else (None, None)
    _check(L.ftk_plan_tables_weighted(n, K, W, eps, ap, bp, nt, None, 0, ctypes.byref(H), None, None, None, None,
                                      None, None, ctypes.byref(sn)), "ftk_plan_tables")
    H = H.value
    ell = np.zeros(H, np.int32)
    sig = np.zeros(H)
    G = np.zeros((H, K))
    k = np.zeros(K)
    w = np.zeros(K)
    N = 0
    Y = None
    sh = None
    if shifts_px is not None:
        sh = np.ascontiguousarray(shifts_px, dtype=np.float64).reshape(-1, 2)
        N = sh.shape[0]
        Y = np.zeros((N, H), np.complex128)
    Hc = ctypes.c_int(0)
    _check(L.ftk_plan_tables_weighted(n, K, W, eps, ap, bp, nt, sh.ctypes.data if sh is not None else None, N,
                                      ctypes.byref(Hc), ell.ctypes.data, sig.ctypes.data, G.ctypes.data, k.ctypes.data,
                                      w.ctypes.data, Y.ctypes.data if Y is not None else None, ctypes.byref(sn)),
           "ftk_plan_tables")
    return dict(H=H, ell=ell, sigma=sig, G=G, k=k, w=w, Y=Y, sigma_next=sn.value)


def _ctf(c) -> "Ctf":
    """Ctf from a dict with the ftk_ctf_t field names (or a Ctf)."""
    return c if isinstance(c, Ctf) else Ctf(**c)


def ftk_plan_tables_ctf(n: int, K: int, W: float, eps: float, ctf, shifts_px=None, defocus_A=None):
    """Host-only FP64 tables of a plan with a CTF (ftk_plan_tables_ctf)."""
    L = lib()
    c = _ctf(ctf)
    H = ctypes.c_int(0)
    sn = ctypes.c_double(0)
    _check(L.ftk_plan_tables_ctf(n, K, W, eps, ctypes.byref(c), None, None, 0, ctypes.byref(H), None, None, None,
                                 None, None, None, ctypes.byref(sn)), "ftk_plan_tables_ctf")
    H = H.value
    ell, sig, G, k, w = np.zeros(H, np.int32), np.zeros(H), np.zeros((H, K)), np.zeros(K), np.zeros(K)
    N, Y, sh, df = 0, None, None, None
    if shifts_px is not None:
        sh = np.ascontiguousarray(shifts_px, dtype=np.float64).reshape(-1, 2)
        df = np.ascontiguousarray(defocus_A, dtype=np.float64).reshape(-1)
        N = sh.shape[0]
        Y = np.zeros((N, H), np.complex128)
    _check(L.ftk_plan_tables_ctf(n, K, W, eps, ctypes.byref(c), sh.ctypes.data if sh is not None else None,
                                 df.ctypes.data if df is not None else None, N, ctypes.byref(ctypes.c_int(0)),
                                 ell.ctypes.data, sig.ctypes.data, G.ctypes.data, k.ctypes.data, w.ctypes.data,
                                 Y.ctypes.data if Y is not None else None, ctypes.byref(sn)), "ftk_plan_tables_ctf")
    return dict(H=H, ell=ell, sigma=sig, G=G, k=k, w=w, Y=Y, sigma_next=sn.value)


class Plan:
    """Owns an ftk_plan (ftk_plan_create / ftk_plan_destroy)."""

    def __init__(self, n: int, K: int, Q: int, W: float, eps: float, precision="fp32", weight=None, ctf=None):
        """weight: None, or (alpha, beta) of the k-side weight of the operator
        SVD (ftk_plan_create_weighted).  ctf: None, or the ftk_ctf_t fields
        as a dict (ftk_plan_create_ctf; poses then come from set_poses)."""
        L = lib()
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        if ctf is not None:
            c = _ctf(ctf)
            _check(L.ftk_plan_create_ctf(ctypes.byref(h), n, K, Q, W, eps, prec, ctypes.byref(c)),
                   "ftk_plan_create_ctf")
        else:
            a, b, nt = _weight_arrays(weight)
            _check(L.ftk_plan_create_weighted(ctypes.byref(h), n, K, Q, W, eps, prec, a.ctypes.data if nt else None,
                                              b.ctypes.data if nt else None, nt), "ftk_plan_create")
        self._h = h
        self.n, self.M, self.Qa = n, K, Q
        self.N = 0
        self.up = 1

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ftk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().ftk_plan_info(self._h, ctypes.byref(inf)), "ftk_plan_info")
        return inf.as_dict()

    STAGES = ("transform", "step1", "step3", "bookkeeping", "operand_prep", "bft_translate", "bfr_spectra",
              "bfr_correlation")

    def profile(self, enable: bool = True):
        _check(lib().ftk_plan_profile(self._h, 1 if enable else 0), "ftk_plan_profile")

    def stage_times(self) -> dict:
        """Per-stage (milliseconds, launches) since profile() or the last read."""
        ms = np.zeros(len(self.STAGES))
        cnt = np.zeros(len(self.STAGES), np.int64)
        _check(lib().ftk_plan_stage_times(self._h, ms.ctypes.data, cnt.ctypes.data, len(self.STAGES)),
               "ftk_plan_stage_times")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(self.STAGES)}

    def tuning(self) -> dict:
        t = Tuning()
        _check(lib().ftk_plan_get_tuning(self._h, ctypes.byref(t)), "ftk_plan_get_tuning")
        return t.as_dict()

    def set_tuning(self, step3_waves=0, step1_zblk=0, step1_wgs=0, stage_mib=0):
        t = Tuning(step3_waves, step1_zblk, step1_wgs, stage_mib)
        _check(lib().ftk_plan_set_tuning(self._h, ctypes.byref(t)), "ftk_plan_set_tuning")

    def set_shift_windows(self, centers_px, half_width_px: float):
        """ftk_plan_set_shift_windows: annuli of shifts for the proposal's
        restricted search (empty centers removes them)."""
        c = np.ascontiguousarray(centers_px, dtype=np.float64).reshape(-1)
        _check(lib().ftk_plan_set_shift_windows(self._h, c.ctypes.data if c.size else None, c.size,
                                                float(half_width_px)), "ftk_plan_set_shift_windows")

    def set_rotations(self, upsample: int):
        """ftk_plan_set_rotations: U * Qa rotations (rotation upsampling)."""
        _check(lib().ftk_plan_set_rotations(self._h, int(upsample)), "ftk_plan_set_rotations")
        self.up = int(upsample)

    def set_poses(self, shifts_px, defocus_A):
        """ftk_set_poses: pose i = (shift_i, defocus_i) of a plan with a CTF."""
        sh = np.ascontiguousarray(shifts_px, dtype=np.float64).reshape(-1, 2)
        df = np.ascontiguousarray(defocus_A, dtype=np.float64).reshape(-1)
        if df.size != sh.shape[0]:
            raise ValueError("one defocus per shift")
        _check(lib().ftk_set_poses(self._h, sh.ctypes.data, df.ctypes.data, sh.shape[0]), "ftk_set_poses")
        self.N = sh.shape[0]

    def set_shifts(self, shifts_px):
        sh = np.ascontiguousarray(shifts_px, dtype=np.float64).reshape(-1, 2)
        _check(lib().ftk_set_shifts(self._h, sh.ctypes.data, sh.shape[0]), "ftk_set_shifts")
        self.N = sh.shape[0]

    def transform(self, imgs, coeffs=None, stream=None):
        import torch
        _require_cuda(imgs, torch.float32, "imgs")
        cnt = imgs.shape[0]
        if coeffs is None:
            coeffs = torch.empty((cnt, self.Qa, self.M), dtype=torch.complex64, device=imgs.device)
        _require_cuda(coeffs, torch.complex64, "coeffs")
        _check(lib().ftk_transform(self._h, _ptr(imgs), cnt, _ptr(coeffs), _stream(stream)), "ftk_transform")
        return coeffs

    def _outputs(self, nA, nB, want_X, device, X, best):
        import torch
        if want_X and X is None:
            X = torch.empty((nA, nB, self.N, self.Qa * self.up), dtype=torch.float32, device=device)
        if best is None:
            best = torch.empty((nA, nB, 3), dtype=torch.int32, device=device)
        return X, best

    def align_coeffs(self, a, b, want_X=False, X=None, best=None, stream=None):
        import torch
        _require_cuda(a, torch.complex64, "img_coeffs")
        _require_cuda(b, torch.complex64, "tmpl_coeffs")
        X, best = self._outputs(a.shape[0], b.shape[0], want_X, a.device, X, best)
        _check(lib().ftk_align_coeffs(self._h, _ptr(a), a.shape[0], _ptr(b), b.shape[0], _ptr(X), _ptr(best),
                                      _stream(stream)), "ftk_align_coeffs")
        return X, best

    def align_coeffs_noalloc(self, a, b, X=None, best=None, stream=None):
        """ftk_align_coeffs_noalloc: the caller passes the outputs (X and/or
        best, device tensors); the library allocates nothing."""
        import torch
        _require_cuda(a, torch.complex64, "img_coeffs")
        _require_cuda(b, torch.complex64, "tmpl_coeffs")
        _check(lib().ftk_align_coeffs_noalloc(self._h, _ptr(a), a.shape[0], _ptr(b), b.shape[0], _ptr(X), _ptr(best),
                                              _stream(stream)), "ftk_align_coeffs_noalloc")
        return X, best

    def align(self, images, templates, want_X=False, X=None, best=None, stream=None):
        import torch
        _require_cuda(images, torch.float32, "images")
        _require_cuda(templates, torch.float32, "templates")
        X, best = self._outputs(images.shape[0], templates.shape[0], want_X, images.device, X, best)
        _check(lib().ftk_align(self._h, _ptr(images), images.shape[0], _ptr(templates), templates.shape[0],
                               _ptr(X), _ptr(best), _stream(stream)), "ftk_align")
        return X, best

    def bft_align(self, images, templates, want_X=False, X=None, best=None, stream=None):
        """ftk_bft_align: brute-force translations (the paper's comparison
        method, FP32) on this plan's grids and shifts; outputs as align()."""
        import torch
        _require_cuda(images, torch.float32, "images")
        _require_cuda(templates, torch.float32, "templates")
        X, best = self._outputs(images.shape[0], templates.shape[0], want_X, images.device, X, best)
        _check(lib().ftk_bft_align(self._h, _ptr(images), images.shape[0], _ptr(templates), templates.shape[0],
                                   _ptr(X), _ptr(best), _stream(stream)), "ftk_bft_align")
        return X, best

    def bfr_align(self, images, templates, want_X=False, X=None, best=None, stream=None):
        """ftk_bfr_align: brute-force rotations (the paper's other comparison
        method, FP32) on this plan's shifts and rotations; outputs as align()."""
        import torch
        _require_cuda(images, torch.float32, "images")
        _require_cuda(templates, torch.float32, "templates")
        X, best = self._outputs(images.shape[0], templates.shape[0], want_X, images.device, X, best)
        _check(lib().ftk_bfr_align(self._h, _ptr(images), images.shape[0], _ptr(templates), templates.shape[0],
                                   _ptr(X), _ptr(best), _stream(stream)), "ftk_bfr_align")
        return X, best


class Batch:
    """Owns an ftk_batch over stacks (plan, images, templates[, X], best).

    The torch tensors of every stack are kept referenced for the batch's
    lifetime (the C object holds their addresses)."""

    def __init__(self, stacks, lanes: int = 1, graph: bool = False, autotune: bool = False, stream=None):
        import torch
        arr = (Stack * max(1, len(stacks)))()
        self._keep = []
        for i, st in enumerate(stacks):
            plan, imgs, tmps = st["plan"], st["images"], st["templates"]
            _require_cuda(imgs, torch.float32, "images")
            _require_cuda(tmps, torch.float32, "templates")
            X, best = st.get("X"), st.get("best")
            if best is not None:
                _require_cuda(best, torch.int32, "best")
            if X is not None:
                _require_cuda(X, torch.float32, "X")
            arr[i] = Stack(plan._h.value, imgs.data_ptr(), imgs.shape[0], tmps.data_ptr(), tmps.shape[0],
                           X.data_ptr() if X is not None else None, best.data_ptr() if best is not None else None)
            self._keep.append((plan, imgs, tmps, X, best))
        flags = (FTK_BATCH_GRAPH if graph else 0) | (FTK_BATCH_AUTOTUNE if autotune else 0)
        h = ctypes.c_void_p()
        _check(lib().ftk_batch_create(ctypes.byref(h), arr, len(stacks), lanes, flags, _stream(stream)),
               "ftk_batch_create")
        self._h = h

    def run(self, stream=None):
        _check(lib().ftk_batch_run(self._h, _stream(stream)), "ftk_batch_run")

    def info(self) -> dict:
        inf = BatchInfo()
        _check(lib().ftk_batch_info(self._h, ctypes.byref(inf)), "ftk_batch_info")
        return inf.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ftk_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _i32(t, name):
    import torch
    _require_cuda(t, torch.int32, name)
    return _ptr(t)


class MLP:
    """Owns an ftk_mlp (the template-proposal network)."""

    def __init__(self, dims, n_template: int, n_shift: int, precision="bf16", max_batch: int = 1024):
        dims = [int(d) for d in dims]
        arr = (ctypes.c_int * len(dims))(*dims)
        prec = MLP_PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        _check(lib().ftk_mlp_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), len(dims) - 1, n_template,
                                    n_shift, prec, max_batch), "ftk_mlp_create")
        self._h = h
        self.dims, self.n_template, self.n_shift, self.max_batch = dims, n_template, n_shift, max_batch

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ftk_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = MLPInfo()
        _check(lib().ftk_mlp_info(self._h, ctypes.byref(inf)), "ftk_mlp_info")
        return inf.as_dict()

    def set_layer(self, layer: int, W, b):
        W = np.ascontiguousarray(W, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        if W.shape != (self.dims[layer + 1], self.dims[layer]) or b.shape != (self.dims[layer + 1],):
            raise ValueError("layer shape mismatch")
        _check(lib().ftk_mlp_set_layer(self._h, layer, W.ctypes.data, b.ctypes.data), "ftk_mlp_set_layer")

    def get_layer(self, layer: int):
        W = np.zeros((self.dims[layer + 1], self.dims[layer]), np.float32)
        b = np.zeros(self.dims[layer + 1], np.float32)
        _check(lib().ftk_mlp_get_layer(self._h, layer, W.ctypes.data, b.ctypes.data), "ftk_mlp_get_layer")
        return W, b

    def set_params(self, params):
        for l, (W, b) in enumerate(params):
            self.set_layer(l, W, b)

    def params(self):
        return [self.get_layer(l) for l in range(len(self.dims) - 1)]

    def set_input_norm(self, mu, inv_sigma):
        mu = np.ascontiguousarray(mu, dtype=np.float32)
        inv_sigma = np.ascontiguousarray(inv_sigma, dtype=np.float32)
        _check(lib().ftk_mlp_set_input_norm(self._h, mu.ctypes.data, inv_sigma.ctypes.data), "ftk_mlp_set_input_norm")

    def forward(self, x, logits=None, stream=None):
        import torch
        _require_cuda(x, torch.float32, "x")
        if logits is None:
            logits = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device=x.device)
        _check(lib().ftk_mlp_forward(self._h, _ptr(x), x.shape[0], _ptr(logits), _stream(stream)), "ftk_mlp_forward")
        return logits

    def gradients(self, x_all, lab_t, lab_s, idx, loss=None, stream=None):
        import torch
        _require_cuda(x_all, torch.float32, "x_all")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x_all.device)
        _check(lib().ftk_mlp_gradients(self._h, _ptr(x_all), _i32(lab_t, "lab_t"),
                                       _i32(lab_s, "lab_s") if lab_s is not None else None, _i32(idx, "idx"),
                                       idx.shape[0], _ptr(loss), _stream(stream)), "ftk_mlp_gradients")
        return loss

    def grad(self, layer: int):
        dW = np.zeros((self.dims[layer + 1], self.dims[layer]), np.float32)
        db = np.zeros(self.dims[layer + 1], np.float32)
        _check(lib().ftk_mlp_get_grad(self._h, layer, dW.ctypes.data, db.ctypes.data), "ftk_mlp_get_grad")
        return dW, db

    def train_step(self, x_all, lab_t, lab_s, idx, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0, loss=None,
                   stream=None):
        import torch
        _require_cuda(x_all, torch.float32, "x_all")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=x_all.device)
        _check(lib().ftk_mlp_train_step(self._h, _ptr(x_all), _i32(lab_t, "lab_t"),
                                        _i32(lab_s, "lab_s") if lab_s is not None else None, _i32(idx, "idx"),
                                        idx.shape[0], lr, beta1, beta2, eps, wd, _ptr(loss), _stream(stream)),
               "ftk_mlp_train_step")
        return loss

    def propose(self, x, topk: int, stream=None):
        import torch
        _require_cuda(x, torch.float32, "x")
        n = x.shape[0]
        top = torch.empty((n, topk), dtype=torch.int32, device=x.device)
        mass = torch.empty(n, dtype=torch.float32, device=x.device)
        sbin = torch.empty(n, dtype=torch.int32, device=x.device)
        _check(lib().ftk_propose(self._h, _ptr(x), n, topk, _ptr(top), _ptr(mass), _ptr(sbin), _stream(stream)),
               "ftk_propose")
        return top, mass, sbin


FTK_FEATURES_POWER = 0
FTK_FEATURES_CROSS = 1
FTK_FEATURES_INVARIANT = 2
FEATURE_KINDS = {"power": FTK_FEATURES_POWER, "cross": FTK_FEATURES_CROSS, "invariant": FTK_FEATURES_INVARIANT}


def feature_count(kind, n_r: int, n_q: int) -> int:
    k = FEATURE_KINDS[kind] if isinstance(kind, str) else int(kind)
    return n_r * n_r * n_q if k == FTK_FEATURES_CROSS else n_r * n_q


def features(plan: "Plan", coeffs, n_r: int, n_q: int, kind="power", out=None, stream=None):
    import torch
    _require_cuda(coeffs, torch.complex64, "coeffs")
    k = FEATURE_KINDS[kind] if isinstance(kind, str) else int(kind)
    if out is None:
        out = torch.empty((coeffs.shape[0], feature_count(k, n_r, n_q)), dtype=torch.float32, device=coeffs.device)
    _check(lib().ftk_features(plan._h, _ptr(coeffs), coeffs.shape[0], k, n_r, n_q, _ptr(out), _stream(stream)),
           "ftk_features")
    return out


def best_template(poses, lists=None, stream=None):
    """Per-image best over the pairs of poses [nA][K][3] (int32 view)."""
    import torch
    _require_cuda(poses, torch.int32, "poses")
    nA, K = poses.shape[0], poses.shape[1]
    bt = torch.empty(nA, dtype=torch.int32, device=poses.device)
    bp = torch.empty((nA, 3), dtype=torch.int32, device=poses.device)
    _check(lib().ftk_best_template(_ptr(poses), _i32(lists, "lists") if lists is not None else None, nA, K, _ptr(bt),
                                   _ptr(bp), _stream(stream)), "ftk_best_template")
    return bt, bp


def align_refined(coarse: "Plan", fine: "Plan", a, b, k: int, best=None, stream=None):
    """Two-pass alignment (ftk_align_refined): poses of every pair [nA][nB][3],
    then the best template [nA] and its pose [nA][3] after refinement."""
    import torch
    _require_cuda(a, torch.complex64, "img_coeffs")
    _require_cuda(b, torch.complex64, "tmpl_coeffs")
    nA, nB = a.shape[0], b.shape[0]
    if best is None:
        best = torch.empty((nA, nB, 3), dtype=torch.int32, device=a.device)
    bt = torch.empty(nA, dtype=torch.int32, device=a.device)
    bp = torch.empty((nA, 3), dtype=torch.int32, device=a.device)
    _check(lib().ftk_align_refined(coarse._h, fine._h, _ptr(a), nA, _ptr(b), nB, k, _ptr(best), _ptr(bt), _ptr(bp),
                                   _stream(stream)), "ftk_align_refined")
    return best, bt, bp


def align_lists(plan: "Plan", a, b, lists, stream=None):
    import torch
    _require_cuda(a, torch.complex64, "img_coeffs")
    _require_cuda(b, torch.complex64, "tmpl_coeffs")
    nA, K = lists.shape
    best = torch.empty((nA, K, 3), dtype=torch.int32, device=a.device)
    _check(lib().ftk_align_lists(plan._h, _ptr(a), a.shape[0], _ptr(b), b.shape[0], _i32(lists, "lists"), K,
                                 _ptr(best), _stream(stream)), "ftk_align_lists")
    return best


def align_proposed(plan: "Plan", mlp: MLP, images, tmpl_coeffs, n_r: int, n_q: int, topk: int, tau: float,
                   kind="power", stream=None):
    """Proposal search: (best template [nA], best pose [nA][3], fallback flags [nA], fallback count)."""
    import torch
    _require_cuda(images, torch.float32, "images")
    _require_cuda(tmpl_coeffs, torch.complex64, "tmpl_coeffs")
    nA = images.shape[0]
    k = FEATURE_KINDS[kind] if isinstance(kind, str) else int(kind)
    bt = torch.empty(nA, dtype=torch.int32, device=images.device)
    bp = torch.empty((nA, 3), dtype=torch.int32, device=images.device)
    fb = torch.empty(nA, dtype=torch.int32, device=images.device)
    cnt = ctypes.c_int(0)
    _check(lib().ftk_align_proposed(plan._h, mlp._h, _ptr(images), nA, _ptr(tmpl_coeffs), tmpl_coeffs.shape[0], k,
                                    n_r, n_q, topk, tau, _ptr(bt), _ptr(bp), _ptr(fb), ctypes.byref(cnt),
                                    _stream(stream)), "ftk_align_proposed")
    return bt, bp, fb, cnt.value


def poses_numpy(best) -> np.ndarray:
    """Device ftk_pose tensor [..., 3] (int32 view) -> structured numpy array."""
    raw = best.detach().cpu().numpy().astype(np.int32, copy=False)
    return raw.view(POSE_DTYPE).reshape(raw.shape[:-1])
