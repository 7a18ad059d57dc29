"""Python binding of libks (C ABI in include/ks.h): argument marshalling only.

Every step of the smoother runs in the HIP kernels of libks.so; this module
checks tensor shapes, dtypes and devices, allocates outputs and the workspace
with torch (device memory and streams are the only things torch provides), and
calls the C entry points with raw device pointers.  There is no CPU fallback:
if the library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libks.so")
TUNE_PATH = os.path.join(_HERE, "tune_mi355x.json")  # autotuned schedule table (autotune.py)

KS_OK, KS_E_ARG, KS_E_WORKSPACE, KS_E_NOT_SPD, KS_E_RANK = 0, -1, -2, -3, -4
KS_E_NONFINITE, KS_E_HIP, KS_E_ORDER, KS_E_BUSY = -5, -6, -7, -8
KS_FP64, KS_FP32_FORM = 0, 1
KS_COV_DENSE, KS_COV_DIAG = 0, 1

SYMBOLS = ("ks_workspace_bytes", "ks_supported", "ks_create", "ks_smooth", "ks_covariances",
           "ks_smooth_cov", "ks_destroy", "ks_status_string", "ks_plan_layout",
           "ks_time_kernels", "ks_kernel_time", "ks_batch_workspace_bytes", "ks_batch_create",
           "ks_batch_smooth", "ks_batch_destroy", "ks_engine_create", "ks_engine_submit",
           "ks_engine_step", "ks_engine_wait", "ks_engine_retired", "ks_engine_poll", "ks_engine_query", "ks_engine_destroy",
           "ks_set_tuning", "ks_get_tuning", "ks_plan_schedule", "ks_smooth_cov_lag1", "ks_objective",
           "ks_smooth_cov_static", "ks_kernel_variants")
KS_TIME_OFF, KS_TIME_FWD_LEVEL0, KS_TIME_BWD_LEVEL0, KS_TIME_FWD_ALL, KS_TIME_BWD_ALL = range(5)


class Desc(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("n", ctypes.c_int32), ("m", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("K_layout", ctypes.c_int32),
                ("C_layout", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("fwd_tail_passes", ctypes.c_int32), ("bwd_tail_passes", ctypes.c_int32),
                ("fp32_switch_columns", ctypes.c_int64), ("fwd_group", ctypes.c_int32),
                ("fwd_group_from", ctypes.c_int32), ("bwd_group", ctypes.c_int32),
                ("bwd_group_from", ctypes.c_int32), ("fwd_variant", ctypes.c_int32),
                ("bwd_variant", ctypes.c_int32)]


TUNING_KEYS = tuple(f for f, _t in Tuning._fields_)
TUNING_DEFAULTS = dict(fwd_tail_passes=2, bwd_tail_passes=2, fp32_switch_columns=1024, fwd_group=1,
                       fwd_group_from=1, bwd_group=1, bwd_group_from=1, fwd_variant=0, bwd_variant=0)


class Layout(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("rrow_offset", ctypes.c_int64),
                ("rrow_stride", ctypes.c_int64), ("level_rec_offset", ctypes.c_int64 * 64),
                ("level_columns", ctypes.c_int64 * 64)]


class Io(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in ("H", "F", "c", "K", "G", "o", "C", "u_out", "cov_out")]


class EngineStats(ctypes.Structure):
    _fields_ = [("inflight", ctypes.c_int64), ("retired_pending", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("region_bytes", ctypes.c_size_t), ("free_bytes", ctypes.c_size_t),
                ("largest_free", ctypes.c_size_t), ("ticks_pending", ctypes.c_int64)]


class KsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = lib().ks_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)
        self.status = status


_lib = None


def lib():
    """Load libks.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the smoother has no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.c_void_p
    L.ks_workspace_bytes.restype = ctypes.c_size_t
    L.ks_workspace_bytes.argtypes = [ctypes.POINTER(Desc)]
    L.ks_supported.restype = ctypes.c_int
    L.ks_supported.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.ks_create.restype = ctypes.c_int
    L.ks_create.argtypes = [ctypes.POINTER(Desc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ks_smooth.restype = ctypes.c_int
    L.ks_smooth.argtypes = [vp] + [dp] * 8
    L.ks_smooth_cov.restype = ctypes.c_int
    L.ks_smooth_cov.argtypes = [vp] + [dp] * 9
    L.ks_smooth_cov_lag1.restype = ctypes.c_int
    L.ks_smooth_cov_lag1.argtypes = [vp] + [dp] * 10
    L.ks_objective.restype = ctypes.c_int
    L.ks_objective.argtypes = [vp] + [dp] * 9 + [ctypes.POINTER(ctypes.c_double)]
    L.ks_covariances.restype = ctypes.c_int
    L.ks_covariances.argtypes = [vp, dp]
    L.ks_destroy.restype = ctypes.c_int
    L.ks_destroy.argtypes = [vp]
    L.ks_status_string.restype = ctypes.c_char_p
    L.ks_status_string.argtypes = [ctypes.c_int]
    L.ks_plan_layout.restype = ctypes.c_int
    L.ks_plan_layout.argtypes = [vp, ctypes.POINTER(Layout)]
    L.ks_time_kernels.restype = ctypes.c_int
    L.ks_time_kernels.argtypes = [vp, ctypes.c_int32]
    L.ks_kernel_time.restype = ctypes.c_int
    L.ks_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.ks_batch_workspace_bytes.restype = ctypes.c_size_t
    L.ks_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc)]
    L.ks_batch_create.restype = ctypes.c_int
    L.ks_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc), vp, ctypes.c_size_t, vp,
                                  ctypes.POINTER(vp)]
    L.ks_batch_smooth.restype = ctypes.c_int
    L.ks_batch_smooth.argtypes = [vp, ctypes.POINTER(Io), ctypes.c_int32, ctypes.POINTER(ctypes.c_int)]
    L.ks_batch_destroy.restype = ctypes.c_int
    L.ks_batch_destroy.argtypes = [vp]
    L.ks_engine_create.restype = ctypes.c_int
    L.ks_engine_create.argtypes = [vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ks_engine_submit.restype = ctypes.c_int
    L.ks_engine_submit.argtypes = [vp, ctypes.POINTER(Desc), ctypes.POINTER(Io), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_uint64)]
    L.ks_engine_step.restype = ctypes.c_int
    L.ks_engine_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.ks_engine_wait.restype = ctypes.c_int
    L.ks_engine_wait.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.ks_engine_retired.restype = ctypes.c_int
    L.ks_engine_retired.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64),
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int32)]
    L.ks_engine_poll.restype = ctypes.c_int
    L.ks_engine_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    L.ks_engine_query.restype = ctypes.c_int
    L.ks_engine_query.argtypes = [vp, ctypes.POINTER(EngineStats)]
    L.ks_engine_destroy.restype = ctypes.c_int
    L.ks_engine_destroy.argtypes = [vp]
    L.ks_set_tuning.restype = ctypes.c_int
    L.ks_set_tuning.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Tuning)]
    L.ks_get_tuning.restype = ctypes.c_int
    L.ks_get_tuning.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Tuning)]
    L.ks_plan_schedule.restype = ctypes.c_int
    L.ks_plan_schedule.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]
    L.ks_kernel_variants.restype = ctypes.c_int32
    L.ks_kernel_variants.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.ks_smooth_cov_static.restype = ctypes.c_int
    L.ks_smooth_cov_static.argtypes = [ctypes.POINTER(Desc)] + [dp] * 9 + [vp]
    _lib = L
    if not os.environ.get("KS_NO_TUNE"):
        path = os.environ.get("KS_TUNE_FILE", TUNE_PATH)
        if os.path.exists(path):
            load_tuning(path)
    return L


def set_tuning(n: int, fp32: bool, **values):
    """Set the schedule choices of (n, form); keys of TUNING_KEYS, missing ones
    keep their current value."""
    cur = get_tuning(n, fp32)
    unknown = set(values) - set(TUNING_KEYS)
    if unknown:
        raise ValueError(f"unknown tuning keys {sorted(unknown)}")
    cur.update(values)
    t = Tuning(**{k: int(cur[k]) for k in TUNING_KEYS})
    st = lib().ks_set_tuning(int(n), KS_FP32_FORM if fp32 else KS_FP64, ctypes.byref(t))
    if st != KS_OK:
        raise KsError(st, "ks_set_tuning")


def get_tuning(n: int, fp32: bool = False) -> dict:
    t = Tuning()
    st = lib().ks_get_tuning(int(n), KS_FP32_FORM if fp32 else KS_FP64, ctypes.byref(t))
    if st != KS_OK:
        raise KsError(st, "ks_get_tuning")
    return {k: getattr(t, k) for k in TUNING_KEYS}


def load_tuning(path: str) -> int:
    """Apply a tuning table written by autotune.py; returns the entries applied."""
    import json
    with open(path) as fh:
        table = json.load(fh)
    for e in table.get("entries", []):
        vals = {k: e.get(k, TUNING_DEFAULTS[k]) for k in TUNING_KEYS}
        set_tuning(e["n"], e["form"] == "fp32", **vals)
    return len(table.get("entries", []))


def kernel_variants(n: int, m: int, backward: bool) -> int:
    """Compiled forward / backward shape variants of (n, m)."""
    return int(lib().ks_kernel_variants(int(n), int(m), 1 if backward else 0))


def make_desc(k: int, n: int, m: int, K_diag: bool, C_diag: bool, fp32: bool = False) -> Desc:
    return Desc(k=int(k), n=int(n), m=int(m), precision=KS_FP32_FORM if fp32 else KS_FP64,
                K_layout=KS_COV_DIAG if K_diag else KS_COV_DENSE,
                C_layout=KS_COV_DIAG if C_diag else KS_COV_DENSE, flags=0)


def workspace_bytes(k: int, n: int, m: int, K_diag: bool, C_diag: bool, fp32: bool = False) -> int:
    d = make_desc(k, n, m, K_diag, C_diag, fp32)
    return int(lib().ks_workspace_bytes(ctypes.byref(d)))


def supported(n: int, m: int) -> bool:
    return bool(lib().ks_supported(int(n), int(m)))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(t: Optional[torch.Tensor], name: str, shape, device, allow_none=False):
    if t is None:
        if allow_none:
            return
        raise ValueError(f"{name} is required")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _device(device) -> torch.device:
    """A CUDA/HIP device with its index (``"cuda"`` means the current one)."""
    d = torch.device(device) if device is not None else torch.device("cuda")
    if d.type != "cuda":
        raise ValueError(f"libks runs on GPU devices only, got {d}")
    return d if d.index is not None else torch.device("cuda", torch.cuda.current_device())


def _make_io(shape, args, u, cov, device) -> Io:
    """Check one problem's device tensors against its shape
    (k, n, m, K_diag, C_diag, fp32) and return their pointers."""
    k, n, m, kd, cd = shape[:5]
    H, F, c, K, G, o, C = args
    _check(H, "H", (k, n, n), device, allow_none=True)
    _check(F, "F", (k, n, n), device)
    _check(c, "c", (k, n), device)
    _check(K, "K", (k, n) if kd else (k, n, n), device)
    _check(G, "G", (k + 1, m, n), device)
    _check(o, "o", (k + 1, m), device)
    _check(C, "C", (k + 1, m) if cd else (k + 1, m, m), device)
    _check(u, "u_out", (k + 1, n), device)
    if cov is not None:
        _check(cov, "cov_out", (k + 1, n, n), device)
    return Io(*[None if t is None else t.data_ptr() for t in (H, F, c, K, G, o, C)],
              u.data_ptr(), None if cov is None else cov.data_ptr())


class Plan:
    """A smoothing plan for one problem shape, owning its device workspace."""

    def __init__(self, k: int, n: int, m: int, K_diag: bool, C_diag: bool,
                 device: Optional[torch.device] = None, stream: Optional[torch.cuda.Stream] = None,
                 fp32: bool = False):
        self.k, self.n, self.m = int(k), int(n), int(m)
        self.K_diag, self.C_diag = bool(K_diag), bool(C_diag)
        self.fp32 = bool(fp32)
        self.device = _device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._desc = make_desc(k, n, m, K_diag, C_diag, fp32)
        L = lib()
        nbytes = int(L.ks_workspace_bytes(ctypes.byref(self._desc)))
        if nbytes == 0:
            raise KsError(KS_E_ARG, f"unsupported problem (k={k}, n={n}, m={m})")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        h = ctypes.c_void_p()
        st = L.ks_create(ctypes.byref(self._desc), ctypes.c_void_p(self._ws_ptr), nbytes,
                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != KS_OK:
            raise KsError(st, "ks_create")
        self._h = h

    # ---------------------------------------------------------------- checks
    def _check_inputs(self, H, F, c, K, G, o, C):
        k, n, m, dev = self.k, self.n, self.m, self.device
        _check(H, "H", (k, n, n), dev, allow_none=True)
        _check(F, "F", (k, n, n), dev)
        _check(c, "c", (k, n), dev)
        _check(K, "K", (k, n) if self.K_diag else (k, n, n), dev)
        _check(G, "G", (k + 1, m, n), dev)
        _check(o, "o", (k + 1, m), dev)
        _check(C, "C", (k + 1, m) if self.C_diag else (k + 1, m, m), dev)

    def _out(self, t, shape, name):
        if t is None:
            return torch.empty(shape, dtype=torch.float64, device=self.device)
        _check(t, name, shape, self.device)
        return t

    # ------------------------------------------------------------ entry points
    def smooth(self, H, F, c, K, G, o, C, u_out=None):
        """States only (no covariances); the R factor stays in the workspace."""
        self._check_inputs(H, F, c, K, G, o, C)
        u = self._out(u_out, (self.k + 1, self.n), "u_out")
        st = lib().ks_smooth(self._h, _ptr(H), _ptr(F), _ptr(c), _ptr(K), _ptr(G), _ptr(o),
                             _ptr(C), _ptr(u))
        if st != KS_OK:
            raise KsError(st, "ks_smooth")
        return u

    def smooth_cov(self, H, F, c, K, G, o, C, u_out=None, cov_out=None):
        """States and covariance blocks in one pass."""
        self._check_inputs(H, F, c, K, G, o, C)
        u = self._out(u_out, (self.k + 1, self.n), "u_out")
        cov = self._out(cov_out, (self.k + 1, self.n, self.n), "cov_out")
        st = lib().ks_smooth_cov(self._h, _ptr(H), _ptr(F), _ptr(c), _ptr(K), _ptr(G), _ptr(o),
                                 _ptr(C), _ptr(u), _ptr(cov))
        if st != KS_OK:
            raise KsError(st, "ks_smooth_cov")
        return u, cov

    def smooth_cov_lag1(self, H, F, c, K, G, o, C, u_out=None, cov_out=None, lag1_out=None):
        """States, covariance blocks and the lag-one blocks S_{i,i+1} in one pass."""
        self._check_inputs(H, F, c, K, G, o, C)
        u = self._out(u_out, (self.k + 1, self.n), "u_out")
        cov = self._out(cov_out, (self.k + 1, self.n, self.n), "cov_out")
        lag1 = self._out(lag1_out, (self.k, self.n, self.n), "lag1_out")
        st = lib().ks_smooth_cov_lag1(self._h, _ptr(H), _ptr(F), _ptr(c), _ptr(K), _ptr(G), _ptr(o),
                                      _ptr(C), _ptr(u), _ptr(cov), _ptr(lag1) if self.k > 0 else None)
        if st != KS_OK:
            raise KsError(st, "ks_smooth_cov_lag1")
        return u, cov, lag1

    def objective(self, H, F, c, K, G, o, C, u=None, terms_out=None) -> float:
        """||U(Au - b)||^2 at u (None: u = 0, which needs only c, K, o, C);
        terms_out, if given, receives the per-step terms."""
        k, n, m, dev = self.k, self.n, self.m, self.device
        if u is not None:
            _check(u, "u", (k + 1, n), dev)
            self._check_inputs(H, F, c, K, G, o, C)
        else:
            _check(c, "c", (k, n), dev)
            _check(K, "K", (k, n) if self.K_diag else (k, n, n), dev)
            _check(o, "o", (k + 1, m), dev)
            _check(C, "C", (k + 1, m) if self.C_diag else (k + 1, m, m), dev)
            H = F = G = None
        if terms_out is not None:
            _check(terms_out, "terms_out", (k + 1,), dev)
        total = ctypes.c_double()
        st = lib().ks_objective(self._h, _ptr(H), _ptr(F), _ptr(c), _ptr(K), _ptr(G), _ptr(o), _ptr(C),
                                _ptr(u), _ptr(terms_out), ctypes.byref(total))
        if st != KS_OK:
            raise KsError(st, "ks_objective")
        return total.value

    def covariances(self, cov_out=None):
        """Covariance blocks from the R factor of the last successful smooth."""
        cov = self._out(cov_out, (self.k + 1, self.n, self.n), "cov_out")
        st = lib().ks_covariances(self._h, _ptr(cov))
        if st != KS_OK:
            raise KsError(st, "ks_covariances")
        return cov

    def schedule(self) -> dict:
        """FP32 levels, first forward-tail level, lowest backward-tail level."""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        st = lib().ks_plan_schedule(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        if st != KS_OK:
            raise KsError(st, "ks_plan_schedule")
        return dict(fp32_levels=a.value, fwd_tail_level=b.value, bwd_tail_level=c.value)

    def layout(self) -> dict:
        lay = Layout()
        st = lib().ks_plan_layout(self._h, ctypes.byref(lay))
        if st != KS_OK:
            raise KsError(st, "ks_plan_layout")
        lv = lay.levels
        return dict(levels=lv, rrow_offset=lay.rrow_offset, rrow_stride=lay.rrow_stride,
                    level_rec_offset=list(lay.level_rec_offset[:lv]),
                    level_columns=list(lay.level_columns[:lv]))

    def r_records(self) -> torch.Tensor:
        """The R-factor records in the workspace, as a [(k+1), n, 3n+1] view."""
        lay = self.layout()
        n = self.n
        off = self._ws_ptr - self.workspace.data_ptr()
        words = self.workspace[off:off + self.ws_bytes].view(torch.float64)
        start = lay["rrow_offset"]
        return words[start:start + (self.k + 1) * lay["rrow_stride"]].view(self.k + 1, n, 3 * n + 1)

    def time_kernels(self, kind: int):
        """Bracket the selected launches of later calls with hipEvents (0 = off)."""
        st = lib().ks_time_kernels(self._h, int(kind))
        if st != KS_OK:
            raise KsError(st, "ks_time_kernels")

    def kernel_time(self):
        """(total milliseconds, number of bracketed launches) since time_kernels."""
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        st = lib().ks_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(cnt))
        if st != KS_OK:
            raise KsError(st, "ks_kernel_time")
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().ks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STATIC_SCRATCH_BYTES = 64 << 20  # KS_STATIC_SCRATCH_BYTES of include/ks.h


def smooth_cov_static(shape, inputs, u_out=None, cov_out=None, device=None, stream=None):
    """States and covariances through ks_smooth_cov_static (the library's
    static device array as working memory; nothing allocated on the device
    beyond the outputs when they are not given).  shape = (k, n, m, K_diag,
    C_diag, fp32); inputs = (H, F, c, K, G, o, C) device tensors."""
    k, n = int(shape[0]), int(shape[1])
    dev = _device(device)
    st_obj = stream if stream is not None else torch.cuda.current_stream(dev)
    u = u_out if u_out is not None else torch.empty((k + 1, n), dtype=torch.float64, device=dev)
    cov = cov_out if cov_out is not None else torch.empty((k + 1, n, n), dtype=torch.float64, device=dev)
    io = _make_io(shape, inputs, u, cov, dev)
    d = make_desc(*shape)
    st = lib().ks_smooth_cov_static(ctypes.byref(d), io.H, io.F, io.c, io.K, io.G, io.o, io.C, io.u_out,
                                    io.cov_out, ctypes.c_void_p(st_obj.cuda_stream))
    if st != KS_OK:
        raise KsError(st, "ks_smooth_cov_static")
    return u, cov


def to_device(p, device="cuda"):
    """Problem arrays (numpy, from gen) as float64 device tensors in ABI order."""
    def t(a):
        return None if a is None else torch.from_numpy(a).to(device=device, dtype=torch.float64).contiguous()
    return tuple(t(a) for a in (p.H, p.F, p.c, p.K, p.G, p.o, p.C))


def smooth_problem(p, want_cov: bool = True, device="cuda", fp32: bool = False):
    """Convenience: smooth a generated problem; returns device tensors (u, cov)."""
    args = to_device(p, device)
    plan = Plan(p.k, p.n, p.m, p.K_diag, p.C_diag, device=device, fp32=fp32)
    try:
        if want_cov:
            return plan.smooth_cov(*args)
        return plan.smooth(*args), None
    finally:
        plan.close()


class Batch:
    """Many problems smoothed together (one launch per level step and kernel
    class; see include/ks.h).  ``shapes`` lists (k, n, m, K_diag, C_diag, fp32)."""

    def __init__(self, shapes, device=None, stream=None):
        self.shapes = [tuple(sh) for sh in shapes]
        self.count = len(self.shapes)
        self.device = _device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        descs = (Desc * self.count)(*[make_desc(k, n, m, kd, cd, f32) for (k, n, m, kd, cd, f32) in self.shapes])
        self._descs = descs
        L = lib()
        nbytes = int(L.ks_batch_workspace_bytes(self.count, descs))
        if nbytes == 0:
            raise KsError(KS_E_ARG, "unsupported batch")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.ws_bytes = nbytes
        h = ctypes.c_void_p()
        st = L.ks_batch_create(self.count, descs, ctypes.c_void_p(ptr), nbytes,
                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != KS_OK:
            raise KsError(st, "ks_batch_create")
        self._h = h

    def outputs(self, want_cov=True):
        us = [torch.empty((k + 1, n), dtype=torch.float64, device=self.device) for (k, n, *_r) in self.shapes]
        covs = ([torch.empty((k + 1, n, n), dtype=torch.float64, device=self.device) for (k, n, *_r) in self.shapes]
                if want_cov else [None] * self.count)
        return us, covs

    def smooth(self, inputs, us, covs=None, check=True):
        """inputs[i] = (H, F, c, K, G, o, C) device tensors; writes us[i] (and
        covs[i]); returns the per-problem status list."""
        want_cov = covs is not None and all(c is not None for c in covs)
        io = (Io * self.count)()
        for i, (shape, args) in enumerate(zip(self.shapes, inputs)):
            io[i] = _make_io(shape, args, us[i], covs[i] if want_cov else None, self.device)
        st = (ctypes.c_int * self.count)()
        r = lib().ks_batch_smooth(self._h, io, 1 if want_cov else 0, st)
        statuses = list(st)
        if check and r != KS_OK:
            raise KsError(r, "ks_batch_smooth")
        return statuses

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().ks_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """Continuous batching of requests over one device workspace (see
    include/ks.h): ``submit`` admits a request if its region fits now,
    ``step`` advances every in-flight request by one step of its schedule and
    returns the (ticket, status) pairs of the requests that finished."""

    def __init__(self, ws_bytes: int, device=None, stream=None):
        self.device = _device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(int(ws_bytes) + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        h = ctypes.c_void_p()
        st = lib().ks_engine_create(ctypes.c_void_p(ptr), int(ws_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(h))
        if st != KS_OK:
            raise KsError(st, "ks_engine_create")
        self._h = h
        self._live = {}   # ticket -> tensors the request reads or writes

    @staticmethod
    def footprint(shape) -> int:
        """Device bytes a request of shape (k, n, m, K_diag, C_diag, fp32) holds
        while in flight (0 if unsupported)."""
        d = make_desc(*shape)
        return (int(lib().ks_workspace_bytes(ctypes.byref(d))) + 255) // 256 * 256

    def submit(self, shape, inputs, u, cov=None) -> Optional[int]:
        """Admit a request; returns its ticket, or None when it does not fit
        now (retry after a step).  The tensors are held until it retires."""
        d = make_desc(*shape)
        io = _make_io(shape, inputs, u, cov, self.device)
        t = ctypes.c_uint64()
        st = lib().ks_engine_submit(self._h, ctypes.byref(d), ctypes.byref(io), 0 if cov is None else 1,
                                    ctypes.byref(t))
        if st == KS_E_BUSY:
            return None
        if st != KS_OK:
            raise KsError(st, "ks_engine_submit")
        self._live[t.value] = (inputs, u, cov)
        return t.value

    def _collect(self, fin):
        out = []
        cap = max(int(fin), 1)
        tickets = (ctypes.c_uint64 * cap)()
        statuses = (ctypes.c_int * cap)()
        while True:
            cnt = ctypes.c_int32()
            st = lib().ks_engine_retired(self._h, cap, tickets, statuses, ctypes.byref(cnt))
            if st != KS_OK:
                raise KsError(st, "ks_engine_retired")
            for i in range(cnt.value):
                self._live.pop(tickets[i], None)
                out.append((int(tickets[i]), int(statuses[i])))
            if cnt.value < cap:
                return out

    def step(self):
        """Enqueue one tick (asynchronous) and return the (ticket, status)
        pairs of the requests retired meanwhile."""
        fin = ctypes.c_int32()
        st = lib().ks_engine_step(self._h, ctypes.byref(fin))
        if st != KS_OK:
            raise KsError(st, "ks_engine_step")
        return self._collect(fin.value)

    def wait(self):
        """Block until every enqueued tick has completed; returns the retired
        (ticket, status) pairs."""
        fin = ctypes.c_int32()
        st = lib().ks_engine_wait(self._h, ctypes.byref(fin))
        if st != KS_OK:
            raise KsError(st, "ks_engine_wait")
        return self._collect(fin.value)

    def stats(self) -> dict:
        s = EngineStats()
        st = lib().ks_engine_query(self._h, ctypes.byref(s))
        if st != KS_OK:
            raise KsError(st, "ks_engine_query")
        return {f: getattr(s, f) for f, _t in EngineStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().ks_engine_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
