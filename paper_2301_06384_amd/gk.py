"""Python binding of libgk.so (ctypes, argument marshalling only).

Every computation runs inside the HIP library; this module only converts
numpy arrays / torch tensors to pointers and C structs and back.  Importing
it fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2301_06384_amd.build`")
# PyTorch brings its own HIP runtime; it is loaded before the library so that
# the process sets up the device the same way whatever the caller imports first.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)

# ------------------------------------------------------------------ constants
OK, EINVAL, ENOTSYM, ENOTLAP, EDUPSAMPLE, ERANGE, ENOMEM, ENOTSPD, EDEVICE, EUNSUPPORTED, EAGAIN, ESHUTDOWN = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10, -11)
UNIT_WEIGHTS, ASSUME_PSD, REORDER = 0x1, 0x2, 0x4
IO_DEVICE, FULL_REORTH, PHI_EIG, TIMING, NO_REORTH, TWO_PASS = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
VARIANTS = {"cbl": 0, "gbl": 1, "sbl": 2, "cheb": 3, "cheb2": 4}
PRECISIONS = {"fp64": 0, "mixed": 1}
PHI_KINDS = {"diffusion": 0, "spline": 1, "polynomial": 2}
PHI_METHODS = {0: "eig", 1: "banded", 2: "chebyshev", 3: "horner"}


class GKError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        detail = _lib.gk_last_error_detail().decode()
        super().__init__(f"{where}: {_lib.gk_strerror(code).decode()} ({code}): {detail}")


# -------------------------------------------------------------------- structs
class Phi(C.Structure):
    _fields_ = [("kind", C.c_int32), ("t", C.c_double), ("eps", C.c_double), ("k", C.c_double),
                ("poly", C.POINTER(C.c_double)), ("poly_len", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("t_total_ms", C.c_double), ("t_spmm_ms", C.c_double), ("t_orth_ms", C.c_double),
                ("t_reorth_ms", C.c_double), ("t_phi_ms", C.c_double), ("t_asm_ms", C.c_double),
                ("t_fit_ms", C.c_double), ("spmm_launches", C.c_double), ("bytes_spmm", C.c_double),
                ("resid_norm", C.c_double), ("orth_est", C.c_double), ("n_reorth", C.c_int32),
                ("n_deflated", C.c_int32), ("phi_method", C.c_int32), ("n_qr2_series", C.c_int32),
                ("n_qr2_skipped", C.c_int32),
                ("footprint_bytes", C.c_uint64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}
        d["phi_method"] = PHI_METHODS.get(self.phi_method, self.phi_method)
        return d


class Request(C.Structure):
    _fields_ = [("graph", C.c_void_p), ("samples", C.POINTER(C.c_int64)), ("s", C.c_int32),
                ("y", C.POINTER(C.c_double)), ("phi", Phi), ("m", C.c_int32), ("variant", C.c_int32),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("gamma", C.c_double),
                ("coef_out", C.POINTER(C.c_double)), ("pred_out", C.POINTER(C.c_double))]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("t_submit_ms", C.c_double),
                ("t_start_ms", C.c_double), ("t_complete_ms", C.c_double), ("stats", Stats)]


_P = C.c_void_p
_lib.graph_kernel_init.argtypes = [C.c_int64, _P, _P, _P, C.c_uint32, C.POINTER(C.c_void_p)]
_lib.graph_kernel_init.restype = C.c_int
_lib.graph_kernel_release.argtypes = [C.c_void_p]
_lib.graph_kernel_release.restype = None
_lib.gk_graph_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_double)]
_lib.krylov_kernel_columns.argtypes = [C.c_void_p, _P, C.c_int32, C.POINTER(Phi), C.c_int32, C.c_int32,
                                       C.c_int32, C.c_uint32, _P, _P, C.POINTER(Stats)]
_lib.krylov_kernel_columns.restype = C.c_int
_lib.krylov_kernel_columns_noalloc.argtypes = _lib.krylov_kernel_columns.argtypes
_lib.krylov_kernel_columns_noalloc.restype = C.c_int
_lib.kernel_machine_fit_predict.argtypes = [C.c_void_p, _P, C.c_int32, _P, C.POINTER(Phi), C.c_int32,
                                            C.c_int32, C.c_int32, C.c_uint32, C.c_double, _P, _P,
                                            C.POINTER(Stats)]
_lib.kernel_machine_fit_predict.restype = C.c_int
_lib.gk_request_footprint.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32,
                                      C.POINTER(C.c_uint64)]
_lib.gk_serve_start.argtypes = [C.c_int32, C.c_uint64, C.c_int32]
_lib.gk_submit.argtypes = [C.POINTER(Request), C.POINTER(C.c_uint64)]
_lib.gk_poll.argtypes = [C.c_uint64, C.c_int64, C.POINTER(Result)]
_lib.gk_serve_stop.argtypes = []
_lib.gk_strerror.argtypes = [C.c_int]
_lib.gk_strerror.restype = C.c_char_p
_lib.gk_last_error_detail.restype = C.c_char_p
_lib.gk_set_stream.argtypes = [C.c_void_p]
_lib.gk_trim.argtypes = [C.POINTER(C.c_uint64)]
_lib.gk_version.restype = C.c_char_p
_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_lib.gk_set_allocator.argtypes = [_ALLOC_T, _FREE_T, C.c_void_p]

class KernelTiming(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double),
                ("alg_bytes", C.c_double), ("alg_flops", C.c_double)]


_lib.gk_kernel_timings.argtypes = [C.POINTER(KernelTiming), C.c_int32, C.POINTER(C.c_int32)]
_lib.gk_kernel_timings.restype = C.c_int

EXPORTED = ["graph_kernel_init", "graph_kernel_release", "gk_graph_info", "krylov_kernel_columns",
            "krylov_kernel_columns_noalloc", "kernel_machine_fit_predict", "gk_request_footprint", "gk_serve_start", "gk_submit", "gk_poll",
            "gk_serve_stop", "gk_strerror", "gk_last_error_detail", "gk_set_allocator", "gk_set_stream", "gk_trim",
            "gk_version", "gk_kernel_timings"]


def kernel_timings() -> list:
    """Per-kernel-class device times of this thread's last call made with TIMING."""
    cnt = C.c_int32(0)
    _check(_lib.gk_kernel_timings(None, 0, C.byref(cnt)), "gk_kernel_timings")
    arr = (KernelTiming * max(cnt.value, 1))()
    _check(_lib.gk_kernel_timings(arr, cnt.value, C.byref(cnt)), "gk_kernel_timings")
    return [dict(name=r.name.decode(), launches=int(r.launches), total_ms=float(r.total_ms),
                 alg_bytes=float(r.alg_bytes), alg_flops=float(r.alg_flops)) for r in arr[:cnt.value]]


def _check(rc: int, where: str):
    if rc != OK:
        raise GKError(rc, where)


def _ptr(a):
    """Pointer of a numpy array or a torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()   # torch tensor


def make_phi(spec: dict):
    """Phi struct from a spec dict; returns (struct, keepalive)."""
    kind = PHI_KINDS[spec["kind"]]
    coef = None
    p = Phi(kind, float(spec.get("t", 0.0)), float(spec.get("eps", 0.0)), float(spec.get("k", 0.0)), None, 0)
    if spec["kind"] == "polynomial":
        coef = np.ascontiguousarray(spec["coef"], dtype=np.float64)
        p.poly = coef.ctypes.data_as(C.POINTER(C.c_double))
        p.poly_len = coef.size
    return p, coef


def version() -> str:
    return _lib.gk_version().decode()


# ---------------------------------------------------------------------- graph
class Graph:
    """Device-resident Laplacian (graph_kernel_init / graph_kernel_release)."""

    def __init__(self, n, row_ptr, col_idx, vals=None, flags: int = 0):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        vv = None if vals is None else np.ascontiguousarray(vals, dtype=np.float64)
        h = C.c_void_p()
        rc = _lib.graph_kernel_init(int(n), _ptr(rp), _ptr(ci), _ptr(vv), flags, C.byref(h))
        _check(rc, "graph_kernel_init")
        self._h = h
        self.n = int(n)

    @classmethod
    def from_laplacian(cls, L, flags: int = 0):
        """From an inputs.CSRLaplacian (or any object with n/row_ptr/col_idx/vals)."""
        return cls(L.n, L.row_ptr, L.col_idx, L.vals, flags)

    @property
    def handle(self):
        return self._h

    def info(self):
        n, nnz, lam = C.c_int64(), C.c_int64(), C.c_double()
        _check(_lib.gk_graph_info(self._h, C.byref(n), C.byref(nnz), C.byref(lam)), "gk_graph_info")
        return dict(n=n.value, nnz_offdiag=nnz.value, lambda_max=lam.value)

    def release(self):
        if getattr(self, "_h", None):
            _lib.graph_kernel_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


# -------------------------------------------------------------------- compute
def krylov_kernel_columns(graph: Graph, samples, phi: dict, m: int, variant: str = "cbl",
                          precision: str = "fp64", flags: int = 0, want_cols: bool = True,
                          want_kww: bool = True, out_cols=None, out_kww=None):
    """Kernel columns P ~ phi(L) E_W (n x s) and K_W (s x s); returns (P, K, stats).

    Host mode: samples is array-like; returns numpy arrays.  With IO_DEVICE in
    flags, samples / out_cols / out_kww must be device tensors (out arrays
    provided by the caller, column-major n x s, i.e. a (s, n) C-contiguous
    tensor) and the call returns after enqueueing.
    """
    st = Stats()
    p, keep = make_phi(phi)
    if flags & IO_DEVICE:
        s = int(samples.numel())
        rc = _lib.krylov_kernel_columns(graph.handle, _ptr(samples), s, C.byref(p), m, VARIANTS[variant],
                                        PRECISIONS[precision], flags, _ptr(out_cols), _ptr(out_kww), C.byref(st))
        _check(rc, "krylov_kernel_columns")
        return out_cols, out_kww, st
    smp = np.ascontiguousarray(samples, dtype=np.int64)
    s = smp.size
    if out_cols is not None or out_kww is not None:
        # caller-provided host buffers ((s, n) and (s, s), C-contiguous; e.g.
        # pinned torch CPU tensors), filled in place
        rc = _lib.krylov_kernel_columns(graph.handle, _ptr(smp), s, C.byref(p), m, VARIANTS[variant],
                                        PRECISIONS[precision], flags, _ptr(out_cols), _ptr(out_kww), C.byref(st))
        _check(rc, "krylov_kernel_columns")
        return out_cols, out_kww, st
    cols = np.empty((s, graph.n), dtype=np.float64) if want_cols else None   # column-major n x s
    kww = np.empty((s, s), dtype=np.float64) if want_kww else None
    rc = _lib.krylov_kernel_columns(graph.handle, _ptr(smp), s, C.byref(p), m, VARIANTS[variant],
                                    PRECISIONS[precision], flags, _ptr(cols), _ptr(kww), C.byref(st))
    _check(rc, "krylov_kernel_columns")
    del keep
    return (None if cols is None else cols.T), (None if kww is None else kww.T), st


def krylov_kernel_columns_noalloc(graph: Graph, samples, phi: dict, m: int, variant: str, precision: str,
                                  out_cols, out_kww, flags: int = 0):
    """krylov_kernel_columns on the library's static device scratch (no device
    allocation).  samples, out_cols ((s, n) tensor, i.e. column-major n x s) and
    out_kww are device tensors; returns (out_cols, out_kww, stats)."""
    st = Stats()
    p, keep = make_phi(phi)
    s = int(samples.numel())
    rc = _lib.krylov_kernel_columns_noalloc(graph.handle, _ptr(samples), s, C.byref(p), m, VARIANTS[variant],
                                            PRECISIONS[precision], flags | IO_DEVICE, _ptr(out_cols),
                                            _ptr(out_kww), C.byref(st))
    _check(rc, "krylov_kernel_columns_noalloc")
    del keep
    return out_cols, out_kww, st


STATIC_SCRATCH_BYTES = 128 << 20


def kernel_machine_fit_predict(graph: Graph, samples, y, phi: dict, m: int, gamma: float,
                               variant: str = "cbl", precision: str = "fp64", flags: int = 0,
                               want_pred: bool = True):
    """(coefficients c, predictions on all n nodes, stats)."""
    st = Stats()
    p, keep = make_phi(phi)
    smp = np.ascontiguousarray(samples, dtype=np.int64)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    s = smp.size
    coef = np.empty(s)
    pred = np.empty(graph.n) if want_pred else None
    rc = _lib.kernel_machine_fit_predict(graph.handle, _ptr(smp), s, _ptr(yy), C.byref(p), m,
                                         VARIANTS[variant], PRECISIONS[precision], flags, float(gamma),
                                         _ptr(coef), _ptr(pred), C.byref(st))
    _check(rc, "kernel_machine_fit_predict")
    del keep
    return coef, pred, st


def request_footprint(n: int, s: int, m: int, variant: str = "cbl", precision: str = "mixed",
                      flags: int = 0) -> int:
    b = C.c_uint64()
    _check(_lib.gk_request_footprint(n, s, m, VARIANTS[variant], PRECISIONS[precision], flags, C.byref(b)),
           "gk_request_footprint")
    return b.value


def strerror(code: int) -> str:
    return _lib.gk_strerror(code).decode()


def trim() -> int:
    """Return the library's cached free device blocks to HIP; bytes released."""
    b = C.c_uint64()
    _check(_lib.gk_trim(C.byref(b)), "gk_trim")
    return b.value


def set_stream(stream) -> None:
    """Use a HIP stream (torch.cuda.Stream or raw handle) for the calling thread."""
    h = getattr(stream, "cuda_stream", stream)
    _check(_lib.gk_set_stream(C.c_void_p(h)), "gk_set_stream")


_alloc_keep = []


def use_torch_allocator() -> None:
    """Route the library's device allocations through torch's caching allocator."""
    import torch

    def _alloc(nbytes, ctx):
        dev = torch.cuda.current_device()
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, torch.cuda.current_stream(dev))

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = _ALLOC_T(_alloc), _FREE_T(_free)
    _alloc_keep[:] = [fa, ff]
    _check(_lib.gk_set_allocator(fa, ff, None), "gk_set_allocator")


def reset_allocator() -> None:
    """Back to the library's own device cache (gk_set_allocator(NULL, NULL))."""
    _check(_lib.gk_set_allocator(_ALLOC_T(), _FREE_T(), None), "gk_set_allocator")
    _alloc_keep[:] = []


# -------------------------------------------------------------------- serving
class Server:
    """Continuous-batching serving loop (gk_serve_start / gk_submit / gk_poll)."""

    def __init__(self, max_active: int = 8, hbm_budget: int = 0, n_streams: int = 4):
        _check(_lib.gk_serve_start(max_active, hbm_budget, n_streams), "gk_serve_start")
        self._keep = {}

    def submit(self, graph: Graph, samples, y, phi: dict, m: int, gamma: float, variant="cbl",
               precision="mixed", flags: int = 0, want_pred: bool = True) -> int:
        smp = np.ascontiguousarray(samples, dtype=np.int64)
        yy = np.ascontiguousarray(y, dtype=np.float64)
        p, pk = make_phi(phi)
        coef = np.empty(smp.size)
        pred = np.empty(graph.n) if want_pred else None
        r = Request(graph.handle, smp.ctypes.data_as(C.POINTER(C.c_int64)), smp.size,
                    yy.ctypes.data_as(C.POINTER(C.c_double)), p, m, VARIANTS[variant], PRECISIONS[precision],
                    flags, float(gamma), coef.ctypes.data_as(C.POINTER(C.c_double)),
                    None if pred is None else pred.ctypes.data_as(C.POINTER(C.c_double)))
        t = C.c_uint64()
        _check(_lib.gk_submit(C.byref(r), C.byref(t)), "gk_submit")
        self._keep[t.value] = (coef, pred, smp, yy, pk)
        return t.value

    def poll(self, ticket: int, timeout_us: int = -1):
        """Returns None if not done, else dict(status, coef, pred, times, stats)."""
        res = Result()
        rc = _lib.gk_poll(ticket, timeout_us, C.byref(res))
        if rc == EAGAIN:
            return None
        _check(rc, "gk_poll")
        coef, pred, *_ = self._keep.pop(ticket)
        return dict(status=res.status, coef=coef, pred=pred, t_submit_ms=res.t_submit_ms,
                    t_start_ms=res.t_start_ms, t_complete_ms=res.t_complete_ms, stats=res.stats.as_dict())

    def stop(self):
        _check(_lib.gk_serve_stop(), "gk_serve_stop")
