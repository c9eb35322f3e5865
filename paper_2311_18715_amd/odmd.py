"""Python binding of the C ABI in include/odmd.h (argument marshalling only).

Every computation runs in the HIP kernels of ``libodmd.so``; this module
only converts torch tensors to device pointers and host arrays to ctypes
buffers.  If the library is not built, importing the binding's functions
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libodmd.so")
RMAX = 64

F64, F32, BF16 = 0, 1, 2
STATUS = {
    0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EEMPTY", 4: "ENONFINITE",
    5: "ENOCONV", 6: "ESEQ", 7: "EDEVICE",
}
EXPORTS = [
    "odmd_create", "odmd_create_ex", "odmd_state_bytes", "odmd_update", "odmd_update_batch",
    "odmd_eigs", "odmd_predict", "odmd_predict_batch", "odmd_sync", "odmd_destroy", "odmd_release",
    "odmd_status_str",
    "odmd_get_info", "odmd_get_state", "odmd_get_basis", "odmd_profile", "odmd_profile_read",
    "odmd_profile_samples", "odmd_profile_latency", "odmd_create_general", "odmd_state_bytes_general",
    "odmd_default_shape", "odmd_create_shaped", "odmd_state_bytes_shaped", "odmd_autotune",
    "odmd_plan_create", "odmd_plan_launch", "odmd_plan_destroy", "odmd_update_batch_noalloc",
    "odmd_peek_status",
]


def status_name(code: int) -> str:
    """Name of an odmd_status code ("ESEQ", ...)."""
    return STATUS.get(int(code), str(code))


class OdmdError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        self.name = STATUS.get(code, str(code))
        super().__init__(f"{where}: {self.name} ({lib().odmd_status_str(code).decode()})")


class Info(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_int32), ("r_max", ctypes.c_int32), ("n", ctypes.c_int64),
        ("m", ctypes.c_int64), ("tol_eff", ctypes.c_double), ("last_rho", ctypes.c_double),
        ("last_sweeps", ctypes.c_int32), ("nblocks", ctypes.c_int32),
        ("threads", ctypes.c_int32), ("stored", ctypes.c_int32), ("capacity", ctypes.c_int32),
    ]


_LIB = None


def lib() -> ctypes.CDLL:
    """Load libodmd.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2311_18715_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        pd = ctypes.POINTER(ctypes.c_double)
        sig = {
            "odmd_create": ([i64, i32, dbl, ctypes.POINTER(vp)], ctypes.c_int),
            "odmd_create_ex": ([i64, i32, dbl, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_size_t,
                                ctypes.POINTER(vp)], ctypes.c_int),
            "odmd_state_bytes": ([i64, i32, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
            "odmd_create_general": ([i64, i32, dbl, ctypes.c_int, ctypes.c_int, vp, vp,
                                     ctypes.c_size_t, ctypes.POINTER(vp)], ctypes.c_int),
            "odmd_state_bytes_general": ([i64, i32, ctypes.c_int, ctypes.c_int], ctypes.c_size_t),
            "odmd_default_shape": ([i64, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)], ctypes.c_int),
            "odmd_create_shaped": ([i64, i32, dbl, ctypes.c_int, ctypes.c_int, vp, i32, i32, i32,
                                    i32, vp, ctypes.c_size_t, ctypes.POINTER(vp)], ctypes.c_int),
            "odmd_state_bytes_shaped": ([i64, i32, ctypes.c_int, ctypes.c_int, i32, i32, i32, i32],
                                        ctypes.c_size_t),
            "odmd_plan_create": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32,
                                  ctypes.POINTER(vp)], ctypes.c_int),
            "odmd_plan_launch": ([vp], ctypes.c_int),
            "odmd_plan_destroy": ([vp], ctypes.c_int),
            "odmd_autotune": ([i64, i32, ctypes.c_int, ctypes.c_int, i32, vp, ctypes.POINTER(i32),
                               ctypes.POINTER(i32), ctypes.POINTER(i32), pd, pd], ctypes.c_int),
            "odmd_update": ([vp, vp, vp], ctypes.c_int),
            "odmd_update_batch": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i32],
                                  ctypes.c_int),
            "odmd_update_batch_noalloc": ([ctypes.POINTER(vp), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), i32], ctypes.c_int),
            "odmd_eigs": ([vp, i32, ctypes.POINTER(i32), pd, pd, pd, pd], ctypes.c_int),
            "odmd_predict": ([vp, i32, vp], ctypes.c_int),
            "odmd_predict_batch": ([ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(vp), i32],
                                   ctypes.c_int),
            "odmd_sync": ([vp], ctypes.c_int),
            "odmd_peek_status": ([vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "odmd_destroy": ([vp], ctypes.c_int),
            "odmd_release": ([vp], ctypes.c_int),
            "odmd_status_str": ([ctypes.c_int], ctypes.c_char_p),
            "odmd_get_info": ([vp, ctypes.POINTER(Info)], ctypes.c_int),
            "odmd_get_state": ([vp, i32, pd, pd, pd, pd, pd], ctypes.c_int),
            "odmd_get_basis": ([vp, vp], ctypes.c_int),
            "odmd_profile": ([vp, i32], ctypes.c_int),
            "odmd_profile_read": ([vp, pd, pd, ctypes.POINTER(i64)], ctypes.c_int),
            "odmd_profile_samples": ([vp, i64, pd, pd, pd, ctypes.POINTER(i64)], ctypes.c_int),
            "odmd_profile_latency": ([vp, i32], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def _check(code: int, where: str) -> None:
    if code != 0:
        raise OdmdError(code, where)


def _dptr(t) -> ctypes.c_void_p:
    """Device pointer of a contiguous CUDA (HIP) tensor."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _dbl(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class ODMD:
    """One online-DMD stream on the GPU (a handle of the C library).

    Parameters mirror ``odmd_create_ex``: state size n, rank cap r_max,
    relative tolerance tol, basis storage ('f64' | 'f32' | 'bf16'),
    snapshot type (defaults to the basis type, FP32 for BF16), torch stream
    (defaults to the current one) and an optional caller-owned uint8 device
    workspace.  pairs='general' creates a handle for pairs that need not
    chain (``odmd_create_general``).  shape=(threads, rows_per_block,
    max_blocks) sets the streaming pass's launch shape
    (``odmd_create_shaped``; None keeps the library's default rule);
    shape='latency' or 'throughput' takes the tuned shape of the shipped
    table for that objective (``autotune.lookup``), the default where the
    table has none.
    """

    def __init__(self, n: int, r_max: int, tol: float, basis: str = "f64", io: str | None = None,
                 stream=None, workspace=None, pairs: str = "chained", shape=None):
        import torch
        self._torch = torch
        io = io or ("f32" if basis == "bf16" else basis)     # a BF16 basis takes FP32 snapshots
        bt = {"f64": F64, "f32": F32, "bf16": BF16}[basis]
        it = {"f64": F64, "f32": F32}[io]
        self.n, self.r_max, self.basis, self.io = int(n), int(r_max), basis, io
        self.dtype = torch.float64 if self.io == "f64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        ws, wsb = None, 0
        if workspace is not None:
            ws, wsb = _dptr(workspace), workspace.numel() * workspace.element_size()
        if pairs not in ("chained", "general"):
            raise ValueError("pairs must be 'chained' or 'general'")
        self.pairs = pairs
        if isinstance(shape, str):
            from . import autotune
            shape = autotune.lookup(self.n, self.r_max, basis, io, objective=shape)
        self.shape = shape
        if shape is not None:
            t, rpb, cap = (int(v) for v in shape)
            _check(lib().odmd_create_shaped(self.n, self.r_max, float(tol), bt, it,
                                            ctypes.c_void_p(stream.cuda_stream), t, rpb, cap,
                                            int(pairs == "general"), ws, wsb, ctypes.byref(h)),
                   "odmd_create_shaped")
        else:
            name = "odmd_create_ex" if pairs == "chained" else "odmd_create_general"
            _check(getattr(lib(), name)(self.n, self.r_max, float(tol), bt, it,
                                        ctypes.c_void_p(stream.cuda_stream), ws, wsb,
                                        ctypes.byref(h)), name)
        self._h = h
        self._workspace = workspace

    @staticmethod
    def state_bytes(n: int, r_max: int, basis: str = "f64", io: str | None = None,
                    pairs: str = "chained", shape=None) -> int:
        io = io or ("f32" if basis == "bf16" else basis)
        bt = {"f64": F64, "f32": F32, "bf16": BF16}[basis]
        it = {"f64": F64, "f32": F32}[io]
        if shape is not None:
            t, rpb, cap = (int(v) for v in shape)
            return int(lib().odmd_state_bytes_shaped(int(n), int(r_max), bt, it, t, rpb, cap,
                                                     int(pairs == "general")))
        fn = lib().odmd_state_bytes if pairs == "chained" else lib().odmd_state_bytes_general
        return int(fn(int(n), int(r_max), bt, it))

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def update(self, x, y) -> None:
        _check(lib().odmd_update(self._h, _dptr(x), _dptr(y)), "odmd_update")

    def sync(self) -> None:
        _check(lib().odmd_sync(self._h), "odmd_sync")

    def peek_status(self) -> int:
        """The status code latched by finished device work (0: none), read
        without a device call and without clearing it (odmd_peek_status)."""
        v = ctypes.c_int()
        _check(lib().odmd_peek_status(self._h, ctypes.byref(v)), "odmd_peek_status")
        return v.value

    def eigs(self, vectors: bool = True):
        """(lam, V): complex eigenvalues (r,) and eigenvectors (r, r) of A~."""
        r = ctypes.c_int32()
        lr, li = np.zeros(RMAX), np.zeros(RMAX)
        vr = np.zeros(RMAX * RMAX) if vectors else None
        vi = np.zeros(RMAX * RMAX) if vectors else None
        _check(lib().odmd_eigs(self._h, RMAX, ctypes.byref(r), _dbl(lr), _dbl(li),
                               _dbl(vr) if vectors else None, _dbl(vi) if vectors else None),
               "odmd_eigs")
        k = r.value
        lam = lr[:k] + 1j * li[:k]
        if not vectors:
            return lam, None
        V = (vr[:k * k] + 1j * vi[:k * k]).reshape(k, k).T     # column j = vector j
        return lam, V

    def predict(self, steps: int, out=None):
        """Predicted states a+1..a+steps as a (steps, n) device tensor."""
        if out is None:
            out = self._torch.empty((steps, self.n), dtype=self.dtype, device="cuda")
        _check(lib().odmd_predict(self._h, int(steps), _dptr(out)), "odmd_predict")
        return out

    def info(self) -> Info:
        i = Info()
        _check(lib().odmd_get_info(self._h, ctypes.byref(i)), "odmd_get_info")
        return i

    def state(self) -> dict:
        """Small FP64 state copied to the host: sigma, atilde, p_y, C, w."""
        k = self.info().r
        s, a, p = np.zeros(RMAX), np.zeros(RMAX * RMAX), np.zeros(RMAX)
        c, w = np.zeros(RMAX * RMAX), np.zeros(RMAX)
        _check(lib().odmd_get_state(self._h, RMAX, _dbl(s), _dbl(a), _dbl(p), _dbl(c), _dbl(w)),
               "odmd_get_state")
        return {
            "r": k, "sigma": s[:k].copy(), "p_y": p[:k].copy(), "w": w[:k].copy(),
            "atilde": a[:k * k].reshape(k, k).T.copy(), "C": c[:k * k].reshape(k, k).T.copy(),
        }

    def basis_matrix(self):
        """The current basis U as an (n, r) FP64 device tensor."""
        out = self._torch.empty((self.r_max, self.n), dtype=self._torch.float64, device="cuda")
        _check(lib().odmd_get_basis(self._h, _dptr(out)), "odmd_get_basis")
        k = self.info().r
        return out[:k].T

    def profile(self, capacity: int) -> None:
        """Record per-update events (capacity > 0 reserves them now); 0 stops."""
        _check(lib().odmd_profile(self._h, int(capacity)), "odmd_profile")

    def profile_latency(self, on: bool) -> None:
        """While on, timed updates record only the pass start and the core
        end (their kernel samples read as NaN; update_ms is their latency)."""
        _check(lib().odmd_profile_latency(self._h, 1 if on else 0), "odmd_profile_latency")

    def profile_read(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().odmd_profile_read(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "odmd_profile_read")
        return a.value, b.value, c.value

    def profile_samples(self, cap: int = 1 << 16):
        """Per-update (pass_ms, core_ms, update_ms) arrays of the timed
        updates: kernel durations of the pass and the core, and pass start
        to core end."""
        a, b, u, c = np.zeros(cap), np.zeros(cap), np.zeros(cap), ctypes.c_int64()
        _check(lib().odmd_profile_samples(self._h, cap, _dbl(a), _dbl(b), _dbl(u), ctypes.byref(c)),
               "odmd_profile_samples")
        k = min(cap, c.value)
        return a[:k].copy(), b[:k].copy(), u[:k].copy()

    def close(self, wait: bool = True) -> None:
        """Free the handle: after its stream's work (odmd_destroy), or, with
        wait=False, at once (odmd_release; a caller-owned workspace must then
        outlive the queued work, as torch's allocator on the handle's stream
        ensures)."""
        if getattr(self, "_h", None):
            name = "odmd_destroy" if wait else "odmd_release"
            code = getattr(lib(), name)(self._h)
            if code != 1:            # EINVAL: a live plan holds the handle, which stays valid
                self._h = None
            _check(code, name)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def update_batch(models, xs, ys) -> None:
    """One batched update of several streams (odmd_update_batch: one pass
    launch per group of equal launch shape, storage type and live-column
    bucket, then one small-state launch for all)."""
    n = len(models)
    H = (ctypes.c_void_p * n)(*[m.handle for m in models])
    X = (ctypes.c_void_p * n)(*[_dptr(x) for x in xs])
    Y = (ctypes.c_void_p * n)(*[_dptr(y) for y in ys])
    _check(lib().odmd_update_batch(H, X, Y, n), "odmd_update_batch")


# most streams of one odmd_update_batch_noalloc call (ODMD_NOALLOC_MAX_STREAMS)
NOALLOC_MAX_STREAMS = 1024


def update_batch_noalloc(models, xs, ys) -> None:
    """odmd_update_batch_noalloc: the batched update of several streams with
    no allocation (descriptor tables in the library's fixed device array);
    results equal update_batch's bit for bit."""
    n = len(models)
    H = (ctypes.c_void_p * n)(*[m.handle for m in models])
    X = (ctypes.c_void_p * n)(*[_dptr(x) for x in xs])
    Y = (ctypes.c_void_p * n)(*[_dptr(y) for y in ys])
    _check(lib().odmd_update_batch_noalloc(H, X, Y, n), "odmd_update_batch_noalloc")


class Plan:
    """A fixed batched step (``odmd_plan_create``): the handles of ``models``
    with the fixed snapshot buffers xs, ys (device tensors the caller
    refills between launches).  ``launch()`` enqueues one step on the
    handles' stream; capturing ``launch()`` in a torch.cuda.CUDAGraph on
    that stream gives a graph that replays the step."""

    def __init__(self, models, xs, ys):
        n = len(models)
        H = (ctypes.c_void_p * n)(*[m.handle for m in models])
        X = (ctypes.c_void_p * n)(*[_dptr(x) for x in xs])
        Y = (ctypes.c_void_p * n)(*[_dptr(y) for y in ys])
        p = ctypes.c_void_p()
        _check(lib().odmd_plan_create(H, X, Y, n, ctypes.byref(p)), "odmd_plan_create")
        self._p = p
        self._keep = (list(models), list(xs), list(ys))    # the plan points into these

    def launch(self) -> None:
        _check(lib().odmd_plan_launch(self._p), "odmd_plan_launch")

    def close(self) -> None:
        if self._p is not None and self._p.value:
            _check(lib().odmd_plan_destroy(self._p), "odmd_plan_destroy")
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def predict_batch(models, steps, outs=None):
    """odmd_predict_batch: predicted states of several streams, the
    coefficients of every stream's first chunk of states in one launch.
    Returns one (steps_i, n_i) device tensor per model: outs (contiguous
    tensors of those shapes and the models' output types) or new ones."""
    import torch
    n = len(models)
    steps = [int(s) for s in steps]
    if outs is None:
        outs = [torch.empty((s, m.n), dtype=m.dtype, device="cuda") for m, s in zip(models, steps)]
    else:
        outs = list(outs)
        if len(outs) != n or any(tuple(o.shape) != (s, m.n) or o.dtype != m.dtype or not o.is_contiguous()
                                 for o, m, s in zip(outs, models, steps)):
            raise ValueError("predict_batch: outs must match the models' shapes and types")
    H = (ctypes.c_void_p * n)(*[m.handle for m in models])
    S = (ctypes.c_int32 * n)(*steps)
    O = (ctypes.c_void_p * n)(*[_dptr(o) for o in outs])
    _check(lib().odmd_predict_batch(H, S, O, n), "odmd_predict_batch")
    return outs


def handle_array(models) -> np.ndarray:
    """The models' handles as a uint64 array, for update_batch_ptrs."""
    return np.array([m.handle.value for m in models], dtype=np.uint64)


def update_batch_ptrs(handles: np.ndarray, xptrs: np.ndarray, yptrs: np.ndarray) -> None:
    """odmd_update_batch on pre-built uint64 arrays of handles and device
    pointers (no per-stream Python objects: for loops over many streams).
    The caller keeps the memory behind the pointers alive and correctly
    typed (n elements of each stream's snapshot type)."""
    count = len(handles)
    if len(xptrs) != count or len(yptrs) != count:
        raise ValueError("handles, xptrs and yptrs must have the same length")
    h = np.ascontiguousarray(handles, dtype=np.uint64)
    x = np.ascontiguousarray(xptrs, dtype=np.uint64)
    y = np.ascontiguousarray(yptrs, dtype=np.uint64)
    vpp = ctypes.POINTER(ctypes.c_void_p)
    _check(lib().odmd_update_batch(h.ctypes.data_as(vpp), x.ctypes.data_as(vpp),
                                   y.ctypes.data_as(vpp), count), "odmd_update_batch")


def default_shape(n: int) -> tuple[int, int, int]:
    """The library's default pass launch shape for n (``odmd_default_shape``)."""
    t, r, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().odmd_default_shape(int(n), ctypes.byref(t), ctypes.byref(r), ctypes.byref(c)),
           "odmd_default_shape")
    return t.value, r.value, c.value


def autotune(n: int, r_max: int, basis: str = "f64", io: str | None = None, streams: int = 1,
             stream=None):
    """Time the candidate pass launch shapes (``odmd_autotune``).

    Returns ((threads, rows_per_block, max_blocks), us_best, us_default).
    """
    import torch
    io = io or ("f32" if basis == "bf16" else basis)
    bt = {"f64": F64, "f32": F32, "bf16": BF16}[basis]
    it = {"f64": F64, "f32": F32}[io]
    if stream is None:
        stream = torch.cuda.current_stream()
    t, r, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    best, dflt = ctypes.c_double(), ctypes.c_double()
    _check(lib().odmd_autotune(int(n), int(r_max), bt, it, int(streams),
                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(t), ctypes.byref(r),
                               ctypes.byref(c), ctypes.byref(best), ctypes.byref(dflt)),
           "odmd_autotune")
    return (t.value, r.value, c.value), best.value, dflt.value
