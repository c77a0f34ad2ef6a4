"""Python binding of the lcemd C-ABI (include/lcemd.h): argument marshalling
only.  Every step of the computation runs in the HIP library; there is no
fallback.  numpy arrays go through the host-pointer path; torch tensors on
the GPU go through the device-pointer path on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblcemd.so")

OK = 0
E_INVALID_ARG, E_BAD_CSR, E_NOT_LOADED, E_OOM, E_HIP, E_UNSUPPORTED, E_CAPACITY, E_NO_DEVICE = (
    -1, -2, -3, -4, -5, -6, -7, -8)
RWMD, OMR, ACT, ICT = 0, 1, 2, 3
D2Q, Q2D, SYM = 0, 1, 2
FP32, BF16, FP8 = 0, 1, 2
PTR_DEVICE, NORMALIZE, L2_NORMALIZE, MAKE_BF16, MAKE_FP8 = 0x1, 0x2, 0x4, 0x8, 0x10
MAX_HIST, MAX_L, MAX_K = 1024, 1024, 512
SERVE_MAX_HIST = 512

METHOD = {"rwmd": RWMD, "omr": OMR, "act": ACT, "ict": ICT}
DIRECTION = {"d2q": D2Q, "q2d": Q2D, "sym": SYM}
PRECISION = {"fp32": FP32, "bf16": BF16, "fp8": FP8}


class LcemdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lcemd error {code}: {msg}")
        self.code = code


class lcemd_query(C.Structure):
    _fields_ = [("rowptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("B", C.c_int64), ("flags", C.c_uint32)]


class lcemd_opts(C.Structure):
    _fields_ = [("method", C.c_int32), ("k", C.c_int32), ("direction", C.c_int32),
                ("precision", C.c_int32), ("exclude_self", C.c_int32),
                ("reserved", C.c_int32 * 3)]


class lcemd_phase_time(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("ms", C.c_double), ("launches", C.c_int64),
                ("work", C.c_double)]


class lcemd_server_cfg(C.Structure):
    _fields_ = [("method", C.c_int32), ("k", C.c_int32), ("precision", C.c_int32),
                ("l", C.c_int32), ("max_slots", C.c_int32), ("max_batch_words", C.c_int32),
                ("memory_budget", C.c_int64), ("use_graph", C.c_int32), ("lanes", C.c_int32),
                ("reserved", C.c_int32 * 4)]


# every symbol the header declares, with its ctypes signature
_SIGS = {
    "lcemd_version": (C.c_int, []),
    "lcemd_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "lcemd_destroy": (None, [C.c_void_p]),
    "lcemd_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lcemd_use_own_stream": (C.c_int, [C.c_void_p]),
    "lcemd_last_error": (C.c_char_p, [C.c_void_p]),
    "lcemd_load_embeddings": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_uint32]),
    "lcemd_load_database": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.c_uint32]),
    "lcemd_distances": (C.c_int, [C.c_void_p, C.POINTER(lcemd_query), C.POINTER(lcemd_opts),
                                  C.c_void_p]),
    "lcemd_topl": (C.c_int, [C.c_void_p, C.POINTER(lcemd_query), C.POINTER(lcemd_opts), C.c_int32,
                             C.c_void_p, C.c_void_p]),
    "lcemd_tables": (C.c_int, [C.c_void_p, C.POINTER(lcemd_query), C.POINTER(lcemd_opts),
                               C.c_void_p, C.c_void_p, C.c_void_p]),
    "lcemd_topl_noalloc": (C.c_int, [C.c_void_p, C.POINTER(lcemd_query), C.POINTER(lcemd_opts), C.c_int32,
                                     C.c_void_p, C.c_void_p]),
    "lcemd_selfjoin_topl": (C.c_int, [C.c_void_p, C.POINTER(lcemd_opts), C.c_int32, C.c_uint32,
                                      C.c_void_p, C.c_void_p]),
    "lcemd_used_vocab": (C.c_int64, [C.c_void_p, C.c_void_p]),
    "lcemd_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "lcemd_counters": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "lcemd_profile_get": (C.c_int, [C.c_void_p, C.POINTER(lcemd_phase_time), C.c_int]),
    "lcemd_server_start": (C.c_int, [C.c_void_p, C.POINTER(lcemd_server_cfg),
                                     C.POINTER(C.c_void_p)]),
    "lcemd_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                      C.POINTER(C.c_uint64)]),
    "lcemd_server_wait": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_double)]),
    "lcemd_server_stop": (None, [C.c_void_p]),
    "lcemd_check_histograms": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                         C.c_int, C.c_char_p, C.c_size_t]),
    "lcemd_serve_sim": (C.c_int, [C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int64, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblcemd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1812_02091_amd.build`")
    # One HIP runtime per process: torch bundles a runtime with the same
    # soname as the system one the library links, and whichever is loaded
    # first serves both.  Load torch's first so that torch tensors and the
    # library share it (torch fails to find the GPU under the other one).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class _Arg:
    """One array argument: keeps the owning object alive, exposes its address."""

    def __init__(self, x, dtype, device: bool):
        if device:
            import torch

            tdt = {np.int64: torch.int64, np.int32: torch.int32, np.float32: torch.float32}[dtype]
            if not (_is_torch(x) and x.is_cuda):
                raise TypeError("device call: every array must be a GPU torch tensor")
            if x.dtype != tdt:
                raise TypeError(f"expected {tdt}, got {x.dtype}")
            self.obj = x.contiguous()
            self.ptr = self.obj.data_ptr()
        else:
            if _is_torch(x):
                x = x.detach().cpu().numpy()
            self.obj = np.ascontiguousarray(x, dtype=dtype)
            self.ptr = self.obj.ctypes.data


def _device_mode(*xs) -> bool:
    d = [(_is_torch(x) and x.is_cuda) for x in xs]
    if any(d) and not all(d):
        raise TypeError("mix of host and GPU arrays")
    return all(d)


def _opts(method, k, direction, precision, exclude_self=-1):
    o = lcemd_opts()
    o.method = METHOD[method] if isinstance(method, str) else int(method)
    o.k = int(k)
    o.direction = DIRECTION[direction] if isinstance(direction, str) else int(direction)
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.exclude_self = int(exclude_self)
    return o


class Context:
    """One lcemd context on one GPU (the same names as the C entry points)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        h = C.c_void_p()
        rc = self.lib.lcemd_create(C.byref(h), int(device))
        if rc != OK:
            raise LcemdError(rc, self.lib.lcemd_last_error(None).decode())
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.lcemd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            raise LcemdError(rc, self.lib.lcemd_last_error(self.h).decode())
        return rc

    def last_error(self) -> str:
        return self.lib.lcemd_last_error(self.h).decode()

    def _sync_stream(self, device: bool):
        if device:
            import torch

            self._check(self.lib.lcemd_set_stream(self.h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))
        else:
            self._check(self.lib.lcemd_use_own_stream(self.h))

    # ---- loads ----
    def load_embeddings(self, V, l2_normalize: bool = False, precisions=()):
        """precisions: reduced-precision copies to build now ("bf16", "fp8")
        rather than at the first call that asks for them."""
        dev = _device_mode(V)
        self._sync_stream(dev)
        a = _Arg(V, np.float32, dev)
        v, m = a.obj.shape
        make = {"bf16": MAKE_BF16, "fp8": MAKE_FP8}
        flags = (PTR_DEVICE if dev else 0) | (L2_NORMALIZE if l2_normalize else 0)
        for p in precisions:
            if p not in make:
                raise ValueError(f"precision {p!r}: one of {sorted(make)}")
            flags |= make[p]
        self._check(self.lib.lcemd_load_embeddings(self.h, C.c_void_p(a.ptr), v, m, flags))

    def load_database(self, rowptr, col, val, normalize: bool = False):
        dev = _device_mode(rowptr, col, val)
        self._sync_stream(dev)
        p, c, v = _Arg(rowptr, np.int64, dev), _Arg(col, np.int32, dev), _Arg(val, np.float32, dev)
        n = p.obj.shape[0] - 1
        flags = (PTR_DEVICE if dev else 0) | (NORMALIZE if normalize else 0)
        self._check(self.lib.lcemd_load_database(self.h, C.c_void_p(p.ptr), C.c_void_p(c.ptr),
                                                 C.c_void_p(v.ptr), n, flags))
        self._n = int(n)

    def used_vocab(self) -> np.ndarray:
        cnt = self.lib.lcemd_used_vocab(self.h, None)
        out = np.empty(max(cnt, 0), dtype=np.int32)
        self.lib.lcemd_used_vocab(self.h, C.c_void_p(out.ctypes.data))
        return out

    # ---- queries ----
    def _query(self, qptr, qcol, qval):
        dev = _device_mode(qptr, qcol, qval)
        self._sync_stream(dev)
        p, c, v = _Arg(qptr, np.int64, dev), _Arg(qcol, np.int32, dev), _Arg(qval, np.float32, dev)
        q = lcemd_query()
        q.rowptr, q.col, q.val = p.ptr, c.ptr, v.ptr
        q.B = p.obj.shape[0] - 1
        q.flags = PTR_DEVICE if dev else 0
        return q, (p, c, v), dev

    def distances(self, qptr, qcol, qval, method="act", k=1, direction="sym", precision="fp32",
                  n: Optional[int] = None, out=None):
        """B x n distances; host numpy in -> numpy out, GPU tensors in ->
        GPU tensor out (``out`` may be given)."""
        q, keep, dev = self._query(qptr, qcol, qval)
        o = _opts(method, k, direction, precision)
        n = self.n if n is None else n
        if dev:
            import torch

            if out is None:
                out = torch.empty((q.B, n), dtype=torch.float32, device=qptr.device)
            ptr = out.data_ptr()
        else:
            out = np.empty((q.B, n), dtype=np.float32)
            ptr = out.ctypes.data
        self._check(self.lib.lcemd_distances(self.h, C.byref(q), C.byref(o), C.c_void_p(ptr)))
        return out

    def topl(self, qptr, qcol, qval, l, method="act", k=1, direction="sym", precision="fp32",
             exclude_self=-1, out=None):
        q, keep, dev = self._query(qptr, qcol, qval)
        o = _opts(method, k, direction, precision, exclude_self)
        if dev:
            import torch

            if out is None:
                out = (torch.empty((q.B, l), dtype=torch.int64, device=qptr.device),
                       torch.empty((q.B, l), dtype=torch.float32, device=qptr.device))
            pi, pd = out[0].data_ptr(), out[1].data_ptr()
        else:
            out = (np.empty((q.B, l), dtype=np.int64), np.empty((q.B, l), dtype=np.float32))
            pi, pd = out[0].ctypes.data, out[1].ctypes.data
        self._check(self.lib.lcemd_topl(self.h, C.byref(q), C.byref(o), int(l), C.c_void_p(pi),
                                        C.c_void_p(pd)))
        return out

    def topl_noalloc(self, qptr, qcol, qval, l, out, method="act", k=1, precision="fp32", exclude_self=-1):
        """lcemd_topl_noalloc: D2Q top-l with device tensors only; `out` =
        (idx int64, dist float32) device tensors of shape (B, l)."""
        q, keep, dev = self._query(qptr, qcol, qval)  # the library refuses host arrays
        o = _opts(method, k, "d2q", precision, exclude_self)
        self._check(self.lib.lcemd_topl_noalloc(self.h, C.byref(q), C.byref(o), int(l),
                                                C.c_void_p(out[0].data_ptr()), C.c_void_p(out[1].data_ptr())))
        return out

    def selfjoin_topl(self, l, method="act", k=1, direction="sym", precision="fp32", device=False,
                      exclude_self=-1):
        """Every database histogram against all others (itself excluded):
        (idx, dist) of shape (n, l); torch tensors on the GPU if device."""
        o = _opts(method, k, direction, precision, exclude_self)
        if device:
            import torch

            out = (torch.empty((self.n, l), dtype=torch.int64, device="cuda"),
                   torch.empty((self.n, l), dtype=torch.float32, device="cuda"))
            pi, pd, fl = out[0].data_ptr(), out[1].data_ptr(), PTR_DEVICE
            self._sync_stream(True)
        else:
            out = (np.empty((self.n, l), dtype=np.int64), np.empty((self.n, l), dtype=np.float32))
            pi, pd, fl = out[0].ctypes.data, out[1].ctypes.data, 0
        self._check(self.lib.lcemd_selfjoin_topl(self.h, C.byref(o), int(l), fl, C.c_void_p(pi),
                                                 C.c_void_p(pd)))
        return out

    def tables(self, qptr, qcol, qval, k, precision="fp32"):
        q, keep, dev = self._query(qptr, qcol, qval)
        o = _opts("act", k, "d2q", precision)
        nu = self.lib.lcemd_used_vocab(self.h, None)
        shape = (q.B, nu, k)
        if dev:
            import torch

            S = torch.empty(shape, dtype=torch.int32, device=qptr.device)
            Z = torch.empty(shape, dtype=torch.float32, device=qptr.device)
            W = torch.empty(shape, dtype=torch.float32, device=qptr.device)
            ptrs = (S.data_ptr(), Z.data_ptr(), W.data_ptr())
        else:
            S = np.empty(shape, dtype=np.int32)
            Z = np.empty(shape, dtype=np.float32)
            W = np.empty(shape, dtype=np.float32)
            ptrs = (S.ctypes.data, Z.ctypes.data, W.ctypes.data)
        self._check(self.lib.lcemd_tables(self.h, C.byref(q), C.byref(o), *[C.c_void_p(p) for p in ptrs]))
        return S, Z, W

    # ---- profiling ----
    def profile(self, enable: bool = True):
        self._check(self.lib.lcemd_profile(self.h, int(bool(enable))))

    def profile_get(self):
        cnt = self.lib.lcemd_profile_get(self.h, None, 0)
        arr = (lcemd_phase_time * max(cnt, 1))()
        self.lib.lcemd_profile_get(self.h, arr, cnt)
        return [dict(name=arr[i].name.decode(), ms=arr[i].ms, launches=arr[i].launches,
                     work=arr[i].work) for i in range(cnt)]

    def counters(self):
        """(query tiles redone with float32 keys / deeper lists, bf16 rows
        redone exactly one by one), cumulative since creation."""
        a, b = C.c_int64(), C.c_int64()
        self._check(self.lib.lcemd_counters(self.h, C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    @property
    def n(self) -> int:
        return self._n

    @n.setter
    def n(self, value):
        self._n = value


class Server:
    """Continuous-batching server on a loaded Context (lcemd_server_*).  While
    it runs, the context belongs to the server's worker thread."""

    def __init__(self, ctx: "Context", method="act", k=8, precision="fp32", l=16,
                 max_slots=64, max_batch_words=0, memory_budget=0, use_graph=True, lanes=0):
        self.lib = ctx.lib
        cfg = lcemd_server_cfg()
        cfg.method = METHOD[method] if isinstance(method, str) else int(method)
        cfg.k = int(k)
        cfg.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
        cfg.l = int(l)
        cfg.max_slots = int(max_slots)
        cfg.max_batch_words = int(max_batch_words)
        cfg.memory_budget = int(memory_budget)
        cfg.use_graph = int(bool(use_graph))
        cfg.lanes = int(lanes)
        h = C.c_void_p()
        rc = self.lib.lcemd_server_start(ctx.h, C.byref(cfg), C.byref(h))
        if rc != OK:
            raise LcemdError(rc, self.lib.lcemd_last_error(ctx.h).decode())
        self.h = h
        self.l = int(l)
        self.ctx = ctx

    def submit(self, col, val) -> int:
        c = np.ascontiguousarray(col, dtype=np.int32)
        v = np.ascontiguousarray(val, dtype=np.float32)
        t = C.c_uint64()
        rc = self.lib.lcemd_server_submit(self.h, C.c_void_p(c.ctypes.data), C.c_void_p(v.ctypes.data),
                                          int(c.shape[0]), C.byref(t))
        if rc != OK:
            raise LcemdError(rc, "submit rejected")
        return int(t.value)

    def wait(self, ticket: int):
        idx = np.empty(self.l, dtype=np.int64)
        dist = np.empty(self.l, dtype=np.float32)
        lat = C.c_double()
        rc = self.lib.lcemd_server_wait(self.h, C.c_uint64(ticket), C.c_void_p(idx.ctypes.data),
                                        C.c_void_p(dist.ctypes.data), C.byref(lat))
        if rc != OK:
            raise LcemdError(rc, "query failed")
        return idx, dist, float(lat.value)

    def stop(self):
        if getattr(self, "h", None):
            self.lib.lcemd_server_stop(self.h)
            self.h = None

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def check_histograms(rowptr, col, val, v: int, require_normalized: bool = True):
    """Host-side validation of a CSR histogram batch (no GPU needed): returns
    (status code, message)."""
    lib = load_library()
    p, c, w = _Arg(rowptr, np.int64, False), _Arg(col, np.int32, False), _Arg(val, np.float32, False)
    msg = C.create_string_buffer(512)
    rc = lib.lcemd_check_histograms(C.c_void_p(p.ptr), C.c_void_p(c.ptr), C.c_void_p(w.ptr),
                                    p.obj.shape[0] - 1, int(v), int(require_normalized), msg, 512)
    return rc, msg.value.decode()


def serve_sim(arrival_s, words, lanes: int, max_slots: int, max_words: int, budget: int,
              per_query_bytes: float, t_fixed_s: float, t_per_query_s: float):
    """The serving admission policy on the host with a fake executor
    (lcemd_serve_sim): returns (slots per lane, status, lane, launch, start,
    finish) arrays, one entry per query."""
    lib = load_library()
    a = np.ascontiguousarray(arrival_s, dtype=np.float64)
    w = np.ascontiguousarray(words, dtype=np.int32)
    nq = a.shape[0]
    status, lane, launch = (np.empty(nq, dtype=np.int32) for _ in range(3))
    start, finish = np.empty(nq, dtype=np.float64), np.empty(nq, dtype=np.float64)
    rc = lib.lcemd_serve_sim(nq, a.ctypes.data, w.ctypes.data, int(lanes), int(max_slots), int(max_words),
                             int(budget), float(per_query_bytes), float(t_fixed_s), float(t_per_query_s),
                             status.ctypes.data, lane.ctypes.data, launch.ctypes.data, start.ctypes.data,
                             finish.ctypes.data)
    if rc < 0:
        raise LcemdError(rc, "serve_sim")
    return rc, status, lane, launch, start, finish


def open_context(V, db_rowptr, db_col, db_val, device: int = 0, l2_normalize: bool = False,
                 precisions=()) -> Context:
    """Context with embeddings and database loaded."""
    ctx = Context(device)
    ctx.load_embeddings(V, l2_normalize=l2_normalize, precisions=precisions)
    ctx.load_database(db_rowptr, db_col, db_val)
    ctx.n = int(db_rowptr.shape[0] - 1)
    return ctx
