"""ctypes binding of libdfamin.so: the C-ABI of ``include/dfamin.h``, same names.

This module only marshals arguments; every step of the method runs in the
HIP kernels of the native library.  If the library has not been built, or a
call cannot reach a GPU, it raises -- there is no CPU fallback.

DFAs are passed either as objects with ``n, k, delta, accept, q0`` attributes
(``workloads.DFA``) or as device pointers for the ``*_device`` calls (e.g.
``tensor.data_ptr()`` of torch tensors on the context's device; PyTorch is
only used for device memory and streams).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfamin.so")

DFAMIN_OK = 0
DFAMIN_E_INVAL = -1
DFAMIN_E_BAD_DFA = -2
DFAMIN_E_NOMEM = -3
DFAMIN_E_DEVICE = -4
DFAMIN_E_TIMEOUT = -5
DFAMIN_E_CANCELLED = -6
DFAMIN_E_BUSY = -7
DFAMIN_E_INTERNAL = -8

CLOSURE = {"auto": 0, "off": 1, "on": 2}  # 0 (AUTO) is what a zeroed or NULL options struct means

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "dfamin_create", "dfamin_destroy", "dfamin_minimize", "dfamin_minimize_device",
    "dfamin_minimize_batch", "dfamin_minimize_batch_device", "dfamin_submit", "dfamin_wait",
    "dfamin_cancel", "dfamin_status_str", "dfamin_set_profiling", "dfamin_get_kernel_stats",
    "dfamin_set_tuning", "dfamin_minimal_dfa", "dfamin_minimize_device_noalloc",
]


class Dfa(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("k", ctypes.c_uint32),
                ("delta", ctypes.c_void_p), ("accept", ctypes.c_void_p),
                ("q0", ctypes.c_uint32)]


class Opts(ctypes.Structure):
    _fields_ = [("closure", ctypes.c_uint32), ("max_levels", ctypes.c_uint32),
                ("auto_rounds", ctypes.c_uint32), ("max_rounds", ctypes.c_uint32),
                ("method", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Minimal(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint32), ("q0", ctypes.c_uint32), ("num_blocks", ctypes.c_uint32),
                ("reachable", ctypes.c_uint32), ("bfs_levels", ctypes.c_uint32),
                ("refine_rounds", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 2)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Result(ctypes.Structure):
    _fields_ = [("num_blocks", ctypes.c_uint32), ("initial_block", ctypes.c_uint32),
                ("refine_rounds", ctypes.c_uint32), ("rounds_executed", ctypes.c_uint32),
                ("closure_levels", ctypes.c_uint32), ("closure_letters", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


class DfaminError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {status_str(code)} ({code})" if what else f"{status_str(code)} ({code})")


_lib = None


def load():
    """Load libdfamin.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2410_22764_amd.build.build()")
    # PyTorch bundles its own HIP runtime under the same soname.  Loading it
    # first makes libdfamin bind to that copy, so the process holds a single
    # HIP runtime whether or not the caller uses torch tensors afterwards.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, u32, u64, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
    lib.dfamin_create.argtypes = [i32, u64, P(vp)]
    lib.dfamin_create.restype = i32
    lib.dfamin_destroy.argtypes = [vp]
    lib.dfamin_destroy.restype = None
    lib.dfamin_minimize.argtypes = [vp, P(Dfa), P(Opts), vp, P(Result)]
    lib.dfamin_minimize.restype = i32
    lib.dfamin_minimize_device.argtypes = [vp, P(Dfa), P(Opts), vp, P(Result), vp]
    lib.dfamin_minimize_device.restype = i32
    lib.dfamin_minimize_device_noalloc.argtypes = [vp, P(Dfa), P(Opts), vp, P(Result), vp]
    lib.dfamin_minimize_device_noalloc.restype = i32
    lib.dfamin_minimize_batch.argtypes = [vp, u32, P(Dfa), P(Opts), P(vp), P(Result)]
    lib.dfamin_minimize_batch.restype = i32
    lib.dfamin_minimize_batch_device.argtypes = [vp, u32, P(Dfa), P(Opts), P(vp), P(Result), vp]
    lib.dfamin_minimize_batch_device.restype = i32
    lib.dfamin_submit.argtypes = [vp, P(Dfa), P(Opts), P(u64)]
    lib.dfamin_submit.restype = i32
    lib.dfamin_wait.argtypes = [vp, u64, i64, vp, P(Result)]
    lib.dfamin_wait.restype = i32
    lib.dfamin_cancel.argtypes = [vp, u64]
    lib.dfamin_cancel.restype = i32
    lib.dfamin_status_str.argtypes = [i32]
    lib.dfamin_status_str.restype = ctypes.c_char_p
    lib.dfamin_set_profiling.argtypes = [vp, i32]
    lib.dfamin_set_profiling.restype = i32
    lib.dfamin_get_kernel_stats.argtypes = [vp, P(KernelStat), i32]
    lib.dfamin_get_kernel_stats.restype = i32
    lib.dfamin_set_tuning.argtypes = [vp, i32]
    lib.dfamin_set_tuning.restype = i32
    lib.dfamin_minimal_dfa.argtypes = [vp, P(Dfa), P(Opts), vp, vp, vp, P(Minimal)]
    lib.dfamin_minimal_dfa.restype = i32
    _lib = lib
    return lib


def status_str(code):
    return load().dfamin_status_str(int(code)).decode()


dfamin_status_str = status_str


METHOD = {"signature": 0, "leader": 1}
FLAG_NO_GRAPH = 1
FLAG_QUEUE = 2


def make_opts(closure="auto", max_levels=0, auto_rounds=0, max_rounds=0, method="signature", no_graph=False,
              queue=False):
    c = CLOSURE[closure] if isinstance(closure, str) else int(closure)
    m = METHOD[method] if isinstance(method, str) else int(method)
    flags = (FLAG_NO_GRAPH if no_graph else 0) | (FLAG_QUEUE if queue else 0)
    return Opts(c, max_levels, auto_rounds, max_rounds, m, flags)


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, Opts):
        return ctypes.byref(opts)
    if isinstance(opts, dict):
        return ctypes.byref(make_opts(**opts))
    if isinstance(opts, str):
        return ctypes.byref(make_opts(closure=opts))
    raise TypeError("opts must be None, a closure name, a dict or Opts")


class Ctx:
    """Owning handle of a dfamin_ctx."""

    def __init__(self, handle):
        self.handle = handle
        self.tickets = {}  # serving ticket -> n of the submitted DFA

    def close(self):
        if self.handle:
            load().dfamin_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def dfamin_create(device=0, hbm_budget_bytes=0):
    h = ctypes.c_void_p()
    rc = load().dfamin_create(int(device), int(hbm_budget_bytes), ctypes.byref(h))
    if rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_create")
    return Ctx(h)


def dfamin_destroy(ctx):
    ctx.close()


def _host_dfa(d, check=True):
    """Marshal a host DFA.  The library copies k*n transitions and ceil(n/8)
    accept bytes out of these buffers, so shorter arrays are refused here
    (ValueError) before any native call; check=False marshals as given."""
    n, k = int(d.n), int(d.k)
    delta = np.ascontiguousarray(d.delta, dtype=np.uint32).reshape(-1)
    accept = np.ascontiguousarray(d.accept, dtype=np.uint8).reshape(-1)
    if check:
        if delta.size != n * k:
            raise ValueError(f"delta holds {delta.size} entries, k*n = {n * k}")
        if accept.size < (n + 7) // 8:
            raise ValueError(f"accept holds {accept.size} bytes, ceil(n/8) = {(n + 7) // 8}")
    s = Dfa(n, k, delta.ctypes.data, accept.ctypes.data, int(d.q0))
    return s, (delta, accept)


def dfamin_minimize(ctx, dfa, opts=None, check=True):
    """Minimize a host DFA.  Returns (out: uint32[n], result dict)."""
    s, keep = _host_dfa(dfa)
    out = np.empty(int(dfa.n), np.uint32)
    res = Result()
    rc = load().dfamin_minimize(ctx.handle, ctypes.byref(s), _opts(opts), out.ctypes.data, ctypes.byref(res))
    if check and rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_minimize")
    r = res.as_dict()
    r["rc"] = rc
    return out, r


def dfamin_minimize_device(ctx, n, k, delta_ptr, accept_ptr, q0, out_ptr, opts=None, stream=0,
                           check=True):
    """Minimize a DFA whose buffers are device pointers; returns the result dict."""
    s = Dfa(int(n), int(k), int(delta_ptr), int(accept_ptr), int(q0))
    res = Result()
    rc = load().dfamin_minimize_device(ctx.handle, ctypes.byref(s), _opts(opts), int(out_ptr),
                                       ctypes.byref(res), int(stream) or None)
    if check and rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_minimize_device")
    r = res.as_dict()
    r["rc"] = rc
    return r


def dfamin_minimize_device_noalloc(ctx, n, k, delta_ptr, accept_ptr, q0, out_ptr, opts=None, stream=0,
                                   check=True):
    """As dfamin_minimize_device, through the entry point that allocates
    nothing (its device buffers live in the library's static scratch array)."""
    s = Dfa(int(n), int(k), int(delta_ptr), int(accept_ptr), int(q0))
    res = Result()
    rc = load().dfamin_minimize_device_noalloc(ctx.handle, ctypes.byref(s), _opts(opts), int(out_ptr),
                                               ctypes.byref(res), int(stream) or None)
    if check and rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_minimize_device_noalloc")
    r = res.as_dict()
    r["rc"] = rc
    return r


NOALLOC_SCRATCH_BYTES = 64 << 20


def noalloc_fits(n, k):
    """Whether dfamin_minimize_device_noalloc accepts an instance of n
    states and k letters (the size limit stated with its declaration)."""
    return n * (66 + 16 * (k + 1)) + (1 << 20) <= NOALLOC_SCRATCH_BYTES


def dfamin_minimize_batch(ctx, dfas, opts=None, check=True):
    """Minimize host DFAs together.  Returns (list of outs, list of result dicts)."""
    count = len(dfas)
    arr = (Dfa * max(count, 1))()
    keep = []
    outs = []
    optr = (ctypes.c_void_p * max(count, 1))()
    for i, d in enumerate(dfas):
        s, kp = _host_dfa(d)
        arr[i] = s
        keep.append(kp)
        o = np.empty(int(d.n), np.uint32)
        outs.append(o)
        optr[i] = o.ctypes.data
    res = (Result * max(count, 1))()
    rc = load().dfamin_minimize_batch(ctx.handle, count, arr, _opts(opts), optr, res)
    if check and rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_minimize_batch")
    results = [res[i].as_dict() for i in range(count)]
    for r in results:
        r["rc"] = rc
    return outs, results


class BatchDevice:
    """Arguments of dfamin_minimize_batch_device marshalled once: a batch of
    DFAs in device memory that is minimized repeatedly (same buffers) pays
    for building the ctypes arrays only here, not on every call."""

    def __init__(self, specs, out_ptrs):
        count = len(specs)
        self.count = count
        self.arr = (Dfa * max(count, 1))()
        for i, (n, k, dp, ap, q0) in enumerate(specs):
            self.arr[i] = Dfa(int(n), int(k), int(dp), int(ap), int(q0))
        self.optr = (ctypes.c_void_p * max(count, 1))(*[int(p) for p in out_ptrs])
        self.res = (Result * max(count, 1))()

    def run(self, ctx, opts=None, stream=0, check=True):
        rc = load().dfamin_minimize_batch_device(ctx.handle, self.count, self.arr, _opts(opts), self.optr,
                                                 self.res, int(stream) or None)
        if check and rc != DFAMIN_OK:
            raise DfaminError(rc, "dfamin_minimize_batch_device")
        return rc

    def field(self, name):
        """One result field for every instance, as a numpy array."""
        view = np.ctypeslib.as_array(self.res)
        return np.array(view[name][: self.count])

    def results(self, rc=DFAMIN_OK):
        out = [self.res[i].as_dict() for i in range(self.count)]
        for r in out:
            r["rc"] = rc
        return out


def dfamin_minimize_batch_device(ctx, specs, out_ptrs, opts=None, stream=0, check=True):
    """specs: list of (n, k, delta_ptr, accept_ptr, q0) with device pointers."""
    b = BatchDevice(specs, out_ptrs)
    rc = b.run(ctx, opts, stream, check)
    return b.results(rc)


def dfamin_submit(ctx, dfa, opts=None):
    s, keep = _host_dfa(dfa)
    t = ctypes.c_uint64()
    rc = load().dfamin_submit(ctx.handle, ctypes.byref(s), _opts(opts), ctypes.byref(t))
    if rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_submit")
    ctx.tickets[t.value] = int(dfa.n)
    return t.value


def dfamin_wait(ctx, ticket, n, timeout_us=-1):
    """Returns (rc, out or None, result dict).  The library writes the
    submitted DFA's n classes into `out`, so n must be at least that n for
    tickets of this context (ValueError otherwise)."""
    known = ctx.tickets.get(int(ticket))
    if known is not None and int(n) < known:
        raise ValueError(f"ticket {ticket} holds {known} states, out has room for {n}")
    out = np.empty(max(int(n), known or 0, 1), np.uint32)
    res = Result()
    rc = load().dfamin_wait(ctx.handle, int(ticket), int(timeout_us), out.ctypes.data, ctypes.byref(res))
    if rc != DFAMIN_E_TIMEOUT:
        ctx.tickets.pop(int(ticket), None)
    return rc, (out[: int(n)] if rc == DFAMIN_OK else None), res.as_dict()


def dfamin_cancel(ctx, ticket):
    return load().dfamin_cancel(ctx.handle, int(ticket))


def dfamin_set_profiling(ctx, on=True):
    rc = load().dfamin_set_profiling(ctx.handle, 1 if on else 0)
    if rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_set_profiling")


def dfamin_minimal_dfa(ctx, dfa, opts=None):
    """Minimal DFA of the states reachable from q0.  Returns (n_min,
    delta_min (k*n_min, letter-major), accept bitmap, info dict with q0 etc.,
    canonical class per input state)."""
    s, keep = _host_dfa(dfa)
    md = np.empty(max(dfa.k * dfa.n, 1), np.uint32)
    ma = np.zeros(max((dfa.n + 7) // 8, 1), np.uint8)
    out = np.empty(dfa.n, np.uint32)
    info = Minimal()
    rc = load().dfamin_minimal_dfa(ctx.handle, ctypes.byref(s), _opts(opts), md.ctypes.data, ma.ctypes.data,
                                   out.ctypes.data, ctypes.byref(info))
    if rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_minimal_dfa")
    m = info.n
    return m, md[: dfa.k * m].copy(), ma[: (m + 7) // 8].copy(), info.as_dict(), out


def dfamin_set_tuning(ctx, variant=-1):
    """-1: tune the signature tile per size class; 0, 1, 2: force 256, 512
    or 1024 states per workgroup."""
    rc = load().dfamin_set_tuning(ctx.handle, int(variant))
    if rc != DFAMIN_OK:
        raise DfaminError(rc, "dfamin_set_tuning")


def dfamin_get_kernel_stats(ctx):
    lib = load()
    n = lib.dfamin_get_kernel_stats(ctx.handle, None, 0)
    if n < 0:
        raise DfaminError(n, "dfamin_get_kernel_stats")
    arr = (KernelStat * max(n, 1))()
    lib.dfamin_get_kernel_stats(ctx.handle, arr, n)
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches,
             "total_ms": arr[i].total_ms, "alg_bytes": arr[i].alg_bytes} for i in range(n)]
