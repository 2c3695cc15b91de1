"""CPU oracle for DFA minimization -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It wraps ``liboracle.so`` (plain C99, built by
``oracle/build_oracle.py``) and shares no code with the GPU library: no
kernels, headers, helpers or tables.  Inputs are plain numpy arrays:

* ``delta``: uint32, length ``k*n``, letter-major (``delta[a*n + q]`` is the
  successor of state ``q`` under letter ``a``; the paper's Preliminaries,
  "Representation").
* ``accept``: uint8 bitmap of ``ceil(n/8)`` bytes, LSB first.

Every partition returned is canonical: block ids in increasing order of each
block's least member state.

Pinning (what makes these functions trustworthy, see ``tests/test_oracle_*``):
Hopcroft, Moore, pair marking and literal word enumeration are checked
against each other on every DFA with n <= 3, k <= 2 and n = 4, k = 2; Moore's
round counts and the closure are pinned to the paper's worked example
(Figure 1), its Fibonacci and bit-splitter tables (Table 2), Figure 2's
explicit automata and closed forms for chains.
"""
import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_U32P = ctypes.POINTER(ctypes.c_uint32)
_U8P = ctypes.POINTER(ctypes.c_uint8)


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle
        build_oracle.build()
    lib = ctypes.CDLL(_LIB_PATH)
    u32, u64 = ctypes.c_uint32, ctypes.c_uint64
    lib.oracle_canonicalize.argtypes = [u32, _U32P, _U32P]
    lib.oracle_canonicalize.restype = u32
    lib.oracle_hopcroft.argtypes = [u32, u32, _U32P, _U8P, _U32P, _U32P]
    lib.oracle_hopcroft.restype = ctypes.c_int
    lib.oracle_moore.argtypes = [u32, u32, _U32P, _U8P, u32, _U32P, _U32P, _U32P]
    lib.oracle_moore.restype = ctypes.c_int
    lib.oracle_moore_partial.argtypes = [u32, u32, _U32P, _U8P, u32, _U32P, _U32P, _U32P]
    lib.oracle_moore_partial.restype = ctypes.c_int
    lib.oracle_moore_from.argtypes = [u32, u32, _U32P, _U32P, u32, _U32P, _U32P, _U32P]
    lib.oracle_moore_from.restype = ctypes.c_int
    lib.oracle_naive.argtypes = [u32, u32, _U32P, _U8P, u32, _U32P, _U32P, _U32P]
    lib.oracle_naive.restype = ctypes.c_int
    lib.oracle_minimal_dfa.argtypes = [u32, u32, _U32P, _U8P, u32, _U32P, _U32P, _U8P, _U32P, _U32P]
    lib.oracle_minimal_dfa.restype = ctypes.c_int
    lib.oracle_closure.argtypes = [u32, u32, _U32P, u32, _U32P]
    lib.oracle_closure.restype = ctypes.c_int
    lib.oracle_floor_log2.argtypes = [u32]
    lib.oracle_floor_log2.restype = u32
    lib.oracle_pair_marking.argtypes = [u32, u32, _U32P, _U8P, _U32P, _U32P]
    lib.oracle_pair_marking.restype = ctypes.c_int
    lib.oracle_word_equivalence.argtypes = [u32, u32, _U32P, _U8P, _U32P, _U32P]
    lib.oracle_word_equivalence.restype = ctypes.c_int
    lib.oracle_reachable.argtypes = [u32, u32, _U32P, u32, _U8P]
    lib.oracle_reachable.restype = u32
    lib.oracle_exhaustive_check.argtypes = [u32, u32, ctypes.POINTER(u64)]
    lib.oracle_exhaustive_check.restype = u64
    _lib = lib
    return lib


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_U32P)


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(_U8P)


def _check(rc, name):
    if rc != 0:
        raise OracleError(f"{name} failed with code {rc}")


def floor_log2(n):
    return int(_load().oracle_floor_log2(n))


def canonicalize(labels):
    lab, lp = _u32(labels)
    out = np.empty(lab.size, np.uint32)
    nb = _load().oracle_canonicalize(lab.size, lp, out.ctypes.data_as(_U32P))
    return out, int(nb)


def hopcroft(n, k, delta, accept):
    """Hopcroft's algorithm: returns (canonical block per state, num_blocks)."""
    d, dp = _u32(delta)
    a, ap = _u8(accept)
    out = np.empty(n, np.uint32)
    nb = ctypes.c_uint32()
    _check(_load().oracle_hopcroft(n, k, dp, ap, out.ctypes.data_as(_U32P),
                                   ctypes.byref(nb)), "hopcroft")
    return out, nb.value


def hopcroft_many(dfas, threads=None):
    """Hopcroft on a list of (n, k, delta, accept) tuples over a thread pool.

    ctypes releases the GIL for the duration of each C call, so the pool
    runs the instances truly in parallel."""
    threads = threads or os.cpu_count() or 1
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda t: hopcroft(*t), dfas))


def moore(n, k, delta, accept, max_rounds=0):
    """Moore refinement: returns (canonical blocks, num_blocks, refine_rounds)."""
    d, dp = _u32(delta)
    a, ap = _u8(accept)
    out = np.empty(n, np.uint32)
    nb, rr = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_load().oracle_moore(n, k, dp, ap, max_rounds, out.ctypes.data_as(_U32P),
                                ctypes.byref(nb), ctypes.byref(rr)), "moore")
    return out, nb.value, rr.value


def moore_partial(n, k, delta, accept, rounds):
    """Partition after ``rounds`` Moore rounds: (canonical blocks, count, refining rounds)."""
    d, dp = _u32(delta)
    a, ap = _u8(accept)
    out = np.empty(n, np.uint32)
    nb, rr = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_load().oracle_moore_partial(n, k, dp, ap, rounds, out.ctypes.data_as(_U32P),
                                        ctypes.byref(nb), ctypes.byref(rr)), "moore_partial")
    return out, nb.value, rr.value


def moore_from(n, k, delta, init, max_rounds=0):
    """Moore refinement from an arbitrary starting partition."""
    d, dp = _u32(delta)
    i, ip = _u32(init)
    out = np.empty(n, np.uint32)
    nb, rr = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_load().oracle_moore_from(n, k, dp, ip, max_rounds, out.ctypes.data_as(_U32P),
                                     ctypes.byref(nb), ctypes.byref(rr)), "moore_from")
    return out, nb.value, rr.value


def naive(n, k, delta, accept, max_iter=0):
    """Algorithm 2 (naivePR): (canonical blocks, count, while-loop iterations)."""
    d, dp = _u32(delta)
    a, ap = _u8(accept)
    out = np.empty(n, np.uint32)
    nb, it = ctypes.c_uint32(), ctypes.c_uint32()
    _check(_load().oracle_naive(n, k, dp, ap, max_iter, out.ctypes.data_as(_U32P),
                                ctypes.byref(nb), ctypes.byref(it)), "naive")
    return out, nb.value, it.value


def naive_closure(n, k, delta, accept, L=None, max_iter=0):
    """The paper's transPR: naivePR on the closure automaton (alphabet Sigma^T)."""
    rows = closure(n, k, delta, L)
    return naive(n, rows.shape[0], rows.reshape(-1), accept, max_iter)


def closure(n, k, delta, L=None):
    """Partial transitive closure (Algorithm 5): array of shape (k*(L+1), n)."""
    if L is None:
        L = floor_log2(n)
    d, dp = _u32(delta)
    rows = np.empty(k * (L + 1) * n, np.uint32)
    _check(_load().oracle_closure(n, k, dp, L, rows.ctypes.data_as(_U32P)), "closure")
    return rows.reshape(k * (L + 1), n)


def moore_closure(n, k, delta, accept, L=None, max_rounds=0):
    """Moore refinement on the closure automaton A' (alphabet Sigma^T)."""
    rows = closure(n, k, delta, L)
    return moore(n, rows.shape[0], rows.reshape(-1), accept, max_rounds)


def pair_marking(n, k, delta, accept):
    d, dp = _u32(delta)
    a, ap = _u8(accept)
    out = np.empty(n, np.uint32)
    nb = ctypes.c_uint32()
    _check(_load().oracle_pair_marking(n, k, dp, ap, out.ctypes.data_as(_U32P),
                                       ctypes.byref(nb)), "pair_marking")
    return out, nb.value


def word_equivalence(n, k, delta, accept):
    d, dp = _u32(delta)
    a, ap = _u8(accept)
    out = np.empty(n, np.uint32)
    nb = ctypes.c_uint32()
    _check(_load().oracle_word_equivalence(n, k, dp, ap, out.ctypes.data_as(_U32P),
                                           ctypes.byref(nb)), "word_equivalence")
    return out, nb.value


def reachable(n, k, delta, q0):
    d, dp = _u32(delta)
    mark = np.empty(n, np.uint8)
    cnt = _load().oracle_reachable(n, k, dp, q0, mark.ctypes.data_as(_U8P))
    return mark.astype(bool), int(cnt)


def minimal_dfa(n, k, delta, accept, q0):
    """Minimal DFA of the states reachable from q0:
    (min_n, delta_min (k*min_n, letter-major), accept bitmap, q0_min, reachable count)."""
    d, dp = _u32(delta)
    a, ap = _u8(accept)
    md = np.empty(max(k * n, 1), np.uint32)
    ma = np.zeros(max((n + 7) // 8, 1), np.uint8)
    mn, mq, nr = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(_load().oracle_minimal_dfa(n, k, dp, ap, q0, ctypes.byref(mn), md.ctypes.data_as(_U32P),
                                      ma.ctypes.data_as(_U8P), ctypes.byref(mq), ctypes.byref(nr)),
           "minimal_dfa")
    m = mn.value
    return m, md[: k * m].copy(), ma[: (m + 7) // 8].copy(), mq.value, nr.value


def exhaustive_check(n, k):
    """Returns (number of DFAs checked, number of disagreements)."""
    bad = ctypes.c_uint64()
    checked = _load().oracle_exhaustive_check(n, k, ctypes.byref(bad))
    return int(checked), int(bad.value)
