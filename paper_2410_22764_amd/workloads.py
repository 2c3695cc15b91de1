"""Seeded synthetic DFA generators (inputs only; no minimization arithmetic).

This module is the one piece shared by the GPU path's tests/benchmarks and
the CPU oracle's tests: it produces inputs and nothing else.  It imports
neither the GPU binding nor the oracle.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw ``i`` of stream ``key`` is ``mix(key + (i+1)*GAMMA)``.
Integers below ``n`` are drawn exactly by rejection (values at or above the
largest multiple of ``n`` below 2^64 are redrawn from a derived stream).

DFA layout (the paper's Preliminaries, "Representation"): states
``0..n-1``, letters ``0..k-1``, ``delta`` letter-major uint32 with
``delta[a*n + q] = delta(q, a)``; ``accept`` is a ceil(n/8)-byte bitmap, LSB
first.

Families:

* ``random_dfa``: every delta(q,a) i.i.d. uniform on [0,n), each state
  accepting with probability 1/2, q0 = 0 (no reachability fix-up).
* ``chain_dfa``: letter 0 maps i -> i+1 and n-1 -> n-1, every other letter is
  the identity, only n-1 accepts (generalises Figure 1 of the paper and the
  two-letter chain with an identity second letter).
* ``permuted_chain_dfa``: a chain whose state ids are relabelled by a seeded
  random permutation pi (state pi(i) plays chain state i; q0 = pi(0)).
* ``fib_dfa``: Fibonacci automata of Section 4.1 (unary cycle over the
  Fibonacci word w_i, accepting where the word has a 1).
* ``bitsplitter_dfa``: bit-splitters B_m of Section 4.1, 2^m states and m-1
  letters.  Reading used: a state is the integer x whose binary digits are
  the bit string (leftmost = most significant); letter a_j (j = 1..m-1)
  sends x to x with bit j flipped and bits 0..j-1 cleared when bit j-1 of x
  is set, and leaves x unchanged otherwise; F = {x : bit m-1 set}.  This
  reproduces all sixteen arrows of B_3 drawn in Figure 2.
* ``batch_mixed``: thousands of uneven instances (75% random, 25% permuted
  chains) for the batched workload; ``serving_stream``: a Poisson stream of
  requests for the serving workload.
"""
from dataclasses import dataclass, field
import math

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def _mix_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix_np(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * np.uint64(0xBF58476D1CE4E5B9)
    z = z ^ (z >> np.uint64(27))
    z = z * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _tag(t) -> int:
    if isinstance(t, str):
        v = 0
        for ch in t.encode():
            v = _mix_int(v * 131 + ch + 1)
        return v
    return int(t) & MASK64


def stream_key(seed: int, *tags) -> int:
    """Derive an independent 64-bit stream key from a seed and tags."""
    k = _mix_int((int(seed) & MASK64) * GAMMA + 0x2545F4914F6CDD1D)
    for t in tags:
        k = _mix_int(k ^ _mix_int(_tag(t) + GAMMA))
    return k


def draws(key: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` consecutive uint64 draws of stream ``key`` from ``start``."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(key) + idx * np.uint64(GAMMA)
        return _mix_np(z)


def uniform_below(key: int, count: int, n: int) -> np.ndarray:
    """Exact uniform integers in [0, n) by rejection, as uint64."""
    if n <= 0:
        raise ValueError("n must be positive")
    x = draws(key, count)
    limit = (1 << 64) - ((1 << 64) % n)
    if limit < (1 << 64):
        attempt = 0
        bad = np.nonzero(x >= np.uint64(limit))[0]
        while bad.size:
            attempt += 1
            sub = stream_key(key, "redraw", attempt)
            y = draws(sub, count)[bad]
            x[bad] = y
            bad = bad[y >= np.uint64(limit)]
    return x % np.uint64(n)


def unit_floats(key: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits (input sizes only)."""
    return (draws(key, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def pack_accept(bits: np.ndarray) -> np.ndarray:
    return np.packbits(np.asarray(bits, dtype=bool), bitorder="little")


@dataclass
class DFA:
    """A complete DFA in the boundary's layout."""
    n: int
    k: int
    delta: np.ndarray          # uint32[k*n], letter-major
    accept: np.ndarray         # uint8[ceil(n/8)], LSB first
    q0: int = 0
    name: str = ""
    meta: dict = field(default_factory=dict)

    def accept_bool(self) -> np.ndarray:
        return np.unpackbits(self.accept, bitorder="little", count=self.n).astype(bool)

    def rows(self) -> np.ndarray:
        return self.delta.reshape(self.k, self.n)

    @property
    def transitions(self) -> int:
        return self.n * self.k


def from_rows(rows, accept_bits, q0=0, name="") -> DFA:
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.uint32))
    k, n = rows.shape
    return DFA(n, k, rows.reshape(-1).copy(), pack_accept(accept_bits), q0, name)


def random_dfa(n: int, k: int, seed: int) -> DFA:
    delta = uniform_below(stream_key(seed, "random", n, k, "delta"), n * k, n).astype(np.uint32)
    acc = (draws(stream_key(seed, "random", n, k, "accept"), n) >> np.uint64(63)).astype(bool)
    return DFA(n, k, delta, pack_accept(acc), 0, f"random(n={n},k={k},seed={seed})")


def chain_dfa(n: int, k: int = 2) -> DFA:
    ids = np.arange(n, dtype=np.uint32)
    rows = np.empty((k, n), np.uint32)
    rows[0] = np.minimum(ids + 1, n - 1)
    for a in range(1, k):
        rows[a] = ids
    acc = np.zeros(n, bool)
    acc[n - 1] = True
    d = from_rows(rows, acc, 0, f"chain(n={n},k={k})")
    return d


def random_permutation(n: int, key: int) -> np.ndarray:
    keys = draws(key, n)
    return np.argsort(keys, kind="stable").astype(np.uint32)


def permute_dfa(d: DFA, pi: np.ndarray, name: str = "") -> DFA:
    """State pi[i] of the result plays state i of ``d``."""
    rows = d.rows()
    out = np.empty_like(rows)
    out[:, pi] = pi[rows]
    acc = np.zeros(d.n, bool)
    acc[pi] = d.accept_bool()
    return DFA(d.n, d.k, out.reshape(-1).copy(), pack_accept(acc), int(pi[d.q0]),
               name or d.name + "+perm")


def permuted_chain_dfa(n: int, k: int, seed: int) -> DFA:
    pi = random_permutation(n, stream_key(seed, "perm", n, k))
    d = permute_dfa(chain_dfa(n, k), pi, f"permuted_chain(n={n},k={k},seed={seed})")
    d.meta["perm"] = pi
    return d


def fib_word(i: int) -> str:
    """Fibonacci words: w_0 = 1, w_1 = 0, w_{i+1} = w_i w_{i-1}."""
    if i == 0:
        return "1"
    a, b = "1", "0"  # w_0, w_1
    for _ in range(1, i):
        a, b = b, b + a
    return b


def fib_dfa_word(i: int) -> DFA:
    """The automaton built on w_i: a unary cycle q_j -> q_{j+1 mod |w_i|},
    accepting where w_i has a 1 (Section 4.1 definition, states 0..|w_i|-1)."""
    w = fib_word(i)
    n = len(w)
    ids = np.arange(n, dtype=np.uint32)
    rows = ((ids + 1) % n).reshape(1, n)
    acc = np.array([c == "1" for c in w])
    return from_rows(rows, acc, 0, f"fib_word({i})")


def fib_dfa(m: int) -> DFA:
    """Fib_m as named in the paper's tables: N = |w_{m+1}| states."""
    d = fib_dfa_word(m + 1)
    d.name = f"Fib_{m}"
    return d


def bitsplitter_dfa(m: int) -> DFA:
    """B_m: 2^m states, letters a_1..a_{m-1} stored as letters 0..m-2."""
    if m < 1:
        raise ValueError("m >= 1")
    n = 1 << m
    x = np.arange(n, dtype=np.uint64)
    k = max(m - 1, 0)
    rows = np.empty((max(k, 1), n), np.uint32)
    if k == 0:
        rows[0] = x  # B_1 has no letters; one identity letter keeps delta complete
    for j in range(1, m):
        cond = ((x >> np.uint64(j - 1)) & np.uint64(1)) == 1
        moved = (x ^ np.uint64(1 << j)) & ~np.uint64((1 << j) - 1)
        rows[j - 1] = np.where(cond, moved, x).astype(np.uint32)
    acc = ((x >> np.uint64(m - 1)) & np.uint64(1)) == 1
    return from_rows(rows, acc, 0, f"B_{m}")


# --------------------------------------------------------------------------
# Benchmark workloads

def plain_single(seed: int = 1) -> DFA:
    """Random complete DFA, n = 16,384, |Sigma| = 2."""
    return random_dfa(16384, 2, seed)


def plain_large(seed: int = 1) -> DFA:
    """Random complete DFA, n = 2^24, |Sigma| = 4."""
    return random_dfa(1 << 24, 4, seed)


def deep_chain() -> DFA:
    """Chain DFA, n = 2^20, |Sigma| = 2 (second letter the identity)."""
    return chain_dfa(1 << 20, 2)


def batch_mixed(seed: int = 1, count: int = 4096, n_min: int = 64, n_max: int = 65536,
                k_min: int = 2, k_max: int = 8, chain_fraction: float = 0.25):
    """Uneven batch: n log-uniform in [n_min, n_max], k uniform in [k_min,k_max];
    exactly round(count*chain_fraction) permuted chains at shuffled positions,
    the rest random DFAs."""
    u = unit_floats(stream_key(seed, "batch", "n"), count)
    span = math.log2(n_max / n_min)
    ns = np.clip(np.floor(n_min * np.exp2(span * u)), n_min, n_max).astype(np.int64)
    ks = (k_min + uniform_below(stream_key(seed, "batch", "k"), count, k_max - k_min + 1)).astype(np.int64)
    n_chain = int(round(count * chain_fraction))
    order = random_permutation(count, stream_key(seed, "batch", "chains"))
    is_chain = np.zeros(count, bool)
    is_chain[order[:n_chain]] = True
    out = []
    for i in range(count):
        s = stream_key(seed, "batch", "instance", i)
        if is_chain[i]:
            out.append(permuted_chain_dfa(int(ns[i]), int(ks[i]), s))
        else:
            out.append(random_dfa(int(ns[i]), int(ks[i]), s))
    return out


def serving_stream(seed: int, count: int, rate_per_s: float, log2_min: int = 8,
                   log2_max: int = 22, k_min: int = 2, k_max: int = 16,
                   chain_fraction: float = 0.2):
    """Poisson request stream: returns (arrival_times_s, specs) where each spec
    is (kind, n, k, seed) and ``make_request(spec)`` builds the DFA."""
    u = unit_floats(stream_key(seed, "serve", "gap"), count)
    gaps = -np.log1p(-u) / rate_per_s
    arrivals = np.cumsum(gaps)
    un = unit_floats(stream_key(seed, "serve", "n"), count)
    ns = np.floor(np.exp2(log2_min + (log2_max - log2_min) * un)).astype(np.int64)
    ns = np.clip(ns, 1 << log2_min, 1 << log2_max)
    ks = (k_min + uniform_below(stream_key(seed, "serve", "k"), count, k_max - k_min + 1)).astype(np.int64)
    uc = unit_floats(stream_key(seed, "serve", "kind"), count)
    specs = []
    for i in range(count):
        kind = "chain" if uc[i] < chain_fraction else "random"
        specs.append((kind, int(ns[i]), int(ks[i]), stream_key(seed, "serve", "instance", i)))
    return arrivals, specs


def make_request(spec) -> DFA:
    kind, n, k, s = spec
    if kind == "chain":
        return permuted_chain_dfa(n, k, s)
    return random_dfa(n, k, s)
