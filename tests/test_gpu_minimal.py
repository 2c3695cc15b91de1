"""The minimal DFA of the states reachable from q0 on the GPU (breadth-first
reachability and the quotient) against the oracle's construction: the same
numbering (least member of each class) on both sides, so results are
compared exactly."""
import numpy as np
import pytest

import oracle
from paper_2410_22764_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_22764_amd import dfamin
    c = dfamin.dfamin_create(0)
    yield c
    c.close()


def _check(ctx, d, closure="auto"):
    from paper_2410_22764_amd import dfamin
    print(f"[case] minimal {d.name} n={d.n} k={d.k} q0={d.q0}", flush=True)
    m, dm, am, info, out = dfamin.dfamin_minimal_dfa(ctx, d, {"closure": closure})
    em, edm, eam, eq0, enr = oracle.minimal_dfa(d.n, d.k, d.delta, d.accept, d.q0)
    assert m == em and info["q0"] == eq0 and info["reachable"] == enr
    assert np.array_equal(dm, edm) and np.array_equal(am, eam)
    want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
    assert info["num_blocks"] == nb and np.array_equal(out, want)
    return info


@pytest.mark.parametrize("seed", range(6))
def test_minimal_random(ctx, seed):
    n = [1, 7, 300, 4097, 70000, 1 << 21][seed]
    d = W.random_dfa(n, 1 + seed % 4, seed + 3)
    d.q0 = (seed * 104729) % n
    _check(ctx, d)


def test_minimal_structured(ctx):
    _check(ctx, W.chain_dfa(1000, 2))
    _check(ctx, W.permuted_chain_dfa(2000, 3, 4))
    _check(ctx, W.fib_dfa(14))
    info = _check(ctx, W.bitsplitter_dfa(12))
    assert info["reachable"] == 1
    d = W.random_dfa(5000, 2, 8)
    acc = np.zeros(d.n, bool)
    acc[::41] = True
    d.accept = W.pack_accept(acc)
    _check(ctx, d)
    d.accept = W.pack_accept(np.zeros(d.n, bool))
    _check(ctx, d, "off")


def test_minimal_deep_chain_uses_closure_edges(ctx):
    """A chain of 2^16 states from state 0: after 64 levels the closure
    letters join the search, so far fewer levels than states run."""
    d = W.chain_dfa(1 << 16, 2)
    info = _check(ctx, d, "off")
    assert info["n"] == d.n and info["reachable"] == d.n
    assert info["bfs_levels"] < 64 + 4 * 17
