"""Leader-based refinement (Algorithm 2, naivePR; with the closure, transPR)
on the GPU against the oracle's Algorithm 2: same partition as Hopcroft and
the same number of while-loop iterations (the election is deterministic on
both sides: the least candidate wins)."""
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


def _leader(ctx, d, closure="off", no_graph=False):
    from paper_2410_22764_amd import dfamin
    print(f"[case] leader {d.name} n={d.n} k={d.k} closure={closure} no_graph={no_graph}", flush=True)
    return dfamin.dfamin_minimize(ctx, d, dict(closure=closure, method="leader", no_graph=no_graph))


def _expect(d, closure):
    want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
    if closure == "on":
        _, _, it = oracle.naive_closure(d.n, d.k, d.delta, d.accept)
    else:
        _, _, it = oracle.naive(d.n, d.k, d.delta, d.accept)
    return want, nb, it


CASES = [
    lambda: W.random_dfa(1, 2, 1),
    lambda: W.random_dfa(257, 1, 2),
    lambda: W.random_dfa(1025, 3, 3),
    lambda: W.random_dfa(6000, 2, 4),
    lambda: W.chain_dfa(300, 2),
    lambda: W.permuted_chain_dfa(1000, 3, 5),
    lambda: W.fib_dfa(12),
    lambda: W.bitsplitter_dfa(9),
]


@pytest.mark.parametrize("closure", ["off", "on"])
@pytest.mark.parametrize("which", range(len(CASES)))
def test_leader_matches_oracle_iterations(ctx, which, closure):
    d = CASES[which]()
    want, nb, it = _expect(d, closure)
    out, res = _leader(ctx, d, closure)
    assert res["num_blocks"] == nb and np.array_equal(out, want)
    assert res["rounds_executed"] == it and res["refine_rounds"] == it - 1


def test_leader_coarse_partition(ctx):
    d = W.random_dfa(5000, 3, 9)
    acc = np.zeros(d.n, bool)
    acc[::53] = True
    d.accept = W.pack_accept(acc)
    want, nb, it = _expect(d, "off")
    out, res = _leader(ctx, d)
    assert np.array_equal(out, want) and res["rounds_executed"] == it


def test_table2_naive_fib20_on_gpu(ctx):
    """Table 2 prints 17,710 naivePR iterations for Fib_20."""
    d = W.fib_dfa(20)
    out, res = _leader(ctx, d)
    assert res["num_blocks"] == 17711 and np.array_equal(out, np.arange(17711))
    assert res["rounds_executed"] == 17710


def test_leader_graph_and_direct_launches_agree(ctx):
    """Rounds replayed from the captured graph (reused across calls with the
    same buffers) and launched one by one give the same result each time."""
    d = W.permuted_chain_dfa(3000, 2, 7)
    base, rb = _leader(ctx, d, no_graph=True)
    for _ in range(3):
        out, r = _leader(ctx, d)
        assert np.array_equal(out, base) and r == rb
        other = W.random_dfa(2000, 2, 8)  # other work between the replays
        o2, _ = _leader(ctx, other)
        want, _ = oracle.hopcroft(other.n, other.k, other.delta, other.accept)
        assert np.array_equal(o2, want)


def test_leader_auto_closure(ctx):
    for d in [W.chain_dfa(2000, 2), W.fib_dfa(14), W.random_dfa(3000, 2, 11)]:
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        out, res = _leader(ctx, d, "auto")
        assert res["num_blocks"] == nb and np.array_equal(out, want)


def test_leader_batch_matches_solo(ctx):
    from paper_2410_22764_amd import dfamin
    dfas = W.batch_mixed(seed=6, count=30, n_min=16, n_max=3000)
    for closure in ["off", "on"]:
        print(f"[case] leader batch closure={closure}", flush=True)
        outs, results = dfamin.dfamin_minimize_batch(ctx, dfas, dict(closure=closure, method="leader"))
        for d, o, r in zip(dfas, outs, results):
            want, nb, it = _expect(d, closure)
            assert r["num_blocks"] == nb and np.array_equal(o, want), d.name
            assert r["rounds_executed"] == it, d.name


def test_leader_options_rejected(ctx):
    from paper_2410_22764_amd import dfamin
    d = W.random_dfa(100, 2, 1)
    _, res = dfamin.dfamin_minimize(ctx, d, dfamin.make_opts(method=2), check=False)
    assert res["rc"] == dfamin.DFAMIN_E_INVAL
    o = dfamin.make_opts()
    o.flags = 4  # no such flag
    _, res = dfamin.dfamin_minimize(ctx, d, o, check=False)
    assert res["rc"] == dfamin.DFAMIN_E_INVAL
    with pytest.raises(dfamin.DfaminError):
        dfamin.dfamin_submit(ctx, d, dict(method="leader"))
