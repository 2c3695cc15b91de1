"""GPU tests of the options and error paths: the default closure policy, the
memory-capped closure (a context's HBM budget, max_levels, auto_rounds),
E_NOMEM, and outputs left untouched on E_BAD_DFA.

The partition must always equal the oracle's; round counts follow from the
oracle's Moore partitions and closure levels (Section 3.4: every closure
letter is a word over Sigma, so any subset of levels gives the same classes
and only the number of rounds changes).
"""
import numpy as np
import pytest

import oracle
from paper_2410_22764_amd import workloads as W

pytestmark = pytest.mark.gpu

SENTINEL = 0x5A5A5A5A


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_22764_amd import dfamin
    c = dfamin.dfamin_create(0)
    yield c
    c.close()


def shift_dfa(n, shifts, name):
    """Letter s sends i to min(i + s, n - 1); only state n - 1 accepts.  With
    several shifts every letter is a non-identity letter (no doubling), and
    plain refinement needs about n / max(shift) rounds."""
    ids = np.arange(n, dtype=np.int64)
    rows = np.stack([np.minimum(ids + s, n - 1) for s in shifts]).astype(np.uint32)
    acc = np.zeros(n, bool)
    acc[n - 1] = True
    return W.from_rows(rows, acc, name=name)


def _hop(d):
    return oracle.hopcroft(d.n, d.k, d.delta, d.accept)


def test_null_options_mean_auto(ctx):
    """A NULL options pointer and a zeroed struct select closure AUTO: on a
    chain (one non-identity letter) the rounds double from the first one,
    ceil(log2(n - 1)) of them instead of the n - 2 of plain refinement."""
    from paper_2410_22764_amd import dfamin
    d = W.permuted_chain_dfa(5000, 3, 17)
    print("[case] NULL options on a 5000-state chain", flush=True)
    a, ra = dfamin.dfamin_minimize(ctx, d, None)
    z, rz = dfamin.dfamin_minimize(ctx, d, dfamin.Opts())
    e, re = dfamin.dfamin_minimize(ctx, d, "auto")
    assert np.array_equal(a, np.arange(d.n)) and np.array_equal(z, a) and np.array_equal(e, a)
    assert ra == rz == re
    assert ra["refine_rounds"] == 13 and ra["closure_levels"] > 0


def test_max_levels_caps_the_closure(ctx):
    """max_levels = 3: closure ON builds levels 0..3 only, and the rounds are
    Moore's on the closure automaton with L = 3; AUTO on a unary instance
    doubles with steps of at most 2^3."""
    from paper_2410_22764_amd import dfamin
    d = shift_dfa(3000, [1, 3], "shift(1,3) n=3000")
    want, nb = _hop(d)
    print("[case] max_levels=3, closure on", flush=True)
    out, r = dfamin.dfamin_minimize(ctx, d, dict(closure="on", max_levels=3))
    _, _, rr = oracle.moore_closure(d.n, d.k, d.delta, d.accept, L=3)
    assert np.array_equal(out, want) and r["num_blocks"] == nb
    assert r["closure_levels"] == 3 and r["refine_rounds"] == rr
    c = W.chain_dfa(3000, 2)
    print("[case] max_levels=3, AUTO on a chain", flush=True)
    out, r = dfamin.dfamin_minimize(ctx, c, dict(closure="auto", max_levels=3))
    assert np.array_equal(out, np.arange(c.n))
    # doubling with t = 2^min(floor(log2(j+1)), 3): P_j for j = 0, 1, 3, 7, 15, 23, ...
    j = r_want = 0
    while j < c.n - 2:
        j += 2 ** min(oracle.floor_log2(j + 1), 3)
        r_want += 1
    assert r["refine_rounds"] == r_want and r["closure_levels"] == 3


@pytest.mark.parametrize("auto_rounds", [0, 3, 5])
def test_auto_rounds_before_the_closure(ctx, auto_rounds):
    """A deep instance with two non-identity letters under AUTO: plain rounds
    until auto_rounds (0 = the default, 8), then the closure's letters from
    that partition on.  r* = A + Moore's refining rounds on the closure
    automaton started from P_A."""
    from paper_2410_22764_amd import dfamin
    d = shift_dfa(4000, [1, 2], "shift(1,2) n=4000")
    A = auto_rounds or 8
    print(f"[case] auto_rounds={auto_rounds}", flush=True)
    out, r = dfamin.dfamin_minimize(ctx, d, dict(closure="auto", auto_rounds=auto_rounds))
    want, nb = _hop(d)
    assert np.array_equal(out, want) and r["num_blocks"] == nb
    pa, _, ra = oracle.moore_partial(d.n, d.k, d.delta, d.accept, A)
    assert ra == A  # still refining after A rounds
    L = oracle.floor_log2(d.n)
    rows = oracle.closure(d.n, d.k, d.delta, L)
    _, _, rc = oracle.moore_from(d.n, rows.shape[0], rows.reshape(-1), pa)
    assert r["refine_rounds"] == A + rc
    assert r["closure_levels"] > 0


def test_hbm_budget_caps_the_closure_and_reports_nomem():
    """Closure storage is capped at half of a context's remaining budget.
    Over a range of budgets each call either fails with E_NOMEM or returns
    the oracle's partition with L' <= floor(log2 n) closure levels and
    exactly the rounds of Moore's refinement on the closure cut at L'.  Some
    budget must stop the closure early, a large one must build every level,
    and a budget below the base buffers must give E_NOMEM."""
    from paper_2410_22764_amd import dfamin
    d = shift_dfa(20000, [1, 7, 31, 127], "shift(1,7,31,127) n=20000")
    want, nb = _hop(d)
    L = oracle.floor_log2(d.n)
    rounds_at = {}
    seen = {"nomem": 0, "capped": 0, "full": 0}
    for mib in [64, 32, 16, 12, 10, 8, 7, 6, 5, 4, 3, 2, 1, 0.25]:
        budget = int(mib * (1 << 20))
        print(f"[case] closure on, budget {budget} bytes", flush=True)
        with dfamin.dfamin_create(0, budget) as c:
            out, r = dfamin.dfamin_minimize(c, d, "on", check=False)
        if r["rc"] == dfamin.DFAMIN_E_NOMEM:
            seen["nomem"] += 1
            continue
        assert r["rc"] == dfamin.DFAMIN_OK, (mib, r)
        assert np.array_equal(out, want) and r["num_blocks"] == nb, mib
        lv = r["closure_levels"]
        assert lv <= L
        if lv not in rounds_at:
            rounds_at[lv] = oracle.moore_closure(d.n, d.k, d.delta, d.accept, L=lv)[2]
        assert r["refine_rounds"] == rounds_at[lv], (mib, lv)
        seen["full" if lv == L else "capped"] += 1
    assert seen["full"] and seen["capped"] and seen["nomem"], seen


def test_bad_dfa_leaves_device_outputs_untouched(ctx):
    """E_BAD_DFA is found on the device before anything is written: a
    sentinel-filled output stays as it was, alone and in a batch (where no
    instance is minimized when one is bad)."""
    import torch
    from paper_2410_22764_amd import dfamin
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    for n, k in [(300, 2), (5000, 3), (70000, 2)]:
        d = W.random_dfa(n, k, n)
        delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
        delta[(k - 1) * n + n // 3] = n  # letter k-1, state n/3: out of range
        accept = torch.from_numpy(d.accept).to(dev)
        out = torch.full((n,), SENTINEL, dtype=torch.int32, device=dev)
        print(f"[case] bad DFA n={n} device entry", flush=True)
        r = dfamin.dfamin_minimize_device(ctx, n, k, delta.data_ptr(), accept.data_ptr(), 0, out.data_ptr(),
                                          stream=stream, check=False)
        torch.cuda.synchronize()
        assert r["rc"] == dfamin.DFAMIN_E_BAD_DFA
        assert bool((out == SENTINEL).all())
    good = [W.random_dfa(n, 2, n + 1) for n in (100, 4000, 30000)]
    bad = W.random_dfa(2000, 3, 9)
    bad.delta = bad.delta.copy()
    bad.delta[-1] = 2000
    ds = good[:2] + [bad] + good[2:]
    tens = [(torch.from_numpy(x.delta.view(np.int32)).to(dev), torch.from_numpy(x.accept).to(dev)) for x in ds]
    outs = [torch.full((x.n,), SENTINEL, dtype=torch.int32, device=dev) for x in ds]
    specs = [(x.n, x.k, t[0].data_ptr(), t[1].data_ptr(), x.q0) for x, t in zip(ds, tens)]
    print("[case] bad DFA in a device batch", flush=True)
    res = dfamin.dfamin_minimize_batch_device(ctx, specs, [o.data_ptr() for o in outs], stream=stream, check=False)
    torch.cuda.synchronize()
    assert res[0]["rc"] == dfamin.DFAMIN_E_BAD_DFA
    assert [r["status"] for r in res] == [0, 0, dfamin.DFAMIN_E_BAD_DFA, 0]
    for o in outs:
        assert bool((o == SENTINEL).all())
    # host entry point: the caller's buffer keeps its contents too
    h = np.full(bad.n, SENTINEL, np.uint32)
    s, keep = dfamin._host_dfa(bad)
    rr = dfamin.Result()
    rc = dfamin.load().dfamin_minimize(ctx.handle, dfamin.ctypes.byref(s), None, h.ctypes.data,
                                       dfamin.ctypes.byref(rr))
    assert rc == dfamin.DFAMIN_E_BAD_DFA and bool((h == SENTINEL).all())
