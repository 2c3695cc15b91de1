"""Serving (continuous batching) through dfamin_submit / dfamin_wait / dfamin_cancel.

Every result must be identical alone and in any mix (tolerance 0: the output
is an exact integer partition) and identical to the CPU oracle.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import oracle
from paper_2410_22764_amd import workloads as W

pytestmark = pytest.mark.gpu

EXPECTED = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "expected_workloads.json")))


def digest(out):
    return hashlib.sha256(np.ascontiguousarray(out, dtype="<u4").tobytes()).hexdigest()[:32]


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_22764_amd import dfamin
    c = dfamin.dfamin_create(0)
    yield c
    c.close()


def _mix(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(2 ** rng.uniform(4, 15))
        k = int(rng.integers(1, 7))
        kind = rng.choice(["random", "chain", "coarse"], p=[0.6, 0.2, 0.2])
        closure = ["off", "auto", "on"][i % 3]
        if kind == "chain":
            d = W.permuted_chain_dfa(n, k, seed * 1000 + i)
        else:
            d = W.random_dfa(n, k, seed * 1000 + i)
            if kind == "coarse":
                acc = np.zeros(n, bool)
                acc[:: 37] = True
                d.accept = W.pack_accept(acc)
        if kind == "chain" and closure == "off":
            closure = "auto"  # keep plain chain rounds bounded
        out.append((d, closure))
    return out


def test_mix_matches_alone_and_oracle(ctx):
    from paper_2410_22764_amd import dfamin
    reqs = _mix(1, 60)
    print("[case] serving mix of 60", flush=True)
    tickets = [dfamin.dfamin_submit(ctx, d, {"closure": c}) for d, c in reqs]
    for (d, c), t in zip(reqs, tickets):
        rc, out, res = dfamin.dfamin_wait(ctx, t, d.n, timeout_us=20_000_000)
        assert rc == dfamin.DFAMIN_OK, (d.name, rc)
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        assert res["num_blocks"] == nb and np.array_equal(out, want), d.name
        alone, ra = dfamin.dfamin_minimize(ctx, d, {"closure": c})
        assert np.array_equal(alone, out)
        assert ra["refine_rounds"] == res["refine_rounds"], d.name
        assert res["initial_block"] == want[d.q0]


def test_staggered_arrivals(ctx):
    """Requests submitted while others are resident join the running set."""
    from paper_2410_22764_amd import dfamin
    reqs = _mix(2, 40)
    print("[case] serving staggered", flush=True)
    tickets = []
    for i, (d, c) in enumerate(reqs):
        tickets.append(dfamin.dfamin_submit(ctx, d, {"closure": c}))
        if i % 5 == 0:
            time.sleep(0.002)
    for (d, c), t in zip(reqs, tickets):
        rc, out, res = dfamin.dfamin_wait(ctx, t, d.n)
        assert rc == dfamin.DFAMIN_OK
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        assert np.array_equal(out, want)


def test_short_request_overtakes_long_one(ctx):
    """Continuous batching: a short request that arrives after a long one
    finishes while the long one is still refining."""
    from paper_2410_22764_amd import dfamin
    long = W.chain_dfa(20000, 1)  # closure off: ~20000 rounds
    short = W.random_dfa(500, 2, 7)
    print("[case] serving overtake", flush=True)
    tl = dfamin.dfamin_submit(ctx, long, {"closure": "off"})
    time.sleep(0.01)
    ts = dfamin.dfamin_submit(ctx, short, None)
    rc, out, res = dfamin.dfamin_wait(ctx, ts, short.n, timeout_us=30_000_000)
    assert rc == dfamin.DFAMIN_OK
    rc_long, _, _ = dfamin.dfamin_wait(ctx, tl, long.n, timeout_us=0)
    assert rc_long == dfamin.DFAMIN_E_TIMEOUT  # still on the device
    rc_long, out_long, res_long = dfamin.dfamin_wait(ctx, tl, long.n)
    assert rc_long == dfamin.DFAMIN_OK
    assert np.array_equal(out_long, np.arange(long.n)) and res_long["refine_rounds"] == long.n - 2
    want, _ = oracle.hopcroft(short.n, short.k, short.delta, short.accept)
    assert np.array_equal(out, want)


def test_cancel_and_errors(ctx):
    from paper_2410_22764_amd import dfamin
    print("[case] serving cancel", flush=True)
    long = W.chain_dfa(20000, 1)
    t = dfamin.dfamin_submit(ctx, long, {"closure": "off"})
    time.sleep(0.01)
    assert dfamin.dfamin_cancel(ctx, t) == dfamin.DFAMIN_OK
    rc, out, _ = dfamin.dfamin_wait(ctx, t, long.n)
    assert rc == dfamin.DFAMIN_E_CANCELLED and out is None
    assert dfamin.dfamin_cancel(ctx, 10 ** 12) == dfamin.DFAMIN_E_INVAL
    bad = W.random_dfa(100, 2, 1)
    bad.delta = bad.delta.copy()
    bad.delta[3] = 100
    t = dfamin.dfamin_submit(ctx, bad, None)
    rc, _, _ = dfamin.dfamin_wait(ctx, t, bad.n)
    assert rc == dfamin.DFAMIN_E_BAD_DFA
    # the loop keeps serving afterwards
    d = W.random_dfa(300, 3, 2)
    t = dfamin.dfamin_submit(ctx, d, None)
    rc, out, _ = dfamin.dfamin_wait(ctx, t, d.n)
    want, _ = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
    assert rc == dfamin.DFAMIN_OK and np.array_equal(out, want)


def test_pageable_staging_when_pinned_cap_is_zero(monkeypatch):
    """With the page-locked staging pool capped at 0 bytes every request is
    staged in ordinary host memory; results are unchanged."""
    from paper_2410_22764_amd import dfamin
    monkeypatch.setenv("DFAMIN_SERVING_PINNED_BYTES", "0")
    c = dfamin.dfamin_create(0)
    try:
        reqs = _mix(7, 12)
        print("[case] serving mix of 12, pageable staging", flush=True)
        tickets = [dfamin.dfamin_submit(c, d, {"closure": cl}) for d, cl in reqs]
        for (d, cl), t in zip(reqs, tickets):
            rc, out, res = dfamin.dfamin_wait(c, t, d.n, timeout_us=20_000_000)
            assert rc == dfamin.DFAMIN_OK, (d.name, rc)
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert res["num_blocks"] == nb and np.array_equal(out, want), d.name
    finally:
        c.close()


def test_serving_pool_at_full_sizes_bit_exact(ctx):
    """Requests of the serving workload at its own sizes (n up to 2^22,
    |Sigma| up to 16, permuted chains of over 2^20 states among them), all
    submitted at once so that they share the device: every result equals
    the oracle's (digest, block count, initial block, written by the golden
    script with the CPU oracle only) and the same DFA minimised alone."""
    from paper_2410_22764_amd import dfamin
    exp = EXPECTED["serving_pool"]
    _, specs = W.serving_stream(exp["seed"], exp["draws"], 1.0)
    reqs = exp["requests"]
    assert any(e["n"] >= 1 << 20 and e["k"] == 16 for e in reqs)
    assert any(e["kind"] == "chain" and e["n"] >= 1 << 20 for e in reqs)
    print(f"[case] serving pool of {len(reqs)} at full sizes: generating", flush=True)
    pool = [W.make_request(specs[e["index"]]) for e in reqs]
    print("[case] serving pool: submitting all", flush=True)
    tickets = [dfamin.dfamin_submit(ctx, d, "auto") for d in pool]
    mixed = []
    for d, e, t in zip(pool, reqs, tickets):
        assert (d.n, d.k) == (e["n"], e["k"])
        rc, out, res = dfamin.dfamin_wait(ctx, t, d.n, timeout_us=60_000_000)
        assert rc == dfamin.DFAMIN_OK, (e, rc)
        assert res["num_blocks"] == e["num_blocks"] and res["initial_block"] == e["initial_block"], e
        assert digest(out) == e["sha"], e
        mixed.append((digest(out), res["refine_rounds"]))
    print("[case] serving pool: each request alone", flush=True)
    for d, e, (dg, rr) in zip(pool, reqs, mixed):
        alone, ra = dfamin.dfamin_minimize(ctx, d, "auto")
        assert digest(alone) == dg and ra["refine_rounds"] == rr, e


def test_doubling_requests_report_as_alone(ctx):
    """Chains under AUTO refine by doubling, in the fused kernel (up to
    16,384 states) or in the resident set: each request's round count and
    closure levels (the highest level a splitting round read) are those of
    the same DFA minimised alone."""
    from paper_2410_22764_amd import dfamin
    ds = [W.permuted_chain_dfa(n, k, n + k) for n, k in [(3, 2), (900, 2), (16384, 3), (16385, 2), (70000, 4)]]
    ds.append(W.random_dfa(3000, 1, 5))
    print("[case] serving doubling requests", flush=True)
    tickets = [dfamin.dfamin_submit(ctx, d, "auto") for d in ds]
    for d, t in zip(ds, tickets):
        rc, out, res = dfamin.dfamin_wait(ctx, t, d.n, timeout_us=20_000_000)
        assert rc == dfamin.DFAMIN_OK, d.name
        alone, ra = dfamin.dfamin_minimize(ctx, d, "auto")
        assert np.array_equal(alone, out), d.name
        for f in ("num_blocks", "initial_block", "refine_rounds", "rounds_executed", "closure_levels",
                  "closure_letters"):
            assert res[f] == ra[f], (d.name, f, res, ra)


def _double_step_chain(n, seed):
    """A chain on which both letters move forward (one or two states): two
    non-identity letters, about n/2 plain rounds, so AUTO gives it the
    closure after its first rounds."""
    ids = np.arange(n, dtype=np.uint32)
    rows = np.stack([np.minimum(ids + 1, n - 1), np.minimum(ids + 2, n - 1)])
    acc = np.zeros(n, bool)
    acc[n - 1] = True
    d = W.from_rows(rows, acc, 0, f"double-step chain(n={n})")
    return W.permute_dfa(d, W.random_permutation(n, seed), f"double-step chain(n={n},seed={seed})")


def test_small_budget_deep_auto_requests():
    """A context whose HBM budget leaves the serving loop a few MB: deep
    requests with two non-identity letters under AUTO all come due for the
    closure at once, and a unary chain refines by doubling beside them.
    Level storage runs short (a closure then keeps the levels it has), and a
    request whose signature records for the new letter count do not fit
    keeps refining on its plain letters: every request still ends with the
    oracle's partition, none fails."""
    from paper_2410_22764_amd import dfamin
    c = dfamin.dfamin_create(0, hbm_budget_bytes=8 << 20)
    try:
        ds = [_double_step_chain(6000, 31 + i) for i in range(10)]
        ds.append(W.permuted_chain_dfa(6000, 2, 41))
        print(f"[case] serving {len(ds)} deep requests under an 8 MB budget", flush=True)
        tickets = [dfamin.dfamin_submit(c, d, "auto") for d in ds]
        for d, t in zip(ds, tickets):
            rc, out, res = dfamin.dfamin_wait(c, t, d.n, timeout_us=60_000_000)
            assert rc == dfamin.DFAMIN_OK, (d.name, rc)
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert res["num_blocks"] == nb and np.array_equal(out, want) and res["initial_block"] == want[d.q0]
    finally:
        c.close()


def test_small_request_batches_beside_rounds(ctx):
    """Small requests run as fused batches on their own stream while the
    resident set refines: a burst of them around a long request, every
    fourth cancelled right after its submit, one invalid and one that the
    fused kernel hands back (two non-identity letters, still splitting after
    the AUTO rounds), which then joins the resident set and takes closure
    letters.  Each result is the oracle's, a cancelled request reports
    success or cancellation, the invalid one E_BAD_DFA."""
    from paper_2410_22764_amd import dfamin
    print("[case] serving: small-request batches beside a long request", flush=True)
    long = W.chain_dfa(3000, 1)
    tl = dfamin.dfamin_submit(ctx, long, {"closure": "off"})  # one round per state
    small = [W.random_dfa(200 + 300 * i, 2 + i % 5, 100 + i) for i in range(48)]
    n = 3000
    ids = np.arange(n)
    rows = np.stack([np.minimum(ids + 1, n - 1), np.minimum(ids + 2, n - 1)])
    acc = np.zeros(n, bool)
    acc[-1] = True
    deep = W.from_rows(rows, acc, 0, "two-letter chain")
    bad = W.random_dfa(500, 2, 7)
    bad.delta = bad.delta.copy()
    bad.delta[10] = 500
    tickets, cancelled = [], set()
    for i, d in enumerate(small):
        t = dfamin.dfamin_submit(ctx, d, {"closure": "auto"})
        tickets.append(t)
        if i % 4 == 1:
            assert dfamin.dfamin_cancel(ctx, t) == dfamin.DFAMIN_OK
            cancelled.add(i)
    td = dfamin.dfamin_submit(ctx, deep, {"closure": "auto"})
    tb = dfamin.dfamin_submit(ctx, bad, {"closure": "auto"})
    for i, (d, t) in enumerate(zip(small, tickets)):
        rc, out, res = dfamin.dfamin_wait(ctx, t, d.n, timeout_us=30_000_000)
        if i in cancelled and rc == dfamin.DFAMIN_E_CANCELLED:
            continue
        assert rc == dfamin.DFAMIN_OK, (i, rc)
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        assert res["num_blocks"] == nb and np.array_equal(out, want), i
    rc, out, res = dfamin.dfamin_wait(ctx, td, deep.n, timeout_us=30_000_000)
    want, nb = oracle.hopcroft(deep.n, deep.k, deep.delta, deep.accept)
    assert rc == dfamin.DFAMIN_OK and res["num_blocks"] == nb and np.array_equal(out, want)
    assert res["closure_levels"] > 0  # handed back by the fused kernel, closure built by the loop
    rc, _, _ = dfamin.dfamin_wait(ctx, tb, bad.n, timeout_us=30_000_000)
    assert rc == dfamin.DFAMIN_E_BAD_DFA
    rc, out, res = dfamin.dfamin_wait(ctx, tl, long.n, timeout_us=60_000_000)
    assert rc == dfamin.DFAMIN_OK and np.array_equal(out, np.arange(long.n))
