"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Every comparison is exact (integer output, canonical numbering).  Sizes span
several workgroup tiles (256 states per signature workgroup, 1024 per scan
tile) and ragged tails.
"""
import math

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


@pytest.fixture(autouse=True, params=["fused", "rounds"])
def engine_path(request, monkeypatch):
    """Every test here runs twice: instances of up to 16,384 states through
    the fused one-workgroup kernels (the default), and every instance
    through the round engine."""
    if request.param == "rounds":
        monkeypatch.setenv("DFAMIN_FUSED_MAX_STATES", "0")
    return request.param


def _run(ctx, d, closure="off", **kw):
    from paper_2410_22764_amd import dfamin
    print(f"[case] {d.name} n={d.n} k={d.k} closure={closure}", flush=True)
    return dfamin.dfamin_minimize(ctx, d, dict(closure=closure, **kw))


def _check(ctx, d, closure="off", rounds=None, **kw):
    out, res = _run(ctx, d, closure, **kw)
    want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
    assert res["num_blocks"] == nb
    assert np.array_equal(out, want)
    assert res["initial_block"] == want[d.q0]
    if rounds is not None:
        assert res["refine_rounds"] == rounds
    assert res["rounds_executed"] == res["refine_rounds"] + 1
    return out, res


SIZES = [1, 2, 7, 63, 255, 256, 257, 1000, 1023, 1024, 1025, 4097, 65537]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_random_dfas_match_hopcroft_and_moore_rounds(ctx, n, k):
    d = W.random_dfa(n, k, seed=n * 31 + k)
    _, _, mr = oracle.moore(d.n, d.k, d.delta, d.accept)
    _check(ctx, d, rounds=mr)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_plain_single_workload(ctx, seed):
    d = W.plain_single(seed)
    _, _, mr = oracle.moore(d.n, d.k, d.delta, d.accept)
    _check(ctx, d, rounds=mr)


@pytest.mark.parametrize("seed", range(6))
def test_coarse_partitions(ctx, seed):
    """Few accepting states and small alphabets: big classes, skewed groups."""
    n = [300, 5000, 20000, 70000, 1000, 123457][seed]
    d = W.random_dfa(n, 1 + seed % 3, seed)
    acc = np.zeros(n, bool)
    acc[np.arange(0, n, 97)] = True
    d.accept = W.pack_accept(acc)
    _, _, mr = oracle.moore(d.n, d.k, d.delta, d.accept)
    out, res = _check(ctx, d, rounds=mr)


@pytest.mark.parametrize("closure", ["off", "on", "auto"])
def test_closure_modes_identical(ctx, closure):
    for seed in range(4):
        d = W.random_dfa(3000 + seed, 2, seed)
        _check(ctx, d, closure)
        c = W.permuted_chain_dfa(777 + seed, 3, seed)
        out, res = _check(ctx, c, closure)
        assert np.array_equal(out, np.arange(c.n))


def test_closure_round_count_matches_oracle(ctx):
    for d in [W.chain_dfa(1000, 2), W.permuted_chain_dfa(600, 2, 9), W.fib_dfa(12), W.random_dfa(500, 2, 4)]:
        _, _, rr = oracle.moore_closure(d.n, d.k, d.delta, d.accept)
        _, res = _check(ctx, d, "on", rounds=rr)
        assert res["closure_levels"] == oracle.floor_log2(d.n)


def test_figure1_chain(ctx):
    d = W.chain_dfa(10, 1)
    _check(ctx, d, "off", rounds=8)
    _check(ctx, d, "on", rounds=3)


def test_deep_chain_workload_closed_form(ctx):
    """Chain with n = 2^20: every state is its own class; 19 refining rounds
    with the closure (largest popcount of a distance below 2^20 - 1)."""
    d = W.deep_chain()
    out, res = _run(ctx, d, "on")
    assert res["num_blocks"] == d.n
    assert np.array_equal(out, np.arange(d.n))
    assert res["refine_rounds"] == 19 and res["rounds_executed"] == 20
    assert res["closure_levels"] == 20
    assert res["closure_letters"] == 21  # the identity letter is dropped


def test_deep_chain_auto(ctx):
    """AUTO on the 2^20 chain (one non-identity letter): doubling from the
    first round, t = 1, 2, 4, ..., 2^19, holds P_(2^r - 1) after r rounds and
    reaches P_(2^20 - 1), the first partition with every state alone (it
    needs j >= n - 2), after ceil(log2(n - 1)) = 20 refining rounds.  The
    rounds read levels 0..19, each computed in the round that first reads
    it, so 19 levels are built (no state is left to refine after the last
    split)."""
    d = W.deep_chain()
    out, res = _run(ctx, d, "auto")
    assert res["num_blocks"] == d.n and np.array_equal(out, np.arange(d.n))
    assert res["closure_levels"] == 19 and res["closure_letters"] == 20
    assert res["refine_rounds"] == 20 and res["rounds_executed"] == 21


def _kept_levels(d, a):
    """Closure levels kept for letter a: level 0, then every level that
    differs from its predecessor and is not the identity, up to the first
    that fails that test."""
    L = oracle.floor_log2(d.n)
    rows = oracle.closure(d.n, d.k, d.delta, L)
    ident = np.arange(d.n, dtype=np.uint32)
    kept = 1
    for lv in range(1, L + 1):
        cur, prev = rows[a * (L + 1) + lv], rows[a * (L + 1) + lv - 1]
        if np.array_equal(cur, prev) or np.array_equal(cur, ident):
            break
        kept += 1
    return kept


def _auto_unary_rounds(d, auto_rounds=0):
    """Refining rounds of AUTO on a unary instance, from Moore's partitions
    P_j alone: plain rounds (j -> j + 1) until auto_rounds (none: a unary
    instance doubles from its first round), then j -> j + t with t the
    largest kept level 2^l <= j + 1; stop at the first step that leaves the
    block count unchanged."""
    rows = d.rows()
    letters = [a for a in range(d.k) if not np.array_equal(rows[a], np.arange(d.n))]
    assert len(letters) == 1
    kept = _kept_levels(d, letters[0])
    prev = oracle.moore_partial(d.n, d.k, d.delta, d.accept, 0)[1]
    j = r = 0
    while True:
        t = 1
        if r >= auto_rounds:
            t = 2 ** min(oracle.floor_log2(j + 1), kept - 1)
        c = oracle.moore_partial(d.n, d.k, d.delta, d.accept, j + t)[1]
        if c == prev:
            return r
        prev, j, r = c, j + t, r + 1


@pytest.mark.parametrize("which", range(6))
def test_auto_doubling_rounds(ctx, which):
    """Unary instances under AUTO refine by doubling after the plain rounds:
    same partition as the oracle, round count as derived from P_j."""
    d = [W.chain_dfa(1000, 2), W.permuted_chain_dfa(1500, 3, 5), W.fib_dfa(14),
         W.random_dfa(1200, 1, 3), W.chain_dfa(9, 1), W.fib_dfa_word(9)][which]
    _check(ctx, d, "auto", rounds=_auto_unary_rounds(d))


@pytest.mark.parametrize("m", [8, 10, 14, 18])
def test_fib_family(ctx, m):
    d = W.fib_dfa(m)
    out, res = _check(ctx, d, "auto")
    assert res["num_blocks"] == d.n
    if d.n < 2000:
        _check(ctx, d, "off", rounds=d.n - 2)


@pytest.mark.parametrize("m", [3, 6, 10, 15])
def test_bitsplitter_family(ctx, m):
    d = W.bitsplitter_dfa(m)
    out, res = _check(ctx, d, "off", rounds=m - 1)
    assert res["num_blocks"] == 2 ** m


def test_degenerate_inputs(ctx):
    for n in [1, 2, 300, 5000]:
        for acc in (np.zeros(n, bool), np.ones(n, bool)):
            d = W.random_dfa(n, 2, n)
            d.accept = W.pack_accept(acc)
            out, res = _check(ctx, d, rounds=0)
            assert res["num_blocks"] == 1 and not out.any()
    # all letters the identity
    d = W.from_rows(np.tile(np.arange(100, dtype=np.uint32), (3, 1)), np.arange(100) % 3 == 0)
    _check(ctx, d, rounds=0)
    # duplicate letters
    base = W.random_dfa(999, 2, 3)
    rows = np.vstack([base.rows(), base.rows()[1], base.rows()[0]])
    d = W.from_rows(rows, base.accept_bool())
    out, res = _check(ctx, d)
    out2, _ = _check(ctx, base)
    assert np.array_equal(out, out2)


def test_bad_transition_rejected_output_untouched(ctx):
    from paper_2410_22764_amd import dfamin
    d = W.random_dfa(5000, 3, 1)
    d.delta = d.delta.copy()
    d.delta[2 * 5000 + 4321] = 5000
    out, res = dfamin.dfamin_minimize(ctx, d, None, check=False)
    assert res["rc"] == dfamin.DFAMIN_E_BAD_DFA
    # the context still works afterwards
    _check(ctx, W.random_dfa(100, 2, 2))


def test_invalid_arguments(ctx):
    from paper_2410_22764_amd import dfamin
    d = W.random_dfa(10, 2, 1)
    d.q0 = 10
    _, res = dfamin.dfamin_minimize(ctx, d, None, check=False)
    assert res["rc"] == dfamin.DFAMIN_E_INVAL
    d.q0 = 0
    _, res = dfamin.dfamin_minimize(ctx, d, {"closure": 7}, check=False)
    assert res["rc"] == dfamin.DFAMIN_E_INVAL


def test_round_cap(ctx):
    from paper_2410_22764_amd import dfamin
    d = W.chain_dfa(50, 1)
    _, res = dfamin.dfamin_minimize(ctx, d, dict(closure="off", max_rounds=10), check=False)
    assert res["rc"] == dfamin.DFAMIN_E_INTERNAL


def test_deterministic_repeats(ctx):
    d = W.random_dfa(200000, 3, 11)
    a, ra = _run(ctx, d)
    for _ in range(3):
        b, rb = _run(ctx, d)
        assert np.array_equal(a, b) and ra == rb


def test_batch_matches_solo_and_oracle(ctx):
    from paper_2410_22764_amd import dfamin
    dfas = W.batch_mixed(seed=3, count=96, n_min=16, n_max=5000)
    dfas.append(W.random_dfa(1, 2, 0))
    dfas.append(W.chain_dfa(64, 1))
    for closure in ["off", "auto", "on"]:
        print(f"[case] batch closure={closure}", flush=True)
        outs, results = dfamin.dfamin_minimize_batch(ctx, dfas, dict(closure=closure))
        for d, o, r in zip(dfas, outs, results):
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert r["num_blocks"] == nb and np.array_equal(o, want), d.name
            solo, rs = dfamin.dfamin_minimize(ctx, d, dict(closure=closure))
            assert np.array_equal(solo, o)
            assert rs["refine_rounds"] == r["refine_rounds"]


def test_batch_bad_instance(ctx):
    from paper_2410_22764_amd import dfamin
    dfas = [W.random_dfa(100, 2, i) for i in range(5)]
    dfas[3].delta = dfas[3].delta.copy()
    dfas[3].delta[7] = 1000
    outs, results = dfamin.dfamin_minimize_batch(ctx, dfas, None, check=False)
    assert results[0]["rc"] == dfamin.DFAMIN_E_BAD_DFA
    assert [r["status"] for r in results] == [0, 0, 0, dfamin.DFAMIN_E_BAD_DFA, 0]


def test_device_entry_point_with_torch_buffers(ctx):
    import torch
    from paper_2410_22764_amd import dfamin
    d = W.random_dfa(123457, 4, 5)
    dev = torch.device("cuda:0")
    delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
    accept = torch.from_numpy(d.accept).to(dev)
    out = torch.full((d.n,), -1, dtype=torch.int32, device=dev)
    res = dfamin.dfamin_minimize_device(ctx, d.n, d.k, delta.data_ptr(), accept.data_ptr(), d.q0,
                                        out.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
    got = out.cpu().numpy().view(np.uint32)
    want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
    assert res["num_blocks"] == nb and np.array_equal(got, want)


@pytest.mark.parametrize("variant", [0, 1, 2, -1])
def test_signature_tile_variants_identical(ctx, variant):
    """Every signature tile (256, 512, 1024 states per workgroup) and the
    autotuned choice give the oracle's partition; sizes straddle each tile
    and the tuning threshold (2^18 active states)."""
    from paper_2410_22764_amd import dfamin
    dfamin.dfamin_set_tuning(ctx, variant)
    try:
        for n, k in [(1, 2), (255, 2), (257, 3), (1023, 1), (1025, 4), (70001, 2), (300007, 3)]:
            _check(ctx, W.random_dfa(n, k, seed=n + variant))
        _check(ctx, W.permuted_chain_dfa(300000, 2, 4), "auto")
        dfas = W.batch_mixed(seed=5, count=40, n_min=16, n_max=20000)
        outs, results = dfamin.dfamin_minimize_batch(ctx, dfas, {"closure": "auto"})
        for d, o, r in zip(dfas, outs, results):
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert r["num_blocks"] == nb and np.array_equal(o, want), d.name
    finally:
        dfamin.dfamin_set_tuning(ctx, -1)


def _hash_mode_cases():
    """Inputs whose later rounds group every instance by hash (queued rounds)."""
    return [W.random_dfa(3000, 3, 21), W.random_dfa(2500, 4, 22), W.bitsplitter_dfa(9),
            W.permuted_chain_dfa(1500, 2, 23), W.fib_dfa(13)]


def test_queued_rounds_graph_direct_and_planned_agree(ctx):
    """With the queue flag, once every instance groups by hash the rounds are
    queued on the device.  Replayed from a captured graph (several calls,
    other work in between), launched one by one (no-graph flag), and planned
    by the host round by round (profiling on), they give the oracle's
    partition and the same round counts."""
    from paper_2410_22764_amd import dfamin
    cases = [(d, "on" if d.name.lower().startswith(("permuted_chain", "fib")) else "off")
             for d in _hash_mode_cases()]
    for d, closure in cases:
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        print(f"[case] queued rounds {d.name} closure={closure}", flush=True)
        dfamin.dfamin_set_profiling(ctx, True)
        planned, rp = dfamin.dfamin_minimize(ctx, d, dict(closure=closure))
        dfamin.dfamin_set_profiling(ctx, False)
        assert rp["num_blocks"] == nb and np.array_equal(planned, want), d.name
        direct, rd = dfamin.dfamin_minimize(ctx, d, dict(closure=closure, queue=True, no_graph=True))
        assert np.array_equal(direct, want) and rd == rp, d.name
        for rep in range(3):
            out, r = dfamin.dfamin_minimize(ctx, d, dict(closure=closure, queue=True))
            assert np.array_equal(out, want) and r == rp, (d.name, rep)
            other = W.random_dfa(777 + rep, 2, rep)  # other work between the replays
            o2, _ = dfamin.dfamin_minimize(ctx, other, "off")
            assert np.array_equal(o2, oracle.hopcroft(other.n, other.k, other.delta, other.accept)[0])


def test_weak_hash_collisions_are_redone(ctx, monkeypatch):
    """With signature hashes cut to 16 bits of entropy (a testing knob),
    different signatures of a round share a hash now and then: the full
    comparison in resolve catches every such case and the round is redone
    with another salt.  Rounds planned by the host (profiling on) show the
    redone rounds as extra signature launches; queued rounds redo them on the
    device.  Partitions and round counts stay exact either way.  Cut to 12
    bits, every salt collides: the call fails with E_INTERNAL after the
    bounded retries, in both modes, and the context stays usable."""
    from paper_2410_22764_amd import dfamin
    cases = [(W.bitsplitter_dfa(9), "off"), (W.permuted_chain_dfa(1500, 2, 23), "on")]

    def profiled(d, closure):
        dfamin.dfamin_set_profiling(ctx, True)
        out, r = dfamin.dfamin_minimize(ctx, d, dict(closure=closure), check=False)
        stats = {s["name"]: s["launches"] for s in dfamin.dfamin_get_kernel_stats(ctx)}
        dfamin.dfamin_set_profiling(ctx, False)
        return out, r, stats.get("signature", 0)

    strong = {d.name: profiled(d, closure) for d, closure in cases}
    monkeypatch.setenv("DFAMIN_HASH_BITS", "16")
    for d, closure in cases:
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        print(f"[case] weak hash {d.name} closure={closure}", flush=True)
        _, rs, ls = strong[d.name]
        out, r, lw = profiled(d, closure)
        assert r["rc"] == 0 and np.array_equal(out, want) and r == rs, d.name
        assert lw > ls, d.name  # rounds were redone
        out, r = dfamin.dfamin_minimize(ctx, d, dict(closure=closure, queue=True))
        assert np.array_equal(out, want) and r == rs, d.name
    monkeypatch.setenv("DFAMIN_HASH_BITS", "12")
    for d, closure in cases:
        print(f"[case] hopeless hash {d.name} closure={closure}", flush=True)
        _, r, _ = profiled(d, closure)
        assert r["rc"] == dfamin.DFAMIN_E_INTERNAL, d.name
        _, r = dfamin.dfamin_minimize(ctx, d, dict(closure=closure, queue=True), check=False)
        assert r["rc"] == dfamin.DFAMIN_E_INTERNAL, d.name
    monkeypatch.delenv("DFAMIN_HASH_BITS")
    d, closure = cases[1]
    out, r = dfamin.dfamin_minimize(ctx, d, dict(closure=closure))
    assert np.array_equal(out, oracle.hopcroft(d.n, d.k, d.delta, d.accept)[0]) and r == strong[d.name][1]


def test_first_round_redo_keeps_doubling_levels(ctx, monkeypatch):
    """A hash collision in the first round redoes it for the whole batch.
    The one-letter AUTO instances, which refine by doubling from that round,
    keep their level storage and the level already built for the next round
    (queued while the host waits).  A 40-letter instance groups by hash from
    the first round (41 key components do not fit 31 bits); with hashes cut
    to 16 bits of entropy (a testing knob), its 250 states collide in about a
    third of all attempts.  Every batch that finishes matches the oracle; one
    whose retries all collide fails with E_INTERNAL and is skipped."""
    from paper_2410_22764_amd import dfamin
    monkeypatch.setenv("DFAMIN_HASH_BITS", "16")
    finished = 0
    for seed in range(6):
        ds = [W.random_dfa(250, 40, 100 + seed), W.random_dfa(3000, 1, 200 + seed),
              W.permuted_chain_dfa(2000, 1, 300 + seed)]
        print(f"[case] first-round redo seed={seed}", flush=True)
        outs, res = dfamin.dfamin_minimize_batch(ctx, ds, dict(closure="auto"), check=False)
        if res[0]["rc"] == dfamin.DFAMIN_E_INTERNAL:
            continue
        finished += 1
        for d, o, r in zip(ds, outs, res):
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert r["rc"] == 0 and r["num_blocks"] == nb and np.array_equal(o, want), (seed, d.name)
    monkeypatch.delenv("DFAMIN_HASH_BITS")
    assert finished >= 3


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_table_insertion_orders_agree(ctx, monkeypatch, order):
    """A signature group joins the global table either by reading its home
    slot first or by a CAS straight away, chosen per round and key mode.
    Forcing each combination (a testing knob: bit 0 hash-mode keys, bit 1
    exact keys) changes no partition and no round count, alone or batched."""
    from paper_2410_22764_amd import dfamin
    monkeypatch.setenv("DFAMIN_CAS_FIRST", str(order))
    cases = [W.random_dfa(20000, 3, 7), W.permuted_chain_dfa(3000, 1, 3), W.random_dfa(5000, 1, 2),
             W.fib_dfa(12)]
    for d in cases:
        want, nb, rounds = oracle.moore(d.n, d.k, d.delta, d.accept)
        print(f"[case] insertion order {order} {d.name}", flush=True)
        out, r = dfamin.dfamin_minimize(ctx, d, "off")
        assert r["num_blocks"] == nb and np.array_equal(out, want) and r["refine_rounds"] == rounds, d.name
        out, r = dfamin.dfamin_minimize(ctx, d, "auto")
        assert r["num_blocks"] == nb and np.array_equal(out, want), d.name
    outs, res = dfamin.dfamin_minimize_batch(ctx, cases, "auto")
    for d, o, r in zip(cases, outs, res):
        assert np.array_equal(o, oracle.hopcroft(d.n, d.k, d.delta, d.accept)[0]), d.name


def test_first_round_labels_and_table_agree(ctx, monkeypatch):
    """From {F, Q\\F}, with at most 8 signature letters, the first round
    labels every state by its own accept bit and those of its successors
    (an exact key below 256, or 512 with 8 letters, stored in two bytes)
    instead of grouping through the hash table.
    One instance's exact-key round that a hash round follows leaves slot
    labels for the states of shared groups instead of least members, with
    no resolve step, and both rounds decide whether they split by counting
    groups; where the key space allows, that round groups in a direct count
    table.  A testing knob turns these off (bit 0: first-round labels, bit
    1: slot labels, bit 2: direct tables).  Every setting gives the oracle's partition and the
    same round counts and closure levels, alone and batched.  The batch
    holds instances whose first round splits nothing (F empty, F = Q, no
    non-identity letter), which leave it after that round, and 1- and
    7-letter instances (labels of 2 and 8 bits); it runs as it is, with an
    8-letter instance (9-bit labels for the whole batch, whose 7-letter
    instance then reads two-byte dense numbers in its exact second round)
    and with a 9-letter one (the whole batch through the table)."""
    from paper_2410_22764_amd import dfamin
    empty = W.random_dfa(40000, 3, 11)
    empty.accept = W.pack_accept(np.zeros(empty.n, bool))
    full = W.random_dfa(30000, 2, 12)
    full.accept = W.pack_accept(np.ones(full.n, bool))
    ident = W.from_rows(np.stack([np.arange(20000, dtype=np.uint32)] * 2),
                        np.arange(20000) % 3 == 0, name="identity-letters")
    # (8,192 and 12,000 states over 3 letters: a second round in a count
    # table where most groups have one state, so the compaction reads the
    # counts of lone claimers; 65,536 over 4: keys too wide for a count table)
    cases = [W.random_dfa(20000, 3, 7), W.random_dfa(70000, 7, 3), W.random_dfa(5000, 1, 2),
             W.permuted_chain_dfa(30000, 1, 3), W.chain_dfa(20000, 2), W.fib_dfa(14), empty, full, ident,
             W.random_dfa(1, 1, 1), W.random_dfa(8192, 3, 17), W.random_dfa(12000, 3, 18),
             W.random_dfa(65536, 4, 19), W.random_dfa(40000, 8, 23)]
    fields = ("num_blocks", "initial_block", "refine_rounds", "closure_levels", "closure_letters")
    for closure in ("off", "auto"):
        labelled = {}
        for d in cases:
            if closure == "off" and d.name.startswith("chain"):
                continue  # one state per round: too many rounds to spend here
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            print(f"[case] first round by labels {d.name} closure={closure}", flush=True)
            out, r = dfamin.dfamin_minimize(ctx, d, closure)
            assert r["num_blocks"] == nb and np.array_equal(out, want), d.name
            labelled[d.name] = r
        for knob in ("1", "2", "3", "4"):
            monkeypatch.setenv("DFAMIN_NO_LABELS", knob)
            for d in cases:
                if d.name not in labelled:
                    continue
                print(f"[case] labels off ({knob}) {d.name} closure={closure}", flush=True)
                out, r = dfamin.dfamin_minimize(ctx, d, closure)
                assert np.array_equal(out, oracle.hopcroft(d.n, d.k, d.delta, d.accept)[0]), (knob, d.name)
                assert all(r[f] == labelled[d.name][f] for f in fields), (knob, d.name, r, labelled[d.name])
        monkeypatch.delenv("DFAMIN_NO_LABELS")
    batch = [c for c in cases if not c.name.startswith("chain") and c.k != 8]
    for extra in ([], [W.random_dfa(30000, 8, 5)], [W.random_dfa(30000, 9, 5)]):
        print(f"[case] first round by labels, batch of {len(batch) + len(extra)}", flush=True)
        outs, res = dfamin.dfamin_minimize_batch(ctx, batch + extra, "off")
        for d, o, r in zip(batch + extra, outs, res):
            want, nb, rounds = oracle.moore(d.n, d.k, d.delta, d.accept)
            assert r["num_blocks"] == nb and np.array_equal(o, want) and r["refine_rounds"] == rounds, d.name


def test_all_singleton_results_numbered_directly(ctx):
    """When one instance's rounds end with every block a singleton (a split
    round that keeps no state, or a count of n blocks), each state is its
    own class: out = 0..n-1 without a numbering scan.  Random and chain DFAs
    whose minimal DFA keeps every state, under both closure modes, and the
    minimal DFA built from such a result."""
    from paper_2410_22764_amd import dfamin
    cases = [(W.permuted_chain_dfa(40000, 2, 9), "auto"), (W.chain_dfa(3000, 1), "off"),
             (W.random_dfa(2, 1, 3), "off"), (W.random_dfa(100000, 4, 21), "off")]
    for d, closure in cases:
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        print(f"[case] all singletons {d.name} closure={closure} ({nb} of {d.n} blocks)", flush=True)
        out, r = dfamin.dfamin_minimize(ctx, d, closure)
        assert r["num_blocks"] == nb and np.array_equal(out, want) and r["initial_block"] == want[d.q0]
    d = cases[0][0]
    assert oracle.hopcroft(d.n, d.k, d.delta, d.accept)[1] == d.n
    m, dm, am, info, out = dfamin.dfamin_minimal_dfa(ctx, d, "auto")
    em, edm, eam, eq0, enr = oracle.minimal_dfa(d.n, d.k, d.delta, d.accept, d.q0)
    assert (m, info["q0"], info["reachable"]) == (em, eq0, enr)
    assert np.array_equal(dm, edm) and np.array_equal(am, eam) and np.array_equal(out, np.arange(d.n))


def test_validation_sees_every_row_entry(ctx):
    """The validation pass reads each δ row in 16-byte loads from its first
    16-byte boundary and the (up to three) entries before it one by one.
    Rows start misaligned when n is not a multiple of 4.  A single bad
    transition, or a single non-identity entry, placed at each of the first
    entries, just after the boundary, and at the row's end, must be seen:
    the bad one as E_BAD_DFA, the non-identity one by the partition (letters
    0 and 2 are the identity and only state n-1 accepts, so letter 1 sending
    p to n-1 is the only thing that separates p from states 0..n-2)."""
    from paper_2410_22764_amd import dfamin
    for n in (5, 6, 7, 4097, 8191, 8194):
        ids = np.arange(n, dtype=np.uint32)
        acc = np.zeros(n, bool)
        acc[n - 1] = True
        for p in sorted({0, 1, 2, 3, 4, 5, n // 2, n - 3, n - 2} & set(range(n - 1))):
            rows = np.stack([ids, ids.copy(), ids])
            rows[1][p] = n - 1
            d = W.from_rows(rows, acc, name=f"identity-but-{p} n={n}")
            bad = W.from_rows(np.stack([ids, ids, ids]), acc, name=f"bad-{p} n={n}")
            bad.delta[n + p] = n  # letter 1, state p: out of range
            print(f"[case] validation n={n} p={p}", flush=True)
            # a batch puts every instance at a 16-byte aligned offset, so the
            # rows of letters 1 and 2 start misaligned when n % 4 != 0
            outs, res = dfamin.dfamin_minimize_batch(ctx, [W.random_dfa(3, 2, 1), d], None)
            want = oracle.hopcroft(d.n, d.k, d.delta, d.accept)[0]
            assert np.array_equal(outs[1], want) and res[1]["num_blocks"] == 3, (n, p)
            _, res = dfamin.dfamin_minimize_batch(ctx, [W.random_dfa(3, 2, 1), bad], None, check=False)
            assert res[1]["status"] == dfamin.DFAMIN_E_BAD_DFA and res[0]["status"] == 0, (n, p)


def test_fresh_context_first_call_is_a_large_batch():
    """Uploads are staged in page-locked arenas that start empty and grow
    (draining the stream first) when a phase of a call needs more: on a
    fresh context whose first call is a batch of 3,000 instances, the job
    lists, descriptors and row pointers outgrow them several times within
    the call.  Every instance matches the oracle, and so does a second,
    differently shaped call on the grown arenas."""
    from paper_2410_22764_amd import dfamin
    rng = np.random.default_rng(77)
    ds = []
    for t in range(3000):
        n = int(rng.integers(2, 300))
        ds.append(W.random_dfa(n, int(rng.integers(1, 6)), 1000 + t) if t % 4 else
                  W.permuted_chain_dfa(n, 1, 5000 + t))
    with dfamin.dfamin_create(0) as c:
        print("[case] fresh context, 3,000-instance batch", flush=True)
        outs, res = dfamin.dfamin_minimize_batch(c, ds, "auto")
        for d, o, r in zip(ds, outs, res):
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert r["num_blocks"] == nb and np.array_equal(o, want), d.name
        d = W.random_dfa(50000, 3, 9)
        out, r = dfamin.dfamin_minimize(c, d, "off")
        assert np.array_equal(out, oracle.hopcroft(d.n, d.k, d.delta, d.accept)[0])


def _mixed_case(rng, i):
    kind = rng.choice(["random", "chain", "pchain", "fib", "coarse", "cycle"])
    n = int(2 ** rng.uniform(0, 12)) + 1
    k = int(rng.integers(1, 6))
    seed = int(rng.integers(1, 1 << 30))
    if kind == "random":
        return W.random_dfa(n, k, seed)
    if kind == "chain":
        return W.chain_dfa(max(n, 2), k)
    if kind == "pchain":
        return W.permuted_chain_dfa(max(n, 2), k, seed)
    if kind == "fib":
        return W.fib_dfa(int(rng.integers(3, 15)))
    if kind == "cycle":
        rows = np.array([(np.arange(n) + 1) % n] + [np.arange(n)] * (k - 1), dtype=np.uint32)
        return W.from_rows(rows, rng.random(n) < 0.3, name=f"cycle{n}x{k}")
    d = W.random_dfa(n, k, seed)
    acc = np.zeros(n, bool)
    acc[:: int(rng.integers(2, 50))] = True
    d.accept = W.pack_accept(acc)
    return d


def test_mixed_call_sequence_one_context(ctx):
    """Sixty calls on one context with shapes, methods and options drawn at
    random (seeded): single DFAs and batches, closure off/on/auto, queued
    rounds on and off, signature and leader rounds.  Buffers, captured
    graphs and tuned tiles carried from call to call must not change any
    result: each one is checked against the oracle."""
    from paper_2410_22764_amd import dfamin
    rng = np.random.default_rng(2024)
    for it in range(60):
        ds = [_mixed_case(rng, j) for j in range(int(rng.integers(2, 9)) if rng.random() < 0.25 else 1)]
        opts = dict(closure=str(rng.choice(["off", "on", "auto"])), queue=bool(rng.random() < 0.5),
                    method=str(rng.choice(["signature", "leader"], p=[0.8, 0.2])))
        if opts["method"] == "leader":
            opts.pop("queue")
            if opts["closure"] == "off" and max(d.n for d in ds) > 1000:
                opts["closure"] = "auto"  # plain leader rounds on a long chain take n rounds
        print(f"[case] mixed it={it} {[d.name for d in ds]} {opts}", flush=True)
        outs, res = dfamin.dfamin_minimize_batch(ctx, ds, opts)
        for d, o, r in zip(ds, outs, res):
            want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert r["num_blocks"] == nb and np.array_equal(o, want), (it, d.name, opts)
            assert r["initial_block"] == want[d.q0]


def test_queued_doubling_rounds_agree(ctx):
    """One-letter instances under AUTO with the queue flag: once every
    instance still refining doubles, the device plans the levels and the
    rounds are queued (hash keys).  Alone and in a batch of chains of different lengths, queued
    rounds (graph and direct) match host-planned rounds (profiling on) and
    the oracle, with the round counts derived from Moore's partitions."""
    from paper_2410_22764_amd import dfamin
    singles = [W.chain_dfa(2000, 2), W.fib_dfa(14), W.permuted_chain_dfa(1500, 3, 5), W.random_dfa(1500, 1, 4)]
    for d in singles:
        want, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        print(f"[case] queued doubling {d.name}", flush=True)
        dfamin.dfamin_set_profiling(ctx, True)
        planned, rp = dfamin.dfamin_minimize(ctx, d, "auto")
        dfamin.dfamin_set_profiling(ctx, False)
        assert np.array_equal(planned, want) and rp["refine_rounds"] == _auto_unary_rounds(d), d.name
        for opts in [dict(closure="auto", queue=True), dict(closure="auto", queue=True, no_graph=True),
                     dict(closure="auto", queue=True)]:
            out, r = dfamin.dfamin_minimize(ctx, d, opts)
            assert np.array_equal(out, want) and r == rp, (d.name, opts)
    sizes = (17, 300, 1000, 4097, 20000)
    batch = [W.permuted_chain_dfa(n, 2, 40 + n) for n in sizes] + [W.fib_dfa(12)]
    # a chain of n states needs ceil(log2(n - 1)) doubling rounds (P_(2^r - 1)
    # holds every state alone once 2^r - 1 >= n - 2)
    want_rounds = [math.ceil(math.log2(n - 1)) for n in sizes] + [_auto_unary_rounds(batch[-1])]
    print("[case] queued doubling batch", flush=True)
    dfamin.dfamin_set_profiling(ctx, True)
    po, pr = dfamin.dfamin_minimize_batch(ctx, batch, "auto")
    dfamin.dfamin_set_profiling(ctx, False)
    for opts in [dict(closure="auto", queue=True), dict(closure="auto", queue=True, no_graph=True)]:
        outs, res = dfamin.dfamin_minimize_batch(ctx, batch, opts)
        for d, o, r, p, rp, wr in zip(batch, outs, res, po, pr, want_rounds):
            want, _ = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            assert np.array_equal(o, want) and np.array_equal(p, want), d.name
            assert r == rp and r["refine_rounds"] == wr, d.name
