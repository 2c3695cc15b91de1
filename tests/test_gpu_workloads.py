"""Full-size synthetic workloads on the GPU against oracle results.

Expected values come from tests/golden/expected_workloads.json, written by
tests/golden/make_expected.py with the CPU oracle only.
"""
import hashlib
import json
import os

import numpy as np
import pytest

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


@pytest.mark.parametrize("seed", ["1", "2", "3"])
def test_plain_large_full_size(ctx, seed):
    """Random DFA, n = 2^24, |Sigma| = 4, seeds 1..3, through the device entry
    point with the closure policy the benchmark uses."""
    import torch
    from paper_2410_22764_amd import dfamin
    print(f"[case] plain_large seed {seed}", flush=True)
    d = W.plain_large(int(seed))
    dev = torch.device("cuda:0")
    delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
    accept = torch.from_numpy(d.accept).to(dev)
    out = torch.empty(d.n, dtype=torch.int32, device=dev)
    res = dfamin.dfamin_minimize_device(ctx, d.n, d.k, delta.data_ptr(), accept.data_ptr(), d.q0,
                                        out.data_ptr(), opts="auto",
                                        stream=torch.cuda.current_stream().cuda_stream)
    got = out.cpu().numpy().view(np.uint32)
    exp = EXPECTED["plain_large"][seed]
    assert res["num_blocks"] == exp["num_blocks"]
    assert digest(got) == exp["sha"]
    del delta, accept, out


@pytest.mark.parametrize("closure", ["auto", "on"])
def test_batch_mixed_full_size(ctx, closure):
    """4,096 uneven DFAs (75% random, 25% permuted chains) in one batched call."""
    from paper_2410_22764_amd import dfamin
    print(f"[case] batch_mixed seed 1 closure={closure}", flush=True)
    batch = W.batch_mixed(seed=1)
    outs, results = dfamin.dfamin_minimize_batch(ctx, batch, {"closure": closure})
    exp = EXPECTED["batch_mixed"]["1"]
    assert len(exp) == len(batch) == 4096
    for d, o, r, e in zip(batch, outs, results, exp):
        assert (d.n, d.k) == (e["n"], e["k"])
        assert r["num_blocks"] == e["num_blocks"], d.name
        assert digest(o) == e["sha"], d.name


def test_plain_single_seeds(ctx):
    from paper_2410_22764_amd import dfamin
    for seed, e in EXPECTED["plain_single"].items():
        d = W.plain_single(int(seed))
        out, res = dfamin.dfamin_minimize(ctx, d, "auto")
        assert res["num_blocks"] == e["num_blocks"] and digest(out) == e["sha"]
        assert res["refine_rounds"] == e["refine_rounds"]


@pytest.mark.parametrize("m", [20, 23, 26])
def test_table2_bitsplitters(ctx, m):
    """B_m at the sizes of the paper's Table 2 (B_24..B_26 ran out of memory
    there with the closure).  Closed forms: 2^m classes, all singletons (so
    the canonical output is the identity), m - 1 refining rounds.  Every
    closure level above 0 equals level 0 (a_j applied twice is a_j), so the
    closure keeps only the m - 1 letters."""
    from paper_2410_22764_amd import dfamin
    print(f"[case] B_{m}", flush=True)
    d = W.bitsplitter_dfa(m)
    out, res = dfamin.dfamin_minimize(ctx, d, "auto")
    assert res["num_blocks"] == 2 ** m
    assert np.array_equal(out, np.arange(2 ** m, dtype=np.uint32))
    assert res["refine_rounds"] == m - 1
    assert res["closure_letters"] == m - 1 and res["closure_levels"] == m


def test_table2_fib30(ctx):
    """Fib_30 (2,178,309 states, unary): every state is its own class."""
    from paper_2410_22764_amd import dfamin
    print("[case] Fib_30", flush=True)
    d = W.fib_dfa(30)
    assert d.n == 2178309
    out, res = dfamin.dfamin_minimize(ctx, d, "auto")
    assert res["num_blocks"] == d.n
    assert np.array_equal(out, np.arange(d.n, dtype=np.uint32))


def test_state_limit_rejected_before_staging(ctx):
    """n at the 31-bit state-id limit is refused up front: the host-input
    entry point returns E_INVAL without reading the (here tiny) buffers."""
    from paper_2410_22764_amd import dfamin
    print("[case] n = 2^31 - 256 rejected", flush=True)
    d = W.DFA(n=(1 << 31) - 256, k=1, delta=np.zeros(4, np.uint32), accept=np.zeros(4, np.uint8), q0=0,
              name="over the limit")
    s, keep = dfamin._host_dfa(d, check=False)
    out = np.empty(4, np.uint32)
    res = dfamin.Result()
    rc = dfamin.load().dfamin_minimize(ctx.handle, dfamin.ctypes.byref(s), dfamin._opts(None),
                                       out.ctypes.data, dfamin.ctypes.byref(res))
    assert rc == dfamin.DFAMIN_E_INVAL


def test_huge_chain_64bit_offsets(ctx):
    """A chain of n = 2^27 states over 40 letters, built on the device: the
    last letter is the chain (i -> i+1, n-1 -> n-1), the 39 others are the
    identity, only state n-1 accepts.  delta has 40 * 2^27 = 5.4e9 entries,
    so every row offset past letter 31 needs more than 32 bits.  Closed forms:
    every state is its own class, and AUTO (doubling from the first round)
    takes ceil(log2(n - 1)) = 27 refining rounds."""
    import torch
    from paper_2410_22764_amd import dfamin
    n, k = 1 << 27, 40
    print(f"[case] chain n=2^27 k={k} on the device", flush=True)
    dev = torch.device("cuda:0")
    ar = torch.arange(n, dtype=torch.int32, device=dev)
    delta = torch.empty((k, n), dtype=torch.int32, device=dev)
    delta[:] = ar
    delta[k - 1, :-1] = ar[1:]
    delta[k - 1, -1] = n - 1
    acc = torch.zeros((n + 7) // 8, dtype=torch.uint8, device=dev)
    acc[(n - 1) >> 3] = 1 << ((n - 1) & 7)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    res = dfamin.dfamin_minimize_device(ctx, n, k, delta.data_ptr(), acc.data_ptr(), 0, out.data_ptr(),
                                        {"closure": "auto"}, stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert res["num_blocks"] == n and res["initial_block"] == 0
    assert res["refine_rounds"] == 27 and res["rounds_executed"] == 28
    assert bool(torch.equal(out, ar))
    del delta, acc, out, ar
    torch.cuda.empty_cache()
