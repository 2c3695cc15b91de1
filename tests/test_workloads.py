"""Seeded input generators: determinism and the stated distributions."""
import numpy as np
import pytest

from paper_2410_22764_amd import workloads as W


def test_splitmix64_reference_values():
    """SplitMix64 with state 0: the published first outputs of the generator
    (Steele, Lea & Flood 2014) as produced by its reference Java code."""
    out = [W._mix_int((i + 1) * W.GAMMA) for i in range(3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    vec = W.draws(0, 3)
    assert [int(v) for v in vec] == out


def test_random_dfa_deterministic_and_in_range():
    a = W.random_dfa(1000, 3, 7)
    b = W.random_dfa(1000, 3, 7)
    c = W.random_dfa(1000, 3, 8)
    assert np.array_equal(a.delta, b.delta) and np.array_equal(a.accept, b.accept)
    assert not np.array_equal(a.delta, c.delta)
    assert a.delta.dtype == np.uint32 and a.delta.max() < 1000
    assert a.accept.size == (1000 + 7) // 8


def test_uniform_below_unbiased_for_odd_n():
    n = 7
    x = W.uniform_below(W.stream_key(3, "t"), 70000, n)
    counts = np.bincount(x.astype(np.int64), minlength=n)
    assert counts.min() > 9400 and counts.max() < 10600


def test_accept_bernoulli_half():
    d = W.random_dfa(1 << 16, 2, 1)
    frac = d.accept_bool().mean()
    assert 0.49 < frac < 0.51


def test_chain_and_permuted_chain():
    c = W.chain_dfa(5, 3)
    assert c.rows().tolist() == [[1, 2, 3, 4, 4], [0, 1, 2, 3, 4], [0, 1, 2, 3, 4]]
    assert c.accept_bool().tolist() == [False] * 4 + [True]
    p = W.permuted_chain_dfa(50, 2, 3)
    pi = p.meta["perm"]
    assert sorted(pi.tolist()) == list(range(50))
    assert p.q0 == pi[0]
    for i in range(50):
        assert p.rows()[0][pi[i]] == pi[min(i + 1, 49)]
        assert p.rows()[1][pi[i]] == pi[i]


def test_fib_words():
    assert [W.fib_word(i) for i in range(6)] == ["1", "0", "01", "010", "01001", "01001010"]


def test_batch_mixed_composition():
    batch = W.batch_mixed(seed=1, count=256)
    ns = np.array([d.n for d in batch])
    ks = np.array([d.k for d in batch])
    chains = sum(d.name.startswith("permuted_chain") for d in batch)
    assert chains == 64
    assert ns.min() >= 64 and ns.max() <= 65536
    assert ks.min() >= 2 and ks.max() <= 8


def test_serving_stream():
    t, specs = W.serving_stream(seed=2, count=500, rate_per_s=100.0)
    assert np.all(np.diff(t) > 0)
    assert 3.0 < t[-1] < 7.0  # 500 arrivals at 100/s
    kinds = [s[0] for s in specs]
    assert 0.1 < kinds.count("chain") / 500 < 0.3
    assert all(256 <= s[1] <= 1 << 22 and 2 <= s[2] <= 16 for s in specs)
