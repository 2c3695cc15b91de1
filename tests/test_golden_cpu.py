"""The stored workload expectations agree with the oracle (cheap subset)."""
import hashlib
import json
import os

import numpy as np

import oracle
from paper_2410_22764_amd import workloads as W

EXPECTED = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "expected_workloads.json")))


def digest(out):
    return hashlib.sha256(np.ascontiguousarray(out, dtype="<u4").tobytes()).hexdigest()[:32]


def test_plain_single_expectations_match_oracle():
    for seed, e in EXPECTED["plain_single"].items():
        d = W.plain_single(int(seed))
        out, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        assert nb == e["num_blocks"] and digest(out) == e["sha"]
        assert oracle.moore(d.n, d.k, d.delta, d.accept)[2] == e["refine_rounds"]


def test_batch_expectations_match_oracle_sample():
    batch = W.batch_mixed(seed=1)
    exp = EXPECTED["batch_mixed"]["1"]
    for i in range(0, 4096, 97):
        d = batch[i]
        out, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        assert nb == exp[i]["num_blocks"] and digest(out) == exp[i]["sha"]
    chains = [i for i, d in enumerate(batch) if d.name.startswith("permuted_chain")]
    assert len(chains) == 1024
    for i in chains[:50]:
        assert exp[i]["num_blocks"] == batch[i].n  # chains: every state its own class
