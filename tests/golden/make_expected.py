"""Writes expected_workloads.json: oracle results for the full-size synthetic
workloads, so GPU tests can compare against them without re-running the
oracle on every box.  Calls only the CPU oracle (oracle/) and the seeded
input generators.

    python tests/golden/make_expected.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2410_22764_amd import workloads as W  # noqa: E402


def digest(out):
    return hashlib.sha256(np.ascontiguousarray(out, dtype="<u4").tobytes()).hexdigest()[:32]


def main():
    res = {"note": "oracle (Hopcroft) results: num_blocks and sha256[:32] of the canonical "
                   "block array as little-endian uint32"}
    t = time.time()
    res["plain_single"] = {}
    for seed in range(1, 6):
        d = W.plain_single(seed)
        out, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        _, _, rr = oracle.moore(d.n, d.k, d.delta, d.accept)
        res["plain_single"][str(seed)] = {"num_blocks": nb, "sha": digest(out), "refine_rounds": rr}
    print("plain_single", time.time() - t, flush=True)
    t = time.time()
    d = W.plain_large(1)
    out, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
    res["plain_large"] = {"1": {"num_blocks": nb, "sha": digest(out),
                                "identity": bool(np.array_equal(out, np.arange(d.n)))}}
    print("plain_large", time.time() - t, flush=True)
    t = time.time()
    batch = W.batch_mixed(seed=1)
    outs = oracle.hopcroft_many([(b.n, b.k, b.delta, b.accept) for b in batch])
    res["batch_mixed"] = {"1": [{"n": b.n, "k": b.k, "num_blocks": nb, "sha": digest(o)}
                                for b, (o, nb) in zip(batch, outs)]}
    print("batch_mixed", time.time() - t, flush=True)
    with open(os.path.join(HERE, "expected_workloads.json"), "w") as f:
        json.dump(res, f, indent=0, sort_keys=True)


if __name__ == "__main__":
    main()
