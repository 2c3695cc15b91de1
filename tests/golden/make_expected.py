"""Writes expected_workloads.json: oracle results for the full-size synthetic
workloads, so GPU tests can compare against them without re-running the
oracle on every box.  Calls only the CPU oracle (oracle/) and the seeded
input generators.

    python tests/golden/make_expected.py                 # every section
    python tests/golden/make_expected.py serving_pool    # recompute one section, keep the others

Sections:
  plain_single   random DFAs n = 16,384, |Sigma| = 2, seeds 1..5 (with Moore's r*)
  plain_large    random DFAs n = 2^24, |Sigma| = 4, seeds 1..3
  batch_mixed    the 4,096-instance batch of seed 1
  serving_pool   a pool of requests drawn from the serving stream (seed 11):
                 n log-uniform in [2^8, 2^22], |Sigma| in 2..16, 20% permuted
                 chains; see serving_pool_indices()
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

PATH = os.path.join(HERE, "expected_workloads.json")
SERVING_SEED = 11
SERVING_DRAWS = 3000


def digest(out):
    return hashlib.sha256(np.ascontiguousarray(out, dtype="<u4").tobytes()).hexdigest()[:32]


def serving_pool_indices(specs):
    """Which requests of the stream form the pool: the stream's first 16
    (sizes and kinds as drawn), the first two random DFAs with n >= 2^20 and
    |Sigma| = 16, the first three permuted chains with n >= 2^20, and the
    largest random DFA and the largest chain of all the draws."""
    first = list(range(16))
    big16 = [i for i, s in enumerate(specs) if s[0] == "random" and s[1] >= 1 << 20 and s[2] == 16][:2]
    chains = [i for i, s in enumerate(specs) if s[0] == "chain" and s[1] >= 1 << 20][:3]
    largest_random = max((i for i, s in enumerate(specs) if s[0] == "random"), key=lambda i: specs[i][1])
    largest_chain = max((i for i, s in enumerate(specs) if s[0] == "chain"), key=lambda i: specs[i][1])
    out = []
    for i in first + big16 + chains + [largest_random, largest_chain]:
        if i not in out:
            out.append(i)
    return out


def plain_single():
    res = {}
    for seed in range(1, 6):
        d = W.plain_single(seed)
        out, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        _, _, rr = oracle.moore(d.n, d.k, d.delta, d.accept)
        res[str(seed)] = {"num_blocks": nb, "sha": digest(out), "refine_rounds": rr}
    return res


def plain_large():
    res = {}
    for seed in (1, 2, 3):
        d = W.plain_large(seed)
        out, nb = oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        res[str(seed)] = {"num_blocks": nb, "sha": digest(out),
                          "identity": bool(np.array_equal(out, np.arange(d.n)))}
        del d, out
    return res


def batch_mixed():
    batch = W.batch_mixed(seed=1)
    outs = oracle.hopcroft_many([(b.n, b.k, b.delta, b.accept) for b in batch])
    return {"1": [{"n": b.n, "k": b.k, "num_blocks": nb, "sha": digest(o)}
                  for b, (o, nb) in zip(batch, outs)]}


def serving_pool():
    _, specs = W.serving_stream(SERVING_SEED, SERVING_DRAWS, 1.0)
    idx = serving_pool_indices(specs)
    pool = [W.make_request(specs[i]) for i in idx]
    outs = oracle.hopcroft_many([(d.n, d.k, d.delta, d.accept) for d in pool])
    return {"seed": SERVING_SEED, "draws": SERVING_DRAWS,
            "requests": [{"index": i, "kind": specs[i][0], "n": d.n, "k": d.k, "num_blocks": nb,
                          "initial_block": int(o[d.q0]), "sha": digest(o)}
                         for i, d, (o, nb) in zip(idx, pool, outs)]}


SECTIONS = {"plain_single": plain_single, "plain_large": plain_large, "batch_mixed": batch_mixed,
            "serving_pool": serving_pool}


def main(argv):
    which = argv or list(SECTIONS)
    res = json.load(open(PATH)) if os.path.exists(PATH) else {}
    res["note"] = ("oracle (Hopcroft) results: num_blocks and sha256[:32] of the canonical "
                   "block array as little-endian uint32")
    for name in which:
        t = time.time()
        res[name] = SECTIONS[name]()
        print(name, round(time.time() - t, 1), "s", flush=True)
    with open(PATH, "w") as f:
        json.dump(res, f, indent=0, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
