"""The oracle's pins catch plausible mistakes in the oracle itself.

Each case copies the oracle package to a temporary directory, plants one
mistake in oracle.c (a dropped term, a wrong index or operand, an off-by-one),
builds it with gcc and runs a battery of the pins against it: at least one
pin must fail.  An unmutated copy must pass them all.  CPU only.
"""
import importlib.util
import os
import shutil
import sys

import numpy as np
import pytest

from paper_2410_22764_amd import workloads as W

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

MUTANTS = {
    "moore_without_own_block": ("sig[(size_t)q * k1] = block[q];", "sig[(size_t)q * k1] = 0;"),
    "moore_gathers_state_not_block": ("sig[(size_t)q * k1 + 1 + a] = block[delta[(size_t)a * n + q]];",
                                      "sig[(size_t)q * k1 + 1 + a] = delta[(size_t)a * n + q];"),
    "hopcroft_drops_smaller_half": ("else add = (szZ <= szY) ? Z : Y;", "else continue;"),
    "canonical_ids_from_one": ("if (map[l] == UINT32_MAX) map[l] = next++;",
                               "if (map[l] == UINT32_MAX) map[l] = ++next;"),
    "closure_level_not_squared": ("cur[q] = prev[prev[q]];", "cur[q] = prev[q];"),
    "naive_compares_with_itself": ("block[delta[(size_t)a * n + q]] != block[delta[(size_t)a * n + L]]",
                                   "block[delta[(size_t)a * n + q]] != block[delta[(size_t)a * n + q]]"),
    "quotient_letters_loop": ("= rid[cls[delta[(size_t)a * n + r]]];", "= rid[cls[r]];"),
}


def _build_copy(tmp_path, name, old=None, new=None):
    d = tmp_path / name
    d.mkdir()
    for f in ("__init__.py", "build_oracle.py", "oracle.h", "oracle_selftest.c"):
        shutil.copy(os.path.join(ORACLE_DIR, f), d / f)
    src = open(os.path.join(ORACLE_DIR, "oracle.c")).read()
    if old is not None:
        assert src.count(old) == 1, name
        src = src.replace(old, new)
    (d / "oracle.c").write_text(src)
    modname = f"oracle_copy_{name}"
    spec = importlib.util.spec_from_file_location(modname, d / "__init__.py", submodule_search_locations=[str(d)])
    mod = importlib.util.module_from_spec(spec)
    sys.modules[modname] = mod
    spec.loader.exec_module(mod)
    importlib.import_module(modname + ".build_oracle").build()
    return mod


def _same_language(d, m, dm, am, q0m):
    acc1 = d.accept_bool()
    acc2 = np.unpackbits(am, bitorder="little")[:m].astype(bool)
    r1, r2 = d.rows(), dm.reshape(d.k, m)
    seen, stack = {(d.q0, q0m)}, [(d.q0, q0m)]
    while stack:
        p, q = stack.pop()
        if acc1[p] != acc2[q]:
            return False
        for a in range(d.k):
            nxt = (int(r1[a][p]), int(r2[a][q]))
            if nxt not in seen:
                seen.add(nxt)
                stack.append(nxt)
    return True


def _failed_pins(o):
    """Names of the pins that fail for oracle module o."""
    failed = []

    def check(name, fn):
        try:
            if not fn():
                failed.append(name)
        except Exception:
            failed.append(name)

    check("exhaustive n=3 k=2", lambda: o.exhaustive_check(3, 2)[1] == 0)
    chain = W.chain_dfa(50, 2)
    check("chain closed form", lambda: (lambda r: r[1] == 50 and r[2] == 48 and
                                        np.array_equal(r[0], np.arange(50)))(
        o.moore(chain.n, chain.k, chain.delta, chain.accept)))
    check("figure 1 with the closure", lambda: o.moore_closure(10, 1, W.chain_dfa(10, 1).delta,
                                                                W.chain_dfa(10, 1).accept)[2] == 3)

    def closure_rows():
        d = W.chain_dfa(40, 1)
        rows = o.closure(d.n, d.k, d.delta, 5)
        return all(np.array_equal(rows[i], np.minimum(np.arange(40) + 2 ** i, 39)) for i in range(6))
    check("closure rows", closure_rows)

    def canonical():
        d = W.random_dfa(500, 2, 3)
        out, nb = o.hopcroft(d.n, d.k, d.delta, d.accept)
        firsts = [int(np.argmax(out == b)) for b in range(nb)]
        return out[0] == 0 and out.max() == nb - 1 and firsts == sorted(firsts)
    check("canonical numbering", canonical)

    def naive_eq():
        d = W.random_dfa(300, 2, 5)
        h, _ = o.hopcroft(d.n, d.k, d.delta, d.accept)
        a, _, it = o.naive(d.n, d.k, d.delta, d.accept)
        return np.array_equal(a, h) and o.naive(W.fib_dfa(10).n, 1, W.fib_dfa(10).delta,
                                                W.fib_dfa(10).accept)[2] == W.fib_dfa(10).n - 1
    check("naivePR = Hopcroft, Fib iterations", naive_eq)

    def minimal():
        for seed in range(3):
            d = W.random_dfa(60, 2, seed)
            m, dm, am, q0m, _ = o.minimal_dfa(d.n, d.k, d.delta, d.accept, d.q0)
            if not _same_language(d, m, dm, am, q0m):
                return False
        return True
    check("minimal DFA language", minimal)
    return failed


def test_unmutated_copy_passes_every_pin(tmp_path):
    o = _build_copy(tmp_path, "control")
    assert _failed_pins(o) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    o = _build_copy(tmp_path, name, old, new)
    assert _failed_pins(o), f"no pin caught the mutant {name}"
