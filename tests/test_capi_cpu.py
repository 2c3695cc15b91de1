"""Host-side checks of the C-ABI library (no GPU compute)."""
import ctypes
import os
import re

import pytest

from paper_2410_22764_amd import dfamin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "dfamin.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfamin_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = dfamin.load()
    declared = _declared_functions()
    assert len(declared) >= 12
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(dfamin.EXPORTS) == declared


def test_status_strings():
    for code in range(0, -9, -1):
        s = dfamin.status_str(code)
        assert s and s != "unknown status"
    assert dfamin.status_str(-100) == "unknown status"


def test_null_arguments_rejected_without_device_work():
    lib = dfamin.load()
    assert lib.dfamin_minimize(None, None, None, None, None) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_minimize_device(None, None, None, None, None, None) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_minimize_device_noalloc(None, None, None, None, None, None) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_minimize_batch(None, 0, None, None, None, None) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_submit(None, None, None, None) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_cancel(None, 1) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_set_profiling(None, 1) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_set_tuning(None, -1) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_minimal_dfa(None, None, None, None, None, None, None) == dfamin.DFAMIN_E_INVAL
    assert lib.dfamin_create(0, 0, None) == dfamin.DFAMIN_E_INVAL


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = dfamin.load().dfamin_create(0, 0, ctypes.byref(h))
    assert rc == dfamin.DFAMIN_E_DEVICE and not h.value


def test_binding_refuses_short_host_arrays():
    """The library copies k*n transitions and ceil(n/8) accept bytes out of
    the caller's host buffers; the binding refuses shorter arrays before any
    native call (here: no context, no GPU)."""
    import numpy as np
    from paper_2410_22764_amd import workloads as W

    class NoCtx:
        handle = None
        tickets = {}

    n = 7913
    rows = np.stack([(np.arange(n) + 1) % n, np.arange(n)]).astype(np.uint32)
    acc = np.arange(n) % 3 == 0
    good = W.from_rows(rows, acc)
    assert good.accept.size == (n + 7) // 8
    twice = W.from_rows(rows, W.pack_accept(acc))  # bitmap packed twice: 124 bytes
    assert twice.accept.size < (n + 7) // 8
    for call in (lambda d: dfamin.dfamin_minimize(NoCtx(), d),
                 lambda d: dfamin.dfamin_minimize_batch(NoCtx(), [good, d]),
                 lambda d: dfamin.dfamin_submit(NoCtx(), d),
                 lambda d: dfamin.dfamin_minimal_dfa(NoCtx(), d)):
        with pytest.raises(ValueError, match="accept"):
            call(twice)
        short = W.DFA(n, 2, good.delta[:-1], good.accept)
        with pytest.raises(ValueError, match="delta"):
            call(short)
    # raw marshalling stays available to exercise the C-side checks
    s, _ = dfamin._host_dfa(twice, check=False)
    assert s.n == n


def test_wait_refuses_an_output_shorter_than_the_ticket():
    class FakeCtx:
        handle = None
        tickets = {7: 100}

    with pytest.raises(ValueError, match="room"):
        dfamin.dfamin_wait(FakeCtx(), 7, 99)


def test_zeroed_options_mean_closure_auto():
    """A NULL or zeroed dfamin_opts selects closure AUTO: the header gives
    DFAMIN_CLOSURE_AUTO the value 0, and the binding agrees (its default
    options are a zeroed struct)."""
    text = open(os.path.join(ROOT, "include", "dfamin.h")).read()
    vals = {m: int(v) for m, v in re.findall(r"#define DFAMIN_CLOSURE_(\w+)\s+(\d+)u", text)}
    assert vals == {"AUTO": 0, "OFF": 1, "ON": 2}
    assert dfamin.CLOSURE == {"auto": 0, "off": 1, "on": 2}
    o = dfamin.make_opts()
    assert bytes(o) == bytes(dfamin.Opts())


def test_noalloc_size_limit_matches_header():
    """The binding's size check and scratch size are those the header states."""
    import re as _re
    text = open(os.path.join(ROOT, "include", "dfamin.h")).read()
    m = _re.search(r"#define DFAMIN_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == dfamin.NOALLOC_SCRATCH_BYTES
    assert "n * (66 + 16 * (k + 1)) + 2^20" in text
    assert dfamin.noalloc_fits(579_000, 2) and not dfamin.noalloc_fits(579_500, 2)


def test_exact_keys_after_a_label_round_fit_one_byte():
    """After the first round by labels, the next round's dense numbers are
    written one byte wide.  That is sound because a round groups on exact
    keys only when (k'+1) * ceil(log2 B) <= 31, and after the label round
    B <= 2^(k'+1) with k' >= 0 signature letters (the engine's rule, here
    for every k' and every B that rule can meet, with the same at-least-one
    bit as the engine): such a round never has more than 32 blocks."""
    def ceil_log2(x):
        return max(1, (x - 1).bit_length())
    worst = 0
    for kp in range(0, 9):  # up to 8 signature letters: labels of kp+1 <= 9 bits
        for blocks in range(1, 2 ** (kp + 1) + 1):
            if (kp + 1) * ceil_log2(blocks) <= 31:
                worst = max(worst, blocks)
    assert worst == 32 and worst <= 256
