"""Benchmark: transitions minimized per second on one MI355X.

Default workload: a random complete DFA with n = 2^24 states and |Sigma| = 4
(uniform transitions, accepting with probability 1/2, seed 1), inputs
resident in HBM before the timed region.  One step = one full minimization
(validation, initial partition, every refinement round, canonical numbering
and emission) through the C-ABI's device entry point.

Prints ONE JSON line with the throughput, a roofline entry for the kernel
that takes the most time (algorithmic bytes / HIP-event time, against the
8 TB/s HBM peak) and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "transitions minimized/s (n·|Σ|/wall), batched vs plain; p50/p99 latency"

WORKLOADS = {
    "plain_large": dict(kind="random", n=1 << 24, k=4, closure="auto",
                        desc="random complete DFA, n=2^24, |Sigma|=4, uniform delta, Bernoulli(0.5) accepting"),
    "plain_single": dict(kind="random", n=16384, k=2, closure="auto",
                         desc="random complete DFA, n=16384, |Sigma|=2, uniform delta, Bernoulli(0.5) accepting"),
    "deep_chain": dict(kind="chain", n=1 << 20, k=2, closure="on",
                       desc="chain DFA, n=2^20, |Sigma|=2 (second letter the identity), closure on"),
    "fib20": dict(kind="fib", m=20, closure="auto",
                  desc="Fib_20 of the paper's Table 2: unary, 17,711 states",
                  paper={"system": "NVIDIA TITAN RTX (Table 2)", "sortPR_ms": 3909.2, "sortPR_iterations": 17710,
                         "transPR_ms": 1.7, "transPR_iterations": 14, "naivePR_ms": 308.8,
                         "naivePR_iterations": 17710}),
    "fib30": dict(kind="fib", m=30, closure="auto",
                  desc="Fib_30 of the paper's Table 2: unary, 2,178,309 states, accepting where the "
                       "Fibonacci word w_31 has a 1",
                  paper={"system": "NVIDIA TITAN RTX (Table 2)", "transPR_ms": 1109.3, "transPR_iterations": 914,
                         "naivePR_ms": 141601.0, "sortPR": "timed out"}),
    "bitsplitter23": dict(kind="bitsplitter", m=23, closure="auto",
                          desc="B_23 of the paper's Table 2: 2^23 states, 22 letters",
                          paper={"system": "NVIDIA TITAN RTX (Table 2)", "sortPR_ms": 5612.7,
                                 "sortPR_iterations": 22, "transPR_ms": 1612.1, "naivePR_ms": 170.3}),
    "bitsplitter26": dict(kind="bitsplitter", m=26, closure="auto",
                          desc="B_26 of the paper's Table 2: 2^26 states, 25 letters",
                          paper={"system": "NVIDIA TITAN RTX (Table 2)", "sortPR_ms": 59203.8,
                                 "sortPR_iterations": 25, "transPR": "out of memory", "naivePR_ms": 1541.5}),
    "batch_mixed": dict(kind="batch", closure="auto",
                        desc="4096 DFAs, n log-uniform in [64, 65536], |Sigma| in 2..8, 25% permuted chains, "
                             "closure auto, one batched call per step"),
    "serving": dict(kind="serving", desc="Poisson request stream"),
}


# Sources that decide what the benchmarked kernels do (the kernels, their
# launch parameters and the engine's choices); the serving loop and the C-ABI
# wrappers do not take part in these workloads.
KERNEL_SOURCES = ("kernels.hip", "internal.h", "engine.hip", "engine.h", "closure.hip", "closure.h", "fused.hip")


def kernel_source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_22764_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        t = json.load(open(path))
        e = t.get(workload, {}).get(kernel)
        if not e or e.get("source_hash") != kernel_source_hash():
            return None
        return e["bytes_per_launch"]
    except Exception:
        return None


def make_input(spec, seed):
    from paper_2410_22764_amd import workloads as W
    if spec["kind"] == "random":
        return W.random_dfa(spec["n"], spec["k"], seed)
    if spec["kind"] == "fib":
        return W.fib_dfa(spec["m"])
    if spec["kind"] == "bitsplitter":
        return W.bitsplitter_dfa(spec["m"])
    return W.chain_dfa(spec["n"], spec["k"])


def result_summary(res):
    """The step's result: one instance's dict, or totals / maxima over a batch."""
    if isinstance(res, dict):
        return {k: res[k] for k in ("num_blocks", "refine_rounds", "rounds_executed", "closure_levels")}
    return {"num_blocks": int(res.field("num_blocks").sum()),
            "refine_rounds": int(res.field("refine_rounds").max()),
            "rounds_executed": int(res.field("rounds_executed").max()),
            "closure_levels": int(res.field("closure_levels").max())}


def copy_peak_gbps(reps=5, mib=1024):
    """Device-to-device copy rate on this GPU (bytes read + written / time)."""
    import torch
    src = torch.ones((mib << 20) // 4, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2.0 * (mib << 20) / (ms * 1e-3) / 1e9


def random_access_rates(reps=5):
    """Random accesses per second on this GPU, from torch's own kernels:
    4-byte gathers at 2^26 random indices of a 64 MiB table, and 8-byte
    atomic adds at 2^24 random indices of a 256 MiB table.  These are the
    two accesses a signature launch makes per state at random (the
    successors' block ids; one table update per group)."""
    import torch
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(1)
    n = 1 << 24
    src = torch.arange(n, dtype=torch.int32, device=dev)
    idx = torch.randint(0, n, (4 * n,), device=dev, generator=g)
    out = torch.index_select(src, 0, idx)
    table = torch.zeros(1 << 25, dtype=torch.int64, device=dev)
    aidx = torch.randint(0, 1 << 25, (n,), device=dev, generator=g)
    ones = torch.ones(n, dtype=torch.int64, device=dev)
    table.index_add_(0, aidx, ones)
    rates = []
    for work, count in ((lambda: torch.index_select(src, 0, idx, out=out), 4 * n),
                        (lambda: table.index_add_(0, aidx, ones), n)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            work()
        b.record()
        b.synchronize()
        rates.append(count * reps / (a.elapsed_time(b) * 1e-3))
    del src, idx, out, table, aidx, ones
    torch.cuda.empty_cache()
    return rates[0], rates[1]


def host_info():
    """The host the CPU baselines ran on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model}


def pool_threads():
    """Worker threads for the CPU baselines over many instances: every usable
    host core, at most 16 (the host's share per GPU on a shared box)."""
    return max(1, min(16, host_info()["usable_cpus"] or 1))


def pct(xs, q):
    import numpy as np
    return round(float(np.percentile(xs, q)), 4)


def cpu_baseline(spec, seed, budget_s=20.0):
    """The oracle (Hopcroft, single thread) on a bounded sample of the same
    kind of input, scaled to transitions/s."""
    import oracle
    from paper_2410_22764_amd import workloads as W
    n = spec.get("n", 0)
    if spec["kind"] == "random":
        d = W.random_dfa(min(n, 1 << 22), spec["k"], seed)
    elif spec["kind"] == "fib":
        d = W.fib_dfa(spec["m"])
    elif spec["kind"] == "bitsplitter":
        d = W.bitsplitter_dfa(min(spec["m"], 20))
    elif spec["kind"] == "batch":
        d = W.random_dfa(1 << 20, 5, seed)  # mean |Sigma| of the batch
    else:
        d = W.chain_dfa(n, spec["k"])
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.hopcroft(d.n, d.k, d.delta, d.accept)
        reps += 1
        if time.perf_counter() - t0 > budget_s / 2 or reps >= 5:
            break
    wall = (time.perf_counter() - t0) / reps
    out = {"value": d.n * d.k / wall, "unit": "transitions/s", "cores": 1, "kind": "oracle",
           "sample": f"Hopcroft (C, 1 thread: a sequential algorithm) on {d.name}, {reps} run(s), "
                     f"{wall:.2f} s each"}
    out.update(host_info())
    return out


def cpu_baseline_batch(batch):
    """The oracle over every instance of a batch, one Hopcroft per instance on
    a thread pool over the usable host cores (the C calls release the GIL)."""
    import oracle
    threads = pool_threads()
    tup = [(d.n, d.k, d.delta, d.accept) for d in batch]
    t0 = time.perf_counter()
    oracle.hopcroft_many(tup, threads=threads)
    wall = time.perf_counter() - t0
    trans = sum(d.n * d.k for d in batch)
    out = {"value": trans / wall, "unit": "transitions/s", "cores": threads, "kind": "oracle",
           "ms": round(1e3 * wall, 1),
           "sample": f"Hopcroft (C) on all {len(batch)} instances, {threads} threads"}
    out.update(host_info())
    return out


def time_device_steps(step, reps, warmup=3):
    """Wall time of `reps` calls of step() (each returns when its work is
    done), after `warmup` untimed ones: p50 / p99 / mean in ms."""
    import statistics
    for _ in range(warmup):
        step()
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        step()
        lat.append(1e3 * (time.perf_counter() - t0))
    return {"repeats": reps, "ms_p50": pct(lat, 50), "ms_p99": pct(lat, 99),
            "ms_mean": round(statistics.fmean(lat), 4)}


def config_legs(ctx, reps=30):
    """The small single-instance configurations, each timed over `reps`
    device-resident calls: the random DFA of 16,384 states (seeds 1..5) and
    the 2^20-state chain (closure AUTO, the default, and ON), with the oracle
    on the same input beside each; then the rows of the paper's Table 2
    (Fib_20, Fib_30, B_23, B_26) under AUTO, the oracle beside the two Fib
    rows only (on B_m it would take minutes)."""
    import numpy as np
    import torch
    import oracle
    from paper_2410_22764_amd import dfamin, workloads as W
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream

    def leg(d, closure, reps, with_oracle=True):
        delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
        accept = torch.from_numpy(d.accept).to(dev)
        out = torch.empty(d.n, dtype=torch.int32, device=dev)
        res = {}

        def step():
            res.update(dfamin.dfamin_minimize_device(ctx, d.n, d.k, delta.data_ptr(), accept.data_ptr(), d.q0,
                                                     out.data_ptr(), opts={"closure": closure}, stream=stream))
        t = time_device_steps(step, reps)
        t["value_p50"] = d.n * d.k / (t["ms_p50"] * 1e-3)
        t["result"] = result_summary(res)
        del delta, accept, out
        if with_oracle:
            t0 = time.perf_counter()
            oracle.hopcroft(d.n, d.k, d.delta, d.accept)
            t["cpu_oracle_ms"] = round(1e3 * (time.perf_counter() - t0), 3)
        return t

    print("[bench] configs: plain_single seeds 1..5, deep_chain", file=sys.stderr, flush=True)
    single = {}
    for seed in range(1, 6):
        single[str(seed)] = leg(W.random_dfa(16384, 2, seed), "auto", reps)
    chain = W.chain_dfa(1 << 20, 2)
    out = {
        "plain_single": {"workload": "random DFA, n=16384, |Sigma|=2, closure auto, seeds 1..5",
                         "transitions": 32768, "seeds": single,
                         "ms_p50_median_over_seeds": round(statistics.median(
                             x["ms_p50"] for x in single.values()), 4)},
        "deep_chain_auto": dict(workload="chain DFA, n=2^20, |Sigma|=2, closure auto (doubling)",
                                transitions=2 << 20, **leg(chain, "auto", reps)),
        "deep_chain_on": dict(workload="chain DFA, n=2^20, |Sigma|=2, closure on (Algorithm 5 up front)",
                              transitions=2 << 20, **leg(chain, "on", max(20, reps // 2))),
        "cpu_oracle_note": "cpu_oracle_ms: Hopcroft (C, 1 thread) on the same input, once",
    }
    print("[bench] configs: Table 2 rows", file=sys.stderr, flush=True)
    for name, r, with_oracle in (("fib20", reps, True), ("fib30", 20, True), ("bitsplitter23", 5, False),
                                 ("bitsplitter26", 3, False)):
        spec = WORKLOADS[name]
        d = make_input(spec, 0)
        out[name] = dict(workload=spec["desc"] + ", closure auto", transitions=d.n * d.k, paper=spec["paper"],
                         **leg(d, spec["closure"], r, with_oracle))
        del d
        torch.cuda.empty_cache()
    return out


def upload_batch(dfas, dev):
    """Device copies of a list of DFAs: one flat int32 tensor for every delta,
    one uint8 tensor for every bitmap; returns specs of device pointers."""
    import numpy as np
    import torch
    dsz = sum(d.n * d.k for d in dfas)
    asz = sum(-(-d.n // 8) + 8 for d in dfas)
    flat_d = np.empty(dsz, np.uint32)
    flat_a = np.zeros(asz, np.uint8)
    offs = []
    od = oa = 0
    for d in dfas:
        flat_d[od:od + d.n * d.k] = d.delta
        flat_a[oa:oa + d.accept.size] = d.accept
        offs.append((od, oa))
        od += d.n * d.k
        oa += -(-d.n // 8) + 8
    td = torch.from_numpy(flat_d.view(np.int32)).to(dev)
    ta = torch.from_numpy(flat_a).to(dev)
    to = torch.empty(sum(d.n for d in dfas), dtype=torch.int32, device=dev)
    specs, outs = [], []
    oo = 0
    for d, (od, oa) in zip(dfas, offs):
        specs.append((d.n, d.k, td.data_ptr() + 4 * od, ta.data_ptr() + oa, d.q0))
        outs.append(to.data_ptr() + 4 * oo)
        oo += d.n
    return specs, outs, (td, ta, to)


def batched_vs_plain(ctx, seed=1, reps=10, plain_passes=2):
    """Batched workload: 4,096 uneven DFAs in one call vs. one call per DFA,
    and the oracle over the same instances on a host thread pool."""
    import torch
    from paper_2410_22764_amd import dfamin, workloads as W
    print("[bench] batch: generating 4096 DFAs", file=sys.stderr, flush=True)
    batch = W.batch_mixed(seed=seed)
    dev = torch.device("cuda:0")
    specs, outs, keep = upload_batch(batch, dev)
    stream = torch.cuda.current_stream().cuda_stream
    trans = sum(d.n * d.k for d in batch)
    opts = {"closure": "auto"}
    prepared = dfamin.BatchDevice(specs, outs)  # ctypes arguments built once
    tbat = time_device_steps(lambda: prepared.run(ctx, opts, stream), reps, warmup=1)
    tb = tbat["ms_p50"] * 1e-3
    print("[bench] batch: plain per-instance loop", file=sys.stderr, flush=True)
    for sp, o in zip(specs[:64], outs[:64]):  # warm-up
        dfamin.dfamin_minimize_device(ctx, *sp, o, opts=opts, stream=stream)
    torch.cuda.synchronize()
    passes = []
    for _ in range(plain_passes):
        t0 = time.perf_counter()
        for sp, o in zip(specs, outs):
            dfamin.dfamin_minimize_device(ctx, *sp, o, opts=opts, stream=stream)
        torch.cuda.synchronize()
        passes.append(time.perf_counter() - t0)
    tp = statistics.median(passes)
    print("[bench] batch: cpu oracle on a thread pool", file=sys.stderr, flush=True)
    cpu = cpu_baseline_batch(batch)
    return {"workload": "batch_mixed: 4096 DFAs, n log-uniform in [64, 65536], |Sigma| in 2..8, "
                        "25% permuted chains, seed 1, closure auto",
            "transitions": trans, "batched_ms": round(1e3 * tb, 3),
            "batched_ms_p50": tbat["ms_p50"], "batched_ms_p99": tbat["ms_p99"], "batched_repeats": reps,
            "plain_loop_ms": round(1e3 * tp, 3), "plain_loop_passes_ms": [round(1e3 * x, 1) for x in passes],
            "batched_value": trans / tb, "plain_loop_value": trans / tp, "ratio": round(tp / tb, 2),
            "cpu_baseline": cpu, "vs_cpu_pool": round((trans / tb) / cpu["value"], 1)}


def serving_run(ctx, seed, count, pool_size, load, threads=256, submitters=16):
    """Serving workload: Poisson arrivals of minimization requests at `load`
    times the saturation throughput measured on the same request pool.

    The arrival loop only schedules: each request is submitted at its
    scheduled arrival time by a worker thread, and its latency runs from
    that scheduled time to the end of its dfamin_wait.  Time a request
    spends behind other submits' input copies, or waiting for a free worker,
    therefore counts against it."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    from paper_2410_22764_amd import dfamin, workloads as W
    print(f"[bench] serving: generating a pool of {pool_size} requests", file=sys.stderr, flush=True)
    _, specs = W.serving_stream(seed, pool_size, 1.0)
    with ThreadPoolExecutor(max_workers=pool_threads()) as ex:  # numpy releases the GIL
        pool = list(ex.map(W.make_request, specs))
    opts = {"closure": "auto"}

    def closed_loop():
        # the whole pool at once, submitted by `submitters` threads
        def one(d):
            t = dfamin.dfamin_submit(ctx, d, opts)
            rc, _, _ = dfamin.dfamin_wait(ctx, t, d.n)
            assert rc == 0
        with ThreadPoolExecutor(max_workers=submitters) as ex:
            t0 = time.perf_counter()
            list(ex.map(one, pool))
            return len(pool) / (time.perf_counter() - t0)

    # saturation, closed loop; the first pass warms the library's caches
    # (device pool, page-locked staging, tuned tiles) and is not timed
    print("[bench] serving: saturation", file=sys.stderr, flush=True)
    closed_loop()
    sat = closed_loop()
    rate = load * sat
    arrivals, _ = W.serving_stream(seed + 1, count, rate)
    order = W.uniform_below(W.stream_key(seed, "serve", "order"), count, pool_size)
    lat = [0.0] * count
    lag = [0.0] * count
    done = [0.0] * count
    print(f"[bench] serving: {count} requests at {rate:.1f}/s", file=sys.stderr, flush=True)
    ex = ThreadPoolExecutor(max_workers=threads)
    start = time.perf_counter() + 0.01

    def job(i):
        d = pool[int(order[i])]
        t_sched = start + float(arrivals[i])
        t = dfamin.dfamin_submit(ctx, d, opts)
        lag[i] = time.perf_counter() - t_sched
        rc, _, _ = dfamin.dfamin_wait(ctx, t, d.n)
        assert rc == 0
        done[i] = time.perf_counter()
        lat[i] = done[i] - t_sched

    futs = []
    for i in range(count):
        target = start + float(arrivals[i])
        while True:
            now = time.perf_counter()
            if now >= target:
                break
            time.sleep(min(target - now, 0.0005))
        futs.append(ex.submit(job, i))
    for f in futs:
        f.result()
    ex.shutdown()
    span = float(arrivals[-1])
    wall = max(done) - start
    trans = sum(pool[int(o)].transitions for o in order)
    # every request crosses the host link: delta and bitmap in, one id per state out
    bin_ = sum(4 * d.n * d.k + d.accept.nbytes for d in pool) / len(pool)
    bout = sum(4 * d.n for d in pool) / len(pool)
    h2d, d2h = pinned_copy_rates()
    link = {"in_GBps_at_saturation": round(sat * bin_ / 1e9, 2), "out_GBps_at_saturation": round(sat * bout / 1e9, 2),
            "pinned_h2d_GBps": round(h2d, 2), "pinned_d2h_GBps": round(d2h, 2),
            "in_frac": round(sat * bin_ / 1e9 / h2d, 3),
            "note": "mean request input and output bytes of the pool times the saturation rate, against one "
                    "256 MiB page-locked copy in each direction"}
    return {"requests": count, "pool": pool_size, "offered_rate_per_s": round(rate, 2),
            "offered_rate_realised_per_s": round(count / span, 2),
            "saturation_dfas_per_s": round(sat, 2), "load": load, "dfas_per_s": round(count / wall, 2),
            "achieved_over_offered": round((count / wall) / (count / span), 4),
            "transitions_per_s": trans / wall,
            "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                           "p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                           "from": "scheduled arrival time"},
            "submit_lag_ms": {"p50": round(1e3 * float(np.percentile(lag, 50)), 3),
                              "p99": round(1e3 * float(np.percentile(lag, 99)), 3)},
            "client": f"arrivals scheduled by one thread, submitted by a pool of {threads} worker threads; "
                      f"saturation from {submitters} submitting threads, closed loop over the pool",
            "host_link": link}


def pinned_copy_rates(mib=256, reps=5):
    """GB/s of one page-locked host buffer copied to the device and back."""
    import torch
    h = torch.empty(mib << 20, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    rates = []
    for src, dst in ((h, d), (d, h)):
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            dst.copy_(src, non_blocking=True)
        e1.record()
        torch.cuda.synchronize()
        rates.append(reps * (mib << 20) / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del h, d
    return rates[0], rates[1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plain_large", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--method", default="signature", choices=["signature", "leader"],
                    help="refinement rounds: signature (Algorithm 4) or leader election (Algorithm 2)")
    ap.add_argument("--closure", default=None, choices=["off", "on", "auto"],
                    help="override the workload's closure policy")
    ap.add_argument("--queue", action="store_true",
                    help="queue hash-mode and doubling rounds on the device (DFAMIN_FLAG_QUEUE)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="no HIP-event kernel timing")
    ap.add_argument("--profile-steps", type=int, default=5, help="extra steps timed per kernel")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain and end-to-end legs")
    ap.add_argument("--requests", type=int, default=2000, help="serving: measured requests")
    ap.add_argument("--pool", type=int, default=256, help="serving: distinct pre-generated requests")
    ap.add_argument("--submitters", type=int, default=16,
                    help="serving: submitting threads of the closed-loop saturation pass")
    ap.add_argument("--load", type=float, default=0.7, help="serving: offered load / saturation")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the serving leg in the default run (0: none)")
    ap.add_argument("--serving-pool", type=int, default=256,
                    help="distinct requests of the serving leg in the default run")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB a few times (for scaling "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "launches": 5}))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; sharding across GPUs is "
                                   "described in the design notes but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2410_22764_amd import dfamin

    if args.workload == "serving":
        ctx = dfamin.dfamin_create(0)
        res = serving_run(ctx, args.seed, args.requests, args.pool, args.load, submitters=args.submitters)
        ctx.close()
        line = {"metric": METRIC, "value": res["transitions_per_s"], "unit": "transitions/s", "n_gpus": 1,
                "steps": args.requests, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
                "config": {"workload": "serving: Poisson stream, n log-uniform in [2^8, 2^22], |Sigma| in "
                                       "2..16, 20% permuted chains, closure auto", "seed": args.seed,
                           "parallelism": "single GPU"},
                "serving": res}
        print(json.dumps(line), flush=True)
        return

    spec = WORKLOADS[args.workload]
    print(f"[bench] generating {args.workload}", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ctx = dfamin.dfamin_create(0)
    closure = args.closure or spec["closure"]
    opts = dict(closure=closure, method=args.method, queue=args.queue)
    if spec["kind"] == "batch":
        from paper_2410_22764_amd import workloads as W
        batch = W.batch_mixed(seed=args.seed)
        specs, outs, keep = upload_batch(batch, dev)
        trans = sum(x.n * x.k for x in batch)
        cfg = {"workload": f"{args.workload}: {spec['desc']}", "instances": len(batch),
               "states": sum(x.n for x in batch), "transitions": trans, "seed": args.seed,
               "closure": closure, "method": args.method, "queue": args.queue, "parallelism": "single GPU"}

        prepared = dfamin.BatchDevice(specs, outs)  # ctypes arguments built once

        def step():
            prepared.run(ctx, opts, stream.cuda_stream)
            return prepared
    else:
        d = make_input(spec, args.seed)
        delta = torch.from_numpy(d.delta.view(np.int32)).to(dev)
        accept = torch.from_numpy(d.accept).to(dev)
        out = torch.empty(d.n, dtype=torch.int32, device=dev)
        trans = d.n * d.k
        cfg = {"workload": f"{args.workload}: {spec['desc']}", "n": d.n, "k": d.k, "seed": args.seed,
               "closure": closure, "method": args.method, "queue": args.queue, "parallelism": "single GPU"}
        if "paper" in spec:
            cfg["paper_context"] = spec["paper"]

        def step():
            return dfamin.dfamin_minimize_device(ctx, d.n, d.k, delta.data_ptr(), accept.data_ptr(), d.q0,
                                                 out.data_ptr(), opts=opts, stream=stream.cuda_stream)
    torch.cuda.synchronize()

    print("[bench] warmup", file=sys.stderr, flush=True)
    res = None
    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    print("[bench] timing", file=sys.stderr, flush=True)
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        res = step()
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = 1e3 * wall / args.steps
    value = trans / (wall / args.steps)
    # Kernel times come from separate steps with HIP events around every
    # launch (the events add a little time between kernels, so the timed
    # steps above run without them).
    stats = []
    if not args.no_profile:
        dfamin.dfamin_set_profiling(ctx, True)
        for _ in range(args.profile_steps):
            step()
        torch.cuda.synchronize()
        stats = dfamin.dfamin_get_kernel_stats(ctx)
        dfamin.dfamin_set_profiling(ctx, False)

    end_to_end = None
    if spec["kind"] != "batch" and not args.no_batch:
        # host buffers in and out: pageable -> pinned staging -> device and back
        print("[bench] end-to-end (host buffers)", file=sys.stderr, flush=True)
        dfamin.dfamin_minimize(ctx, d, opts)
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            dfamin.dfamin_minimize(ctx, d, opts)
        te = (time.perf_counter() - t0) / reps
        end_to_end = {"value": trans / te, "unit": "transitions/s", "ms_per_step": round(1e3 * te, 3),
                      "note": "host-resident input and output, PCIe transfers included"}

    roofline = None
    if stats:
        top = max(stats, key=lambda s: s["total_ms"])
        per_launch_ms = top["total_ms"] / max(top["launches"], 1)
        per_launch_bytes = top["alg_bytes"] / max(top["launches"], 1)
        achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
        traffic = load_traffic(top["name"], args.workload)
        roofline = {"bound": "hbm", "kernel": top["name"], "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": traffic,
                    "avg_launch_us": round(per_launch_ms * 1e3, 2),
                    "alg_bytes_per_launch": round(per_launch_bytes)}
        if traffic:
            # counter bytes per launch over the same launch time.  FETCH_SIZE
            # and WRITE_SIZE count what leaves the L2 for the memory fabric:
            # hits in the memory-side cache are included, so this rate is not
            # a fraction of HBM bandwidth (it can exceed a device copy's)
            roofline["counter_GBps"] = round(traffic / (per_launch_ms * 1e-3) / 1e9, 1)
            roofline["traffic_note"] = ("traffic: FETCH_SIZE x2 + WRITE_SIZE per launch (copy-calibrated), "
                                        "bytes between L2 and the memory fabric, memory-side cache hits included")
        if not args.no_batch:
            roofline["copy_GBps"] = round(copy_peak_gbps(), 1)
        if not args.no_batch and args.workload == "plain_large" and top["name"] == "signature":
            # each of C1's two signature launches runs over all n states,
            # gathering k block ids at random and updating one table word per
            # group (nearly every group is a single state)
            gps, aps = random_access_rates()
            n, k = spec["n"], spec["k"]
            tg, ta = k * n / gps, n / aps
            roofline["random_access"] = {
                "gathers_per_s": round(gps), "atomics_per_s": round(aps),
                "per_launch": {"gathers": k * n, "atomics": n},
                "floor_ms": {"overlapped": round(1e3 * max(tg, ta), 3), "serial": round(1e3 * (tg + ta), 3)},
                "avg_launch_ms": round(per_launch_ms, 3),
                "frac_of_floor": round(1e3 * max(tg, ta) / per_launch_ms, 3),
                "note": "rates from torch's index_select (4-byte gathers, 64 MiB table) and index_add_ "
                        "(8-byte atomics, 256 MiB table) on this GPU; floor = the launch's random "
                        "accesses at those rates"}
    batched = None
    configs = None
    if not args.no_batch and args.workload == "plain_large":
        configs = config_legs(ctx)
        batched = batched_vs_plain(ctx, args.seed)
    minimal = None
    if spec["kind"] != "batch" and not args.no_batch:
        # minimal DFA of the reachable part: host input, BFS + quotient on the GPU
        print("[bench] minimal DFA", file=sys.stderr, flush=True)
        dfamin.dfamin_minimal_dfa(ctx, d, opts)
        dfamin.dfamin_set_profiling(ctx, True)
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            m_n, _, _, m_info, _ = dfamin.dfamin_minimal_dfa(ctx, d, opts)
        tm = (time.perf_counter() - t0) / reps
        mstats = {x["name"]: x for x in dfamin.dfamin_get_kernel_stats(ctx)}
        dfamin.dfamin_set_profiling(ctx, False)
        minimal = {"ms_end_to_end": round(1e3 * tm, 3), "states": m_n, "reachable": m_info["reachable"],
                   "bfs_levels": m_info["bfs_levels"],
                   "bfs_ms": round(mstats["bfs_level"]["total_ms"] / reps, 3) if "bfs_level" in mstats else None,
                   "quotient_ms": round(mstats["quotient"]["total_ms"] / reps, 3) if "quotient" in mstats else None,
                   "note": "host input and output (PCIe included); bfs/quotient: HIP-event kernel time"}
    serving = None
    if args.serving_requests and args.workload == "plain_large":
        sctx = dfamin.dfamin_create(0)
        serving = serving_run(sctx, args.seed, args.serving_requests, args.serving_pool, args.load,
                              submitters=args.submitters)
        serving["workload"] = ("serving: Poisson stream, n log-uniform in [2^8, 2^22], |Sigma| in 2..16, "
                               "20% permuted chains, closure auto")
        sctx.close()
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(spec, args.seed)

    line = {
        "metric": METRIC, "value": value, "unit": "transitions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": cfg,
        "latency_ms": {"p50": round(1e3 * statistics.median(lat), 4),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 4)},
        "result": result_summary(res),
        "roofline": roofline,
        "kernels": [{"name": s["name"], "launches": s["launches"], "ms": round(s["total_ms"], 4),
                     "GBps": round(s["alg_bytes"] / (s["total_ms"] * 1e-3) / 1e9, 1) if s["total_ms"] > 0 else None}
                    for s in stats],
        "end_to_end": end_to_end,
        "minimal_dfa": minimal,
        "configs": configs,
        "batched": batched,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
