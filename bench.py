"""Benchmark: Roaring set operations on one MI355X.

Default workload (bitset-bandwidth): 2e4 bitmaps, each with 256 bitset
containers (keys 0..255, 8 KiB each, bit density U(0.2, 0.8)), about 42 GB
resident in HBM, generated on the device; 1e4 random pairs (ia != ib). One
step runs, for each of AND, OR, XOR, ANDNOT, the count-only form (fused op +
popcount, |A op B| per pair) over all pairs, plus the Jaccard index per pair.

value = algorithmic input bytes of the step / step time (GB/s), the metric's
"input GB/s"; container-pairs/s is reported beside it. Inputs are resident in
HBM before timing starts.

The dominant kernel's roofline entry is measured live: the library brackets
each launch of its kernels with HIP events on the launch stream
(rg_profile_*), and achieved = algorithmic bytes per launch / mean launch time.

cpu_baseline: the CPU oracle (plain two-pointer merges over sorted uint32
lists) timed on a bounded sample of the same work, rank 0 only, on one core
and on every host core (a thread pool over pairs: the oracle's C calls release
Python's lock); value is the all-core rate.

Other workloads (--workload): mixed (100 mixed bitmaps, 99 successive pairs,
four operations materialised with counts and Jaccard), array (1e5 array-array
pairs, Zipf sizes, materialised), dense-mat (materialised dense pairs),
batched (1e6 uneven pairs: plan, eager call, one call per pair, learned
dispatch), serve (k-way queries over a 1e5-bitmap index under Poisson
arrivals), dispatch (learned vs heuristic variant choice on held-out pairs),
wide (a 200-way union), access (batched membership and export to uint32),
canonical (non-P1 pool to P1), inplace (op= on mutable bitmaps).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
META_BYTES = 19  # key u16 + type u8 + card u32 + size u32 + off u64 per container
OPS4 = ("and", "or", "xor", "andnot")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bitmaps", type=int, default=20000)
    ap.add_argument("--keys", type=int, default=256)
    ap.add_argument("--pairs", type=int, default=10000)
    ap.add_argument("--cpu-pairs", type=int, default=48, help="dense: pairs in the oracle timing sample")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target single-core oracle time")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", type=int, default=2, help="pairs checked against the oracle before timing")
    ap.add_argument("--workload", choices=("dense", "mixed", "array", "dense-mat", "batched", "serve", "dispatch",
                                           "wide", "access", "canonical", "inplace"),
                    default="dense",
                    help="dense: the bitset-bandwidth headline; mixed / array: the small mixed and array-stress "
                         "pairs, materialised; batched: many uneven pairs, plan vs per-pair; serve: k-way "
                         "queries under Poisson arrivals, batched server vs one query at a time")
    ap.add_argument("--array-pairs", type=int, default=100000, help="array: pairs")
    ap.add_argument("--index", type=int, default=100000, help="serve: bitmaps in the index")
    ap.add_argument("--rates", default="2000,5000,10000,20000,50000,100000,200000",
                    help="serve: arrival rates (queries/s)")
    ap.add_argument("--one-max-rate", type=float, default=50000,
                    help="serve: highest rate also run one query at a time (it saturates far below)")
    ap.add_argument("--duration", type=float, default=2.0, help="serve: seconds of arrivals per rate")
    ap.add_argument("--max-batch", type=int, default=256, help="serve: most queries per step (batched mode)")
    ap.add_argument("--pool", type=int, default=16384, help="batched: bitmaps in the pool")
    ap.add_argument("--batched-pairs", type=int, default=1000000, help="batched: random pairs per step")
    ap.add_argument("--per-pair-sample", type=int, default=500, help="batched: pairs timed one call each")
    ap.add_argument("--dispatch-pairs", type=int, default=300, help="batched: pairs whose costs train the dispatcher")
    ap.add_argument("--dispatch-epochs", type=int, default=10, help="batched: dispatcher training epochs")
    ap.add_argument("--wide", type=int, default=200, help="wide: bitmaps in the union")
    ap.add_argument("--key-index", type=int, default=1, choices=(0, 1),
                    help="serve, wide: the pool carries key-presence indexes (built once, before timing)")
    ap.add_argument("--access-bitmaps", type=int, default=1000, help="access: bitmaps in the pool")
    ap.add_argument("--lookups", type=int, default=10000000, help="access: membership lookups per step")
    ap.add_argument("--canon-bitmaps", type=int, default=1000, help="canonical: bitmaps in the pool")
    ap.add_argument("--acc", type=int, default=64, help="inplace: mutable bitmaps")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES bytes (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is designed (keys partition the universe), not built", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(args.copy_probe // 8, dtype=torch.int64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copied {src.numel() * 8} bytes device to device", file=sys.stderr, flush=True)
        return None
    fn = {"dense": bench_dense, "mixed": bench_mixed, "array": bench_array, "dense-mat": bench_dense_mat,
          "batched": bench_batched, "serve": bench_serve, "dispatch": bench_dispatch, "wide": bench_wide,
          "access": bench_access, "canonical": bench_canonical, "inplace": bench_inplace}[args.workload]
    return fn(args)


# ---------------------------------------------------------------- shared helpers

def say(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)), "model": model}


def cpu_threads():
    # one GPU's share of the host: at most 16 workers, whatever the machine shows
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_baseline_tasks(tasks, work_units, unit, sample, target_s):
    """Times the oracle on `tasks` (zero-argument callables, each one oracle
    call over a slice of the sample): once to size the run, then repeated to
    about target_s on one thread, then the same repeated tasks on every usable
    core. work_units: the metric's units (bytes or container pairs) of one pass."""
    t0 = time.perf_counter()
    for f in tasks:
        f()
    t1 = time.perf_counter() - t0
    if t1 >= 0.5 * target_s:
        reps, t_single = 1, t1  # one pass is long enough to be the single-core measurement
    else:
        reps = max(1, min(100, int(round(target_s / max(t1, 1e-4)))))
        t0 = time.perf_counter()
        for _ in range(reps):
            for f in tasks:
                f()
        t_single = time.perf_counter() - t0
    nt = cpu_threads()
    work = tasks * reps
    with ThreadPoolExecutor(nt) as ex:
        t0 = time.perf_counter()
        list(ex.map(lambda f: f(), work))
        t_multi = time.perf_counter() - t0
    scale = 1e9 if unit == "GB/s" else 1.0
    return {"value": round(work_units * reps / t_multi / scale, 4), "unit": unit, "cores": nt, "kind": "oracle",
            "sample": f"{sample}; {reps} pass(es): {t_single:.1f} s on 1 core, {t_multi:.1f} s on {nt} threads",
            "single_core_value": round(work_units * reps / t_single / scale, 4), "host": host_info()}


def container_payload_bytes(h):
    """Payload bytes of every container of host pool arrays (array 2c, bitset 8192, run 4r)."""
    import numpy as np

    t = h["types"]
    sz = h["size"].astype(np.int64)
    return np.where(t == 1, 2 * sz, np.where(t == 2, 8192, 4 * sz))


def pair_stats(h, ia, ib):
    """Per pair: key counts of both bitmaps, matched containers, payload bytes
    of all containers of each side and of the matched containers of each side
    (host pool arrays h; pairs ia, ib)."""
    import numpy as np

    bb = h["bm_begin"].astype(np.int64)
    pay = container_payload_bytes(h)
    keys = h["keys"].astype(np.int64)
    n = len(ia)

    def side(ids):
        s = bb[ids.astype(np.int64)]
        cnt = bb[ids.astype(np.int64) + 1] - s
        pidx = np.repeat(np.arange(n, dtype=np.int64), cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        cidx = np.repeat(s, cnt) + (np.arange(int(cnt.sum()), dtype=np.int64) - start)
        return pidx, cidx, cnt

    pa, ca, na = side(ia)
    pb, cb, nb = side(ib)
    _, xa, xb = np.intersect1d((pa << 16) | keys[ca], (pb << 16) | keys[cb], assume_unique=True,
                               return_indices=True)
    f = lambda idx, w: np.bincount(idx, weights=w, minlength=n)
    return {"KA": na, "KB": nb, "matched": np.bincount(pa[xa], minlength=n), "payA": f(pa, pay[ca]),
            "payB": f(pb, pay[cb]), "payAm": f(pa[xa], pay[ca[xa]]), "payBm": f(pa[xa], pay[cb[xb]])}


def op_input_bytes(st, op):
    """Algorithmic input bytes per pair of one operation: the payloads it must
    read (matched containers; for union and symmetric difference also every
    one-sided container, for difference A's) plus 19 B of metadata per
    container of both bitmaps."""
    meta = META_BYTES * (st["KA"] + st["KB"])
    if op == "and":
        return st["payAm"] + st["payBm"] + meta
    if op in ("or", "xor"):
        return st["payA"] + st["payB"] + meta
    return st["payA"] + st["payBm"] + meta


def result_payload_bytes(out):
    """Payload bytes and container count of the results in an output arena."""
    import numpy as np

    n = int(out.c.n_containers)
    t = out.types[:n].cpu().numpy()
    sz = out.size[:n].cpu().numpy().astype(np.int64)
    return int(np.where(t == 1, 2 * sz, np.where(t == 2, 8192, 4 * sz)).sum()), n


def time_steps(step, steps, warmup):
    import torch

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


# ---------------------------------------------------------------- dense (headline)

def bench_dense(args):
    import numpy as np
    import torch

    import paper_1709_07821_amd as rg
    import synth

    dev = torch.device("cuda:0")
    ctx = rg.Context(0)
    stream = torch.cuda.current_stream()

    nb, nk, npairs = args.bitmaps, args.keys, args.pairs
    t0 = time.time()
    words = torch.empty(nb * nk * 1024, dtype=torch.int64, device=dev)
    chunk = 1000
    for b0 in range(0, nb, chunk):
        n = min(chunk, nb - b0)
        synth.dense_bitsets_device(words.data_ptr() + b0 * nk * 8192, b0, n, nk, stream.cuda_stream)
    P = rg.Pool.from_dense_words(ctx, words, nb, nk)
    torch.cuda.synchronize()
    say(f"generated {nb} x {nk} bitsets ({words.numel() * 8 / 1e9:.1f} GB) in {time.time() - t0:.1f} s")
    ia, ib = synth.random_pairs(nb, npairs, seed=synth.DENSE_SEED)
    tia = torch.from_numpy(ia.view(np.int32)).to(dev)
    tib = torch.from_numpy(ib.view(np.int32)).to(dev)
    cards = {op: torch.zeros(npairs, dtype=torch.int64, device=dev) for op in rg.OPS}
    jacc = torch.zeros(npairs, dtype=torch.float64, device=dev)

    def step():
        for op in OPS4:
            flags = rg.RG_FLAG_CARD | (rg.RG_FLAG_JACCARD if op == "and" else 0)
            ctx.check(rg.roaring_batch(ctx, op, P, P, tia, tib, flags, None, cards[op],
                                       jacc if op == "and" else None, stream))

    # correctness gate on a few pairs before timing (oracle, CPU)
    step()
    torch.cuda.synchronize()
    if args.check > 0:
        import oracle

        for p in range(args.check):
            a = synth.dense_bitmap_values(int(ia[p]), nk)
            b = synth.dense_bitmap_values(int(ib[p]), nk)
            for op in rg.OPS:
                got = int(cards[op][p].item())
                exp = oracle.count(op, a, b)
                assert got == exp, f"pair {p} {op}: gpu {got} oracle {exp}"
            assert float(jacc[p].item()) == oracle.jaccard(a, b)
        say(f"{args.check} pairs x 4 ops match the oracle")

    for _ in range(args.warmup):
        step()
    rg.profile_enable(ctx, True)
    rg.profile_reset(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = rg.profile_read(ctx)
    rg.profile_enable(ctx, False)
    ctx.sync()

    cont_pairs = npairs * nk                      # matched container pairs per op
    in_bytes_op = cont_pairs * 2 * (8192 + META_BYTES)
    ops_per_step = 4
    step_bytes = in_bytes_op * ops_per_step
    ms = dt / args.steps * 1e3
    value = step_bytes / (dt / args.steps) / 1e9
    cps = cont_pairs * ops_per_step / (dt / args.steps)

    # dominant kernel: the fused match-and-count kernel (one launch per count-only
    # call); its algorithmic bytes per launch are the two 8 KiB bitsets of every
    # matched container pair (every key matches in this workload)
    k = prof.get(("count-fused", False))
    roof = None
    if k and k["launches"]:
        alg_bytes = cont_pairs * 2 * 8192
        mean_s = k["ms"] / k["launches"] / 1e3
        ach = alg_bytes / mean_s / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                "kernel": "k_count_fused", "mean_launch_ms": round(mean_s * 1e3, 4),
                "launches": int(k["launches"]), "bytes_per_launch": int(alg_bytes)}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = dense_cpu_baseline(ia, ib, nk, args.cpu_pairs, args.cpu_seconds)

    line = {
        "metric": "input GB/s and container-pairs/sec for AND/OR/XOR/ANDNOT+card (% HBM peak)",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "dense-bitset pairs: 2e4 bitmaps x 256 bitset containers (U(0.2,0.8) density), "
                               "1e4 random pairs, |A op B| for AND/OR/XOR/ANDNOT + Jaccard",
                   "bitmaps": nb, "keys_per_bitmap": nk, "pairs": npairs, "parallelism": "single GPU"},
        "container_pairs_per_s": round(cps, 1),
        # algorithmic input bytes of the step over the step time
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        # the counters' bytes (FETCH_SIZE + WRITE_SIZE, scaled) of the dominant
        # kernel over its measured launch time, while they match its sources
        "pct_hbm_peak_measured": (round(100 * roof["traffic"] / (roof["mean_launch_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 2)
                                  if roof and roof["traffic"] else None),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def dense_cpu_baseline(ia, ib, nk, n_pairs, target_s):
    """The oracle, as it stands, on the first n_pairs pairs: 4 counts + Jaccard per pair."""
    import oracle
    import synth

    n_pairs = min(n_pairs, len(ia))
    sets = {}
    for p in range(n_pairs):
        for b in (int(ia[p]), int(ib[p])):
            if b not in sets:
                sets[b] = synth.dense_bitmap_values(b, nk)

    def task(p):
        def f():
            a, b = sets[int(ia[p])], sets[int(ib[p])]
            for op in OPS4:
                oracle.count(op, a, b)
            oracle.jaccard(a, b)
        return f

    tasks = [task(p) for p in range(n_pairs)]
    in_bytes = n_pairs * nk * 2 * (8192 + META_BYTES) * 4
    return cpu_baseline_tasks(tasks, in_bytes, "GB/s",
                              f"{n_pairs} of the pairs, 4 count-only ops + Jaccard each (two-pointer merges over "
                              f"sorted uint32)", target_s)


# ---------------------------------------------------------------- materialised pair workloads

def bench_pairs_materialised(args, bs, ia, ib, workload, metric_config):
    """Four operations materialised over the given pairs (result bitmaps in
    preallocated arenas; each op's first call sizes its arena), with the result
    cardinalities and the Jaccard index of every pair in the same calls. Every
    pair's result cardinality, fingerprint and Jaccard are checked against the
    oracle before timing. value = algorithmic input bytes of the step / step
    time; the roofline entry is the k-way evaluation kernel (union, symmetric
    difference, difference): result payload read and written per launch over
    its launch time."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg

    dev = torch.device("cuda:0")
    ctx = rg.Context(0)
    n = len(ia)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    h = rg.Pool.host_arrays(bs.values, bs.offsets)[3]
    tia = torch.from_numpy(ia.view(np.int32)).to(dev)
    tib = torch.from_numpy(ib.view(np.int32)).to(dev)
    arenas, cards, jaccs = {}, {}, {}
    for op in OPS4:
        arenas[op], cards[op], jaccs[op] = rg.batch(ctx, op, P, P, tia, tib, materialize=True, card=True,
                                                    jaccard=True)
    torch.cuda.synchronize()
    # correctness gate: every pair's count, fingerprint and Jaccard against the oracle
    for op in OPS4:
        c_exp, d_exp, j_exp = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib,
                                           want_digest=True, want_jaccard=True)
        dig = rg.rg_pool_digest(ctx, arenas[op].as_pool()).cpu().numpy().view(np.uint64)[:n]
        assert np.array_equal(cards[op].cpu().numpy().view(np.uint64), c_exp), op
        assert np.array_equal(dig, d_exp), op
        assert np.array_equal(jaccs[op].cpu().numpy(), j_exp), op
    say(f"{n} pairs x 4 ops materialised: counts, fingerprints and Jaccard match the oracle")

    # the timed calls write into the arenas and output vectors of the gate
    # (a caller preallocates them; the library call does all the work)
    mat_flags = rg.RG_FLAG_MATERIALIZE | rg.RG_FLAG_CARD | rg.RG_FLAG_JACCARD

    def step():
        for op in OPS4:
            ctx.check(rg.roaring_batch(ctx, op, P, P, tia, tib, mat_flags, arenas[op], cards[op], jaccs[op]))

    dt = time_steps(step, args.steps, args.warmup)
    rg.profile_enable(ctx, True)
    rg.profile_reset(ctx)
    dt_prof = time_steps(step, args.steps, 0)
    prof = rg.profile_read(ctx)
    rg.profile_enable(ctx, False)

    st = pair_stats(h, ia, ib)
    in_bytes = {op: float(op_input_bytes(st, op).sum()) for op in OPS4}
    out_pay = {op: result_payload_bytes(arenas[op]) for op in OPS4}
    out_bytes = {op: out_pay[op][0] + META_BYTES * out_pay[op][1] for op in OPS4}
    step_in = sum(in_bytes.values())
    matched = int(st["matched"].sum())
    # roofline: the k-way evaluation step (the one-wave array and bitset kernels
    # and the workgroup kernel, one launch each per call) reads the containers of every
    # result key of the union, symmetric difference and difference and writes
    # the result; its duration is the two launches'
    kw = dict(prof.get(("kway-eval", True)) or {"ms": 0.0, "launches": 0})
    for extra in ("kway-small", "kway-bb"):
        if prof.get((extra, True)):
            kw["ms"] += prof[(extra, True)]["ms"]
    roof = None
    if kw and kw["launches"]:
        kw_bytes = sum(float((st["payA"] + st["payB"]).sum()) for op in ("or", "xor")) + \
            float((st["payA"] + st["payBm"]).sum()) + sum(out_pay[op][0] for op in ("or", "xor", "andnot"))
        kw_bytes *= args.steps
        ach = kw_bytes / (kw["ms"] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": "k_kw_small + k_kw_bb + k_kw_eval (k-way evaluation step)",
                "mean_launch_ms": round(kw["ms"] / kw["launches"], 4), "launches": int(kw["launches"]),
                "bytes_per_launch": int(kw_bytes / kw["launches"]),
                "share_of_step": round(kw["ms"] / (dt_prof * 1e3 * args.steps), 3)}
    # class 3 materialised is the one-wave array kernel on intersections
    kernels = {f"{'wave-array' if k == ('merge', True) else k[0]}{'-mat' if k[1] else ''}": round(v["ms"] / args.steps, 4)
               for k, v in prof.items() if v["ms"]}

    cpu = None
    if not args.no_cpu_baseline:
        nt = cpu_threads()
        chunk = max(1, n // (4 * nt))

        def task(op, s0):
            s1 = min(n, s0 + chunk)
            return lambda: oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia[s0:s1], ib[s0:s1],
                                        want_digest=True, want_jaccard=True)

        tasks = [task(op, s0) for op in OPS4 for s0 in range(0, n, chunk)]
        cpu = cpu_baseline_tasks(tasks, step_in, "GB/s",
                                 f"all {n} pairs, 4 ops each materialised (sorted result list and its container-"
                                 f"view fingerprint) with the count and Jaccard", args.cpu_seconds)

    line = {
        "metric": "input GB/s and container-pairs/sec for AND/OR/XOR/ANDNOT+card (% HBM peak)",
        "value": round(step_in / dt / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": dict(metric_config, workload=workload, parallelism="single GPU"),
        "container_pairs_per_s": round(4 * matched / dt, 1),
        "pairs_per_s": round(4 * n / dt, 1),
        "input_bytes_per_op": {op: int(v) for op, v in in_bytes.items()},
        "output_bytes_per_op": out_bytes,
        "pct_hbm_peak": round(100 * (step_in + sum(out_bytes.values())) / dt / 1e9 / HBM_PEAK_GBS, 3),
        "cache_resident": True,
        "kernel_ms_per_step": kernels,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def bench_mixed(args):
    import synth

    bs = synth.mixed_small()
    ia, ib = synth.consecutive_pairs(len(bs))
    say(f"mixed small: {len(bs)} bitmaps, {len(bs.values)} values, {len(ia)} successive pairs")
    bench_pairs_materialised(args, bs, ia, ib,
                             "mixed small: 100 bitmaps over [0, 2^26), 1e3..5e4 values, 40/30/30 sparse/dense/"
                             "run, 99 successive pairs; AND/OR/XOR/ANDNOT materialised + counts + Jaccard",
                             {"bitmaps": len(bs), "pairs": len(ia)})


def bench_array(args):
    import synth

    bs, ia, ib = synth.array_stress(n_pairs=args.array_pairs)
    say(f"array stress: {len(ia)} pairs, {len(bs.values)} values")
    bench_pairs_materialised(args, bs, ia, ib,
                             f"array stress: {len(ia)} pairs of sorted uint16 arrays, sizes Zipf(1.2) on "
                             f"[1, 4096], ratio <= 1000; AND/OR/XOR/ANDNOT materialised + counts + Jaccard",
                             {"pairs": len(ia)})


def bench_dense_mat(args):
    """Materialised AND/OR/XOR/ANDNOT of dense bitset pairs: the dense-bitset
    recipe at a tenth of its pairs (--bitmaps 2000 --pairs 1000 by default for
    this workload), every result written into a preallocated arena (each op's
    first call sizes it). GB/s = (input bytes + result payload bytes) / time."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    dev = torch.device("cuda:0")
    ctx = rg.Context(0)
    stream = torch.cuda.current_stream()
    nb = args.bitmaps if args.bitmaps != 20000 else 2000
    npairs = args.pairs if args.pairs != 10000 else 1000
    nk = args.keys
    words = torch.empty(nb * nk * 1024, dtype=torch.int64, device=dev)
    for b0 in range(0, nb, 1000):
        synth.dense_bitsets_device(words.data_ptr() + b0 * nk * 8192, b0, min(1000, nb - b0), nk, stream.cuda_stream)
    P = rg.Pool.from_dense_words(ctx, words, nb, nk)
    ia, ib = synth.random_pairs(nb, npairs, seed=synth.DENSE_SEED)
    tia = torch.from_numpy(ia.view(np.int32)).to(dev)
    tib = torch.from_numpy(ib.view(np.int32)).to(dev)
    arenas = {}
    cards = {}
    for op in rg.OPS:
        arenas[op], cards[op], _ = rg.batch(ctx, op, P, P, tia, tib, materialize=True, card=True)
    torch.cuda.synchronize()
    # correctness gate: two pairs of every op against the oracle (fingerprints)
    for op in rg.OPS:
        dig = rg.rg_pool_digest(ctx, arenas[op].as_pool()).cpu().numpy().view(np.uint64)
        for p in range(2):
            exp = oracle.op(op, synth.dense_bitmap_values(int(ia[p]), nk), synth.dense_bitmap_values(int(ib[p]), nk))
            assert int(dig[p]) == oracle.digest(exp), (op, p)
    say(f"{nb} x {nk} bitsets, {npairs} pairs; 2 pairs x 4 ops match the oracle")
    out_bytes = {op: int(arenas[op].c.payload_used) for op in rg.OPS}

    def step():
        for op in rg.OPS:
            ctx.check(rg.roaring_batch(ctx, op, P, P, tia, tib, rg.RG_FLAG_MATERIALIZE | rg.RG_FLAG_CARD, arenas[op],
                                       cards[op]))

    dt = time_steps(step, args.steps, args.warmup)
    in_bytes = 4 * npairs * nk * 2 * 8192
    total = in_bytes + sum(out_bytes.values())
    line = {
        "metric": "materialised AND/OR/XOR/ANDNOT of dense bitset pairs, input + result GB/s",
        "value": round(total / dt / 1e9, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"dense-bitset pairs, materialised: {nb} bitmaps x {nk} bitset containers, "
                               f"{npairs} random pairs, four operations", "bitmaps": nb, "pairs": npairs,
                   "parallelism": "single GPU"},
        "result_payload_bytes": out_bytes,
        "pct_hbm_peak": round(100 * total / dt / 1e9 / HBM_PEAK_GBS, 2),
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- batched uneven pairs

def bench_batched(args):
    """Many uneven pairs: |A n B| and Jaccard for every pair of a random pair list
    over a pool of mixed bitmaps (lognormal cardinality, median 1e4, sigma 2,
    clipped to [10, 1e7], over [0, 2^32), 40/30/30 sparse/dense/run with a
    256-key hot set). Executions of the same step, same results: one library
    call per pair; one batched call (asynchronous, fused match-and-count
    kernel); a plan (persistent work-stealing kernel, autotuned, replayed as a
    hipGraph), with heuristic and with learned dispatch."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    dev = torch.device("cuda:0")
    ctx = rg.Context(0)
    seed = synth.SEED_BASE + 3
    t0 = time.time()
    bs = build_sets_threaded(batched_pool_gen(args.pool), args.pool)
    h = rg.Pool.host_arrays(bs.values, bs.offsets)[3]
    P = rg.Pool.from_host_arrays(h)
    ia, ib = synth.random_pairs(args.pool, args.batched_pairs, seed)
    n = len(ia)
    tia = torch.from_numpy(ia.view(np.int32)).to(dev)
    tib = torch.from_numpy(ib.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    say(f"pool of {args.pool} bitmaps, {len(bs.values)} values, {P.c.n_containers} containers, "
        f"{n} pairs, built in {time.time() - t0:.1f} s")

    # eager batched call (asynchronous: one fused match-and-count kernel)
    _, c_e, j_e = rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True)
    torch.cuda.synchronize()
    ctx.sync()
    c_e, j_e = c_e.cpu().numpy().view(np.uint64), j_e.cpu().numpy()
    for p in range(0, n, max(1, n // 16)):
        a, b = bs[int(ia[p])], bs[int(ib[p])]
        assert int(c_e[p]) == oracle.count("and", a, b) and j_e[p] == oracle.jaccard(a, b), p
    say("16 sampled pairs match the oracle")

    eager_s = time_steps(lambda: rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True),
                         args.steps, 1)
    # the same calls timed per kernel: the fused kernel's launch time, and the
    # matched container pairs it counts while timed (its profile items)
    rg.profile_enable(ctx, True)
    rg.profile_reset(ctx)
    time_steps(lambda: rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True),
               args.steps, 0)
    prof = rg.profile_read(ctx)
    rg.profile_enable(ctx, False)
    kf = prof.get(("count-fused", False), {"ms": 0, "launches": 0, "items": 0})
    matched = int(kf["items"]) // max(1, int(kf["launches"]))
    say(f"eager batched: {eager_s * 1e3:.2f} ms/step; {matched} matched container pairs per step")
    # the same eager call on a pool that carries packed metadata records
    # (rg_pool_pack_meta); the plans below reuse them
    t_p = time.perf_counter()
    P.pack_meta(ctx)
    torch.cuda.synchronize()
    pack_s = time.perf_counter() - t_p
    eager_packed_s = time_steps(lambda: rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True,
                                                 jaccard=True), args.steps, 1)
    _, c_p, j_p = rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True)
    torch.cuda.synchronize()
    assert np.array_equal(c_p.cpu().numpy().view(np.uint64), c_e) and np.array_equal(j_p.cpu().numpy(), j_e)
    say(f"eager batched, packed metadata: {eager_packed_s * 1e3:.2f} ms/step (packing once: {pack_s * 1e3:.1f} ms), "
        f"results equal")

    # plan: tuned, captured, replayed on a side stream
    st = torch.cuda.Stream()
    pl = rg.Plan(ctx, "and", P, P, tia, tib, card=True, jaccard=True, stream=st)
    pl.tune(stream=st, reps=1)
    pl.capture(st)
    torch.cuda.synchronize()
    plan_s = time_steps(lambda: pl.execute(stream=st), args.steps, args.warmup)
    assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), c_e)
    assert np.array_equal(pl.jacc.cpu().numpy(), j_e)
    info = pl.info()
    say(f"plan (graph, {info}): {plan_s * 1e3:.2f} ms/step, results equal to the eager call")

    # learned dispatch: cost samples measured by the kernels on a subset of the
    # pairs, the network trained on the GPU, installed, and a new plan timed
    t_s = time.perf_counter()
    sub_n = min(args.dispatch_pairs, n)
    X, T, M = rg.dispatch_samples(ctx, P, P, tia[:sub_n], tib[:sub_n])
    # plus array pairs of every size (Zipf), so that larger arrays are covered too
    zs, za, zb = synth.array_stress(n_pairs=4000)
    ZP = rg.Pool.from_sets(zs.values, zs.offsets)
    X2, T2, M2 = rg.dispatch_samples(ctx, ZP, ZP, torch.from_numpy(za.view(np.int32)).to(dev),
                                     torch.from_numpy(zb.view(np.int32)).to(dev))
    X, T, M = torch.cat([X, X2]), torch.cat([T, T2]), torch.cat([M, M2])
    params, losses = rg.dispatch_train(ctx, X, T, M, epochs=args.dispatch_epochs, batch=4096, lr=2e-3, seed=11)
    rg.dispatch_set_mlp(ctx, params)
    losses = losses.cpu().numpy()
    say(f"dispatcher: {int(M.any(1).sum())} sampled container pairs, loss {losses[0]:.3f} -> {losses[-1]:.3f}, "
        f"{time.perf_counter() - t_s:.1f} s")
    pl2 = rg.Plan(ctx, "and", P, P, tia, tib, card=True, jaccard=True, stream=st)
    pl2.tune(stream=st, reps=1)
    pl2.capture(st)
    torch.cuda.synchronize()
    learned_s = time_steps(lambda: pl2.execute(stream=st), args.steps, args.warmup)
    assert np.array_equal(pl2.cards.cpu().numpy().view(np.uint64), c_e)
    assert np.array_equal(pl2.jacc.cpu().numpy(), j_e)
    info2 = pl2.info()
    pl2.close()
    ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)
    say(f"plan with learned dispatch ({info2}): {learned_s * 1e3:.2f} ms/step, results equal")

    # one call per pair, on a sample
    k = min(args.per_pair_sample, n)
    one_c = torch.zeros(1, dtype=torch.int64, device=dev)
    one_j = torch.zeros(1, dtype=torch.float64, device=dev)
    flags = rg.RG_FLAG_CARD | rg.RG_FLAG_JACCARD

    def per_pair():
        for p in range(k):
            ctx.check(rg.roaring_batch(ctx, "and", P, P, tia[p:p + 1], tib[p:p + 1], flags, None, one_c, one_j))

    pp_s = time_steps(per_pair, 1, 0) / k * n
    say(f"one call per pair: {pp_s / n * 1e6:.1f} us/pair on {k} pairs -> {pp_s * 1e3:.1f} ms/step")
    pl.close()

    # roofline: the eager call's fused match-and-count kernel; algorithmic bytes
    # per launch = bytes per matched container pair (payloads of both containers,
    # 19 B metadata per container of both bitmaps, averaged over a sample of the
    # pairs) x the matched container pairs of the launch
    samp = np.random.default_rng(7).choice(n, size=min(4000, n), replace=False)
    stt = pair_stats(h, ia[samp], ib[samp])
    per_matched = float(op_input_bytes(stt, "and").sum()) / max(1, int(stt["matched"].sum()))
    roof = None
    if kf["launches"]:
        alg = per_matched * matched
        mean_s = kf["ms"] / kf["launches"] / 1e3
        roof = {"bound": "hbm", "achieved": round(alg / mean_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(alg / mean_s / 1e9 / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic("k_count_fused_batched_uneven.md"),
                "kernel": "k_count_fused (eager batched call)", "mean_launch_ms": round(mean_s * 1e3, 3),
                "launches": int(kf["launches"]), "bytes_per_launch": int(alg),
                "bytes_per_matched_pair": round(per_matched, 1),
                "bytes_per_matched_pair_sample": f"{len(samp)} random pairs"}
    cpu = None
    if not args.no_cpu_baseline:
        m = min(len(samp), 4000)
        sa, sb = ia[samp[:m]], ib[samp[:m]]
        nt = cpu_threads()
        chunk = max(1, m // (4 * nt))
        tasks = [(lambda s0=s0: oracle.pairs("and", bs.values, bs.offsets, bs.values, bs.offsets, sa[s0:s0 + chunk],
                                             sb[s0:s0 + chunk], want_jaccard=True)) for s0 in range(0, m, chunk)]
        cpu = cpu_baseline_tasks(tasks, float(stt["matched"][:m].sum()), "container-pairs/s",
                                 f"{m} random pairs of the step, |A n B| + Jaccard each", args.cpu_seconds)

    line = {
        "metric": "container-pairs/sec, batched count + Jaccard over uneven pairs",
        "value": round(matched / plan_s, 1), "unit": "container-pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(plan_s * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"batched uneven pairs: pool of {args.pool} mixed bitmaps (lognormal card, median "
                               f"1e4, sigma 2, [10, 1e7], universe 2^32), {n} random pairs, |A n B| + Jaccard",
                   "pool": args.pool, "pairs": n, "parallelism": "single GPU"},
        "pairs_per_s": round(n / plan_s, 1),
        "matched_container_pairs": int(matched),
        "plan": info,
        "eager_batched_ms": round(eager_s * 1e3, 3),
        "eager_batched_packed_ms": round(eager_packed_s * 1e3, 3),
        "per_pair_ms_extrapolated": round(pp_s * 1e3, 3),
        "speedup_plan_vs_per_pair": round(pp_s / plan_s, 2),
        "speedup_plan_vs_eager": round(eager_s / plan_s, 3),
        "plan_learned_dispatch_ms": round(learned_s * 1e3, 3),
        "plan_learned": info2,
        "speedup_learned_vs_heuristic": round(plan_s / learned_s, 3),
        "dispatcher_loss": [round(float(losses[0]), 4), round(float(losses[-1]), 4)],
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def batched_pool_gen(n_pool):
    """The batched workload's bitmap i (i < n_pool): mixed recipe over [0, 2^32)
    with a 256-key hot set, cardinality lognormal (median 1e4, sigma 2, clipped
    to [10, 1e7])."""
    import synth

    seed = synth.SEED_BASE + 3
    hot = synth.hot_keys(seed, 256, 1 << 16)
    cards = [synth.lognormal_card(i, 1e4, 2.0, 10, 10 ** 7, seed) for i in range(n_pool)]
    return lambda i: synth.mixed_bitmap(seed, i, cards[i], 32, hot)


def serve_index_gen(n_index):
    """The serving index's bitmap i (i < n_index): mixed recipe over [0, 2^26)
    with a 32-key hot set, cardinality lognormal (median 5e4, sigma 1, clipped
    to [1e3, 1e6])."""
    import synth

    seed = synth.SEED_BASE + 4
    hot = synth.hot_keys(seed, 32, 1 << 10)
    cards = [synth.lognormal_card(i, 5e4, 1.0, 1000, 10 ** 6, seed) for i in range(n_index)]
    return lambda i: synth.mixed_bitmap(seed, i, cards[i], 26, hot)


def build_sets_threaded(gen, n):
    """BitmapSet of gen(0) .. gen(n - 1), generated by a thread pool (the
    generator's C calls release Python's lock)."""
    import synth

    t0 = time.time()
    with ThreadPoolExecutor(cpu_threads()) as ex:
        lists = list(ex.map(gen, range(n), chunksize=64))
    say(f"generated {n} bitmaps in {time.time() - t0:.1f} s")
    return synth.BitmapSet.from_list(lists)


def build_pool_threaded(gen, n, chunk=2000):
    """Host pool arrays of bitmaps gen(0) .. gen(n - 1), built chunk by chunk
    in a thread pool and joined (offsets shifted), so the values of all
    bitmaps never have to be held at once."""
    import numpy as np

    import paper_1709_07821_amd as rg
    import synth

    def part(c0):
        bs = synth.BitmapSet.from_list([gen(i) for i in range(c0, min(n, c0 + chunk))])
        return rg.Pool.host_arrays(bs.values, bs.offsets)[3]

    t0 = time.time()
    with ThreadPoolExecutor(cpu_threads()) as ex:
        parts = list(ex.map(part, range(0, n, chunk)))
    say(f"generated and built {n} bitmaps in {len(parts)} chunks, {time.time() - t0:.1f} s")
    c_base = np.cumsum([0] + [len(p["keys"]) for p in parts])
    p_base = np.cumsum([0] + [len(p["payload"]) for p in parts])
    out = {"bm_begin": np.concatenate([p["bm_begin"][:-1] + np.uint64(c_base[i]) for i, p in enumerate(parts)] +
                                      [np.array([c_base[-1]], np.uint64)]),
           "off": np.concatenate([p["off"] + np.uint64(p_base[i]) for i, p in enumerate(parts)])}
    for k in ("keys", "types", "card", "size", "payload", "bm_card", "bm_wbytes"):
        out[k] = np.concatenate([p[k] for p in parts])
        for p in parts:
            p[k] = None
    return out


# ---------------------------------------------------------------- learned dispatch

def dispatch_training_set(ctx):
    """Cost samples measured by the kernels on training pools (seeds not used
    for evaluation): array stress, mixed bitmaps, array-bitset pairs."""
    import numpy as np
    import torch

    import paper_1709_07821_amd as rg
    import synth

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
    parts = []
    for bs, ia, ib in (synth.array_stress(n_pairs=20000, seed=555),
                       (lambda m: (m, *synth.consecutive_pairs(len(m))))(synth.mixed_small(n_bitmaps=40, seed=556)),
                       synth.uniform_size_pairs(3000, 557, (500, 4096), (4097, 30000))):
        P = rg.Pool.from_sets(bs.values, bs.offsets)
        parts.append(rg.dispatch_samples(ctx, P, P, t(ia), t(ib)))
    return tuple(torch.cat([p[i] for p in parts]) for i in range(3))


def dispatch_eval_sets():
    """Held-out evaluation pairs: name -> (BitmapSet, ia, ib)."""
    import synth

    mx = synth.mixed_small(n_bitmaps=100)
    return {"array stress (1e5 pairs, Zipf sizes)": synth.array_stress(n_pairs=100000),
            "mid-size arrays (9..62 vs 9..300 values, 5e4 pairs)": synth.uniform_size_pairs(50000, 558, (9, 62),
                                                                                              (9, 300)),
            "array-bitset (500..4096 vs 4097..30000 values, 2e4 pairs)":
                synth.uniform_size_pairs(20000, 559, (500, 4096), (4097, 30000)),
            "mixed small (99 successive pairs)": (mx, *synth.consecutive_pairs(len(mx)))}


def bench_dispatch(args):
    """What the learned dispatcher gains over the size-ratio heuristic it
    replaces, on held-out pairs: the network is trained on kernel-measured
    costs of other pools, installed, and the count-only batched call (|A n B|
    per pair) is timed with heuristic, learned and the best hand-tuned
    heuristic thresholds (thread-size threshold x galloping ratio grid);
    results are identical in every case."""
    import numpy as np
    import torch

    import paper_1709_07821_amd as rg

    ctx = rg.Context(0)
    t0 = time.perf_counter()
    X, T, M = dispatch_training_set(ctx)
    params, losses = rg.dispatch_train(ctx, X, T, M, epochs=30, batch=4096, lr=2e-3, seed=11)
    losses = losses.cpu().numpy()
    say(f"dispatcher: {X.shape[0]} samples, per variant {M.sum(0).tolist()}, loss {losses[0]:.3f} -> "
        f"{losses[-1]:.3f}, {time.perf_counter() - t0:.1f} s")
    rows = {}
    for name, (bs, ia, ib) in dispatch_eval_sets().items():
        P = rg.Pool.from_sets(bs.values, bs.offsets)
        a = torch.from_numpy(ia.view(np.int32)).cuda()
        b = torch.from_numpy(ib.view(np.int32)).cuda()
        cards = torch.zeros(len(ia), dtype=torch.int64, device="cuda")

        def run():
            ctx.check(rg.roaring_batch(ctx, "and", P, P, a, b, rg.RG_FLAG_CARD, None, cards, None))

        ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)
        ctx.set_thresholds(64, 8)
        heur = time_steps(run, 10, 2)
        ref = cards.clone()
        best, best_set = heur, (64, 8)
        for tm in (0, 4, 16, 32, 62):
            for gr in (8, 16, 64, 256):
                ctx.set_thresholds(gr, tm)
                ms = time_steps(run, 10, 1)
                assert torch.equal(cards, ref)
                if ms < best:
                    best, best_set = ms, (gr, tm)
        ctx.set_thresholds(64, 8)
        rg.dispatch_set_mlp(ctx, params)
        learned = time_steps(run, 10, 2)
        assert torch.equal(cards, ref), name
        ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)
        rows[name] = {"pairs": len(ia), "heuristic_ms": round(heur * 1e3, 4), "learned_ms": round(learned * 1e3, 4),
                      "tuned_heuristic_ms": round(best * 1e3, 4),
                      "tuned_setting": {"gallop_ratio": best_set[0], "thread_max": best_set[1]},
                      "gain_learned_vs_heuristic": round(heur / learned, 3),
                      "learned_vs_tuned_heuristic": round(best / learned, 3)}
        say(f"{name}: {rows[name]}")
    first = next(iter(rows.values()))
    line = {
        "metric": "speedup of learned dispatch over the size-ratio heuristic, count-only batch, held-out pairs",
        "value": first["gain_learned_vs_heuristic"], "unit": "x", "n_gpus": 1, "steps": 10, "warmup": 2,
        "ms_per_step": first["learned_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "learned dispatch: 12-64-64-6 network trained on kernel-measured costs of array-"
                               "stress, mixed and array-bitset pools (other seeds), evaluated on held-out pairs",
                   "parallelism": "single GPU"},
        "training_samples": int(X.shape[0]), "loss": [round(float(losses[0]), 3), round(float(losses[-1]), 3)],
        "workloads": rows,
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- serving

def bench_serve(args):
    """k-way AND/OR queries over a device-resident index under open-loop Poisson
    arrivals. Index: mixed bitmaps over [0, 2^26) (40/30/30 sparse/dense/run,
    32-key hot set), cardinality lognormal (median 5e4, sigma 1, clipped to
    [1e3, 1e6]). Mix: 40 % k-AND, 40 % k-OR (both materialised), 20 %
    count-only (half AND, half OR); k uniform in 2..32; ids uniform without
    replacement. Each rate runs the continuous-batching server (up to
    --max-batch queries per step, two steps in flight) and, up to
    --one-max-rate, one query at a time. Achieved rate = queries / the server's
    span (replay start to the last completion; the client's marshalling of the
    query list is outside it)."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    ctx = rg.Context(0)
    seed = synth.SEED_BASE + 4
    t0 = time.time()
    gen = serve_index_gen(args.index)
    h = build_pool_threaded(gen, args.index)
    P = rg.Pool.from_host_arrays(h)
    torch.cuda.synchronize()
    kidx_ms = None
    if args.key_index:
        t1 = time.time()
        P.key_index(ctx)
        torch.cuda.synchronize()
        kidx_ms = (time.time() - t1) * 1e3
    n_values = int(h["bm_card"].sum())
    say(f"index of {args.index} bitmaps, {n_values} values, {P.c.n_containers} containers, "
        f"{len(h['payload']) / 1e9:.1f} GB payload, built in {time.time() - t0:.1f} s"
        + (f" (key-presence indexes {kidx_ms:.1f} ms)" if args.key_index else ""))
    rng = np.random.default_rng(seed)

    def make_queries(n):
        qs = []
        for _ in range(n):
            u = rng.random()
            k = int(rng.integers(2, 33))
            ids = rng.choice(args.index, size=k, replace=False).astype(np.uint32)
            if u < 0.4:
                qs.append(("and", ids, True))
            elif u < 0.8:
                qs.append(("or", ids, True))
            else:
                qs.append(("and" if u < 0.9 else "or", ids, False))
        return qs

    # correctness gate: a sample against the oracle (bitmaps regenerated on the host)
    sample = make_queries(12)
    srv = rg.Server(ctx, P, arena_bytes=4 << 30, max_batch=args.max_batch, max_inflight=2)
    _, c_s, d_s = srv.replay(sample, np.zeros(len(sample), np.uint64), digest=True)
    srv.stop()
    for i, (op, ids, mat) in enumerate(sample):
        e = oracle.kway(op, [gen(int(j)) for j in ids])
        assert c_s[i] == len(e) and d_s[i] == (oracle.digest(e) if mat else 0), i
    say("12 sampled queries match the oracle")

    rows = []
    for lam in [float(x) for x in args.rates.split(",")]:
        n = max(1, int(lam * args.duration))
        qs = make_queries(n)
        gaps = rng.exponential(1.0 / lam, n)
        arrival = (np.cumsum(gaps) * 1e9).astype(np.uint64)
        row = {"rate_qps": lam, "queries": n}
        modes = [("batched", args.max_batch, 2)] + ([("one_at_a_time", 1, 1)] if lam <= args.one_max_rate else [])
        for mode, mb, mi in modes:
            srv = rg.Server(ctx, P, arena_bytes=4 << 30, max_batch=mb, max_inflight=mi)
            # served as a client would: cardinalities and result views, no fingerprints
            lat, c, _ = srv.replay(qs, arrival)
            # the server's span: from the replay's start (arrival offsets count
            # from it) to the last completion, arrival + latency
            wall = float((arrival + lat).max()) / 1e9
            st = srv.stop()
            if mode == "batched":
                ref = c
            else:
                assert np.array_equal(c, ref), "cardinalities differ between modes"
            row[mode] = {"achieved_qps": round(n / wall, 1), "p50_us": round(float(np.percentile(lat, 50)) / 1e3, 1),
                         "p99_us": round(float(np.percentile(lat, 99)) / 1e3, 1),
                         "mean_batch": round(st["mean_batch"], 2), "steps": st["steps"]}
            say(f"rate {lam:.0f}/s {mode}: {row[mode]}")
        rows.append(row)
    best = max(r["batched"]["achieved_qps"] for r in rows)

    # roofline of the evaluation step on queries of the same mix, one
    # roaring_multi call each (its kernels read every container of each result
    # key and write the result): bytes from the host pool arrays
    roof, cpu = serve_roofline_and_cpu(args, ctx, P, h, make_queries(64), gen)
    line = {
        "metric": "queries/sec and p50/p99 latency, k-way AND/OR serving (continuous batching)",
        "value": best, "unit": "queries/s", "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"serving: index of {args.index} mixed bitmaps over [0, 2^26) (lognormal card, median "
                               f"5e4, sigma 1), Poisson arrivals, 40% k-AND / 40% k-OR materialised, 20% "
                               f"count-only, k in 2..32", "index": args.index, "duration_s": args.duration,
                   "key_index": bool(args.key_index), "parallelism": "single GPU"},
        "index_values": n_values, "index_containers": int(P.c.n_containers),
        "key_index_build_ms": None if kidx_ms is None else round(kidx_ms, 2),
        "rates": rows,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def serve_roofline_and_cpu(args, ctx, P, h, qs, gen):
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg

    bb = h["bm_begin"].astype(np.int64)
    keys = h["keys"]
    pay = container_payload_bytes(h)
    in_bytes = 0.0
    out_bytes = 0
    rg.profile_enable(ctx, True)
    rg.profile_reset(ctx)
    for op, ids, mat in qs:
        lists = [keys[bb[b]:bb[b + 1]] for b in ids]
        ks = lists[0]
        for l in lists[1:]:
            ks = np.intersect1d(ks, l) if op == "and" else np.union1d(ks, l)
        for b, l in zip(ids, lists):
            sel = np.isin(l, ks)
            in_bytes += float(pay[bb[b]:bb[b + 1]][sel].sum())
        d_ids = torch.from_numpy(np.ascontiguousarray(ids).view(np.int32)).cuda()
        out, _ = rg.multi(ctx, op, P, d_ids, materialize=True, card=True)
        out_bytes += result_payload_bytes(out)[0]
    torch.cuda.synchronize()
    pr = rg.profile_read(ctx)
    kw = dict(pr.get(("kway-eval", True)) or {"ms": 0.0, "launches": 0})
    for extra in ("kway-small", "kway-bb", "kway-wave"):  # the one-wave kernels
        if pr.get((extra, True)):
            kw["ms"] += pr[(extra, True)]["ms"]
    rg.profile_enable(ctx, False)
    roof = None
    if kw and kw["launches"]:
        tot = in_bytes + out_bytes
        ach = tot / (kw["ms"] / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_kw_small + k_kw_bb + k_kw_eval (k-way evaluation step; one roaring_multi call per query, "
                          "materialised)",
                "mean_launch_ms": round(kw["ms"] / kw["launches"], 4), "launches": int(kw["launches"]),
                "bytes_per_launch": int(tot / kw["launches"]),
                "sample": f"{len(qs)} queries of the mix, all materialised"}
    cpu = None
    if not args.no_cpu_baseline:
        sets = {int(b): gen(int(b)) for _, ids, _ in qs for b in ids}
        tasks = [(lambda op=op, ids=ids: oracle.kway(op, [sets[int(b)] for b in ids])) for op, ids, _ in qs]
        cpu = cpu_baseline_tasks(tasks, float(len(tasks)), "queries/s",
                                 f"{len(tasks)} queries of the mix, k-way left fold of two-pointer merges",
                                 args.cpu_seconds)
    return roof, cpu


# ---------------------------------------------------------------- wide union, access, canonical, in-place

def _line(metric, value, unit, args, ms, config, extra, roof, cpu, dtype="u32"):
    line = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    line.update(extra)
    line["roofline"] = roof
    line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


def _kway_eval_ms(prof):
    """ms and launches of the k-way evaluation step (the two one-wave kernels
    and the workgroup kernel, one launch each per call)."""
    ms = sum(prof[(c, True)]["ms"] for c in ("kway-small", "kway-bb", "kway-wave", "kway-eval") if (c, True) in prof)
    launches = prof[("kway-eval", True)]["launches"] if ("kway-eval", True) in prof else 0
    return ms, launches


def _event_ms(fn, reps):
    """Mean device time of fn() over reps calls, HIP events on the current stream."""
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_wide(args):
    """Wide union (Section 5.9, the union of all bitmaps of a collection;
    Table 8's shape): one roaring_multi call over --wide bitmaps of the mixed
    recipe, materialised with its cardinality; the count-only union beside it.
    value = algorithmic input bytes (every container's payload + 19 B of
    metadata) / time of the materialised union."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    ctx = rg.Context(0)
    k = args.wide
    bs = synth.mixed_small(n_bitmaps=k, seed=synth.SEED_BASE + 7)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    h = rg.Pool.host_arrays(bs.values, bs.offsets)[3]
    in_bytes = float(container_payload_bytes(h).sum()) + META_BYTES * len(h["keys"])
    ids = torch.arange(k, dtype=torch.int32, device="cuda")
    out, card = rg.multi(ctx, "or", P, ids, materialize=True, card=True)
    torch.cuda.synchronize()
    exp = oracle.kway("or", [bs[i] for i in range(k)])
    dig = int(rg.rg_pool_digest(ctx, out.as_pool()).cpu().numpy().view(np.uint64)[0])
    assert int(card.item()) == len(exp) and dig == oracle.digest(exp), "wide union differs from the oracle"
    say(f"wide union of {k} bitmaps ({len(bs.values)} values, {len(h['keys'])} containers): "
        f"{len(exp)} values, matches the oracle")
    flags = rg.RG_FLAG_MATERIALIZE | rg.RG_FLAG_CARD

    def step():
        ctx.check(rg.roaring_multi(ctx, "or", P, ids, flags, out, card))

    def step_count():
        ctx.check(rg.roaring_multi(ctx, "or", P, ids, rg.RG_FLAG_CARD, None, card))

    # without, then with the pool's key-presence indexes (built once)
    dt_plain = time_steps(step, args.steps, args.warmup)
    kidx_ms = None
    if args.key_index:
        t1 = time.time()
        P.key_index(ctx)
        torch.cuda.synchronize()
        kidx_ms = (time.time() - t1) * 1e3
        ctx.check(rg.roaring_multi(ctx, "or", P, ids, flags, out, card))
        torch.cuda.synchronize()
        dig2 = int(rg.rg_pool_digest(ctx, out.as_pool()).cpu().numpy().view(np.uint64)[0])
        assert int(card.item()) == len(exp) and dig2 == dig, "wide union with key indexes differs"
    dt = time_steps(step, args.steps, args.warmup)
    dtc = time_steps(step_count, args.steps, args.warmup)
    rg.profile_enable(ctx, True)
    rg.profile_reset(ctx)
    time_steps(step, args.steps, 0)
    prof = rg.profile_read(ctx)
    rg.profile_enable(ctx, False)
    out_pay, out_n = result_payload_bytes(out)
    ms, launches = _kway_eval_ms(prof)
    roof = None
    if launches:
        per = (in_bytes - META_BYTES * len(h["keys"]) + out_pay)
        mean_s = ms / launches / 1e3
        roof = {"bound": "hbm", "achieved": round(per / mean_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(per / mean_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_kw_eval (+ one-wave kernels; k-way evaluation step)",
                "mean_launch_ms": round(mean_s * 1e3, 4), "launches": int(launches), "bytes_per_launch": int(per)}
    cpu = None
    if not args.no_cpu_baseline:
        lists = [bs[i] for i in range(k)]
        cpu = cpu_baseline_tasks([lambda: oracle.kway("or", lists)], in_bytes, "GB/s",
                                 f"the whole {k}-way union (left fold of two-way unions); the all-core rate runs "
                                 f"independent copies of it side by side", args.cpu_seconds)
    _line("input GB/s of a wide (k-way) union, materialised", round(in_bytes / dt / 1e9, 2), "GB/s", args,
          dt * 1e3,
          {"workload": f"wide union: {k} mixed bitmaps over [0, 2^26), 1e3..5e4 values, 40/30/30 sparse/dense/run; "
                       f"one {k}-way OR materialised with its cardinality", "k": k,
           "key_index": bool(args.key_index), "parallelism": "single GPU"},
          {"union_values": len(exp), "result_containers": out_n, "count_only_ms": round(dtc * 1e3, 4),
           "no_key_index_ms": round(dt_plain * 1e3, 4),
           "key_index_build_ms": None if kidx_ms is None else round(kidx_ms, 2),
           "input_bytes": int(in_bytes)}, roof, cpu)


def bench_access(args):
    """Membership and export (Section 1 random access, Section 3.1 bitset to
    values, Sections 5.5 and 5.6): --lookups (bitmap, value) membership tests,
    half of them members, over a pool of --access-bitmaps mixed bitmaps; and the
    export of the whole pool to sorted uint32. value = lookups/s; the export's
    rate is reported beside it."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    ctx = rg.Context(0)
    nb = args.access_bitmaps
    bs = synth.mixed_small(n_bitmaps=nb, seed=synth.SEED_BASE + 8)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    h = rg.Pool.host_arrays(bs.values, bs.offsets)[3]
    rng = np.random.default_rng(synth.SEED_BASE + 9)
    n = args.lookups
    ids = rng.integers(0, nb, n).astype(np.uint32)
    off = np.asarray(bs.offsets, np.int64)
    member = rng.random(n) < 0.5
    pick = off[ids] + (rng.random(n) * (off[ids + 1] - off[ids])).astype(np.int64)
    xs = np.where(member, bs.values[np.minimum(pick, len(bs.values) - 1)],
                  rng.integers(0, 1 << 26, n).astype(np.uint32)).astype(np.uint32)
    d_ids = torch.from_numpy(ids.view(np.int32)).cuda()
    d_xs = torch.from_numpy(xs.view(np.int32)).cuda()
    d_out = torch.empty(n, dtype=torch.uint8, device="cuda")
    ctx.check(rg.roaring_contains(ctx, P, d_ids, d_xs, d_out))
    torch.cuda.synchronize()
    m = min(n, 200000)
    exp = oracle.contains_many(bs.values, bs.offsets, ids[:m], xs[:m])
    assert np.array_equal(d_out[:m].cpu().numpy().astype(bool), exp.astype(bool)), "membership differs"
    # export: offsets and values sized once, then timed into the same buffers
    offsets, values = rg.to_uint32(ctx, P)
    torch.cuda.synchronize()
    assert np.array_equal(values.cpu().numpy().view(np.uint32), bs.values), "export differs from the input lists"
    say(f"{m} lookups and the export of {nb} bitmaps ({len(bs.values)} values) match the oracle / the input")
    nv = int(values.numel())

    def look():
        ctx.check(rg.roaring_contains(ctx, P, d_ids, d_xs, d_out))

    def export():
        st, _ = rg.roaring_to_uint32(ctx, P, 0, nb, offsets, values, nv)
        ctx.check(st)

    dt = time_steps(look, args.steps, args.warmup)
    dte = time_steps(export, args.steps, args.warmup)
    ms_look = _event_ms(look, args.steps)
    ms_exp = _event_ms(export, args.steps)
    pay = float(container_payload_bytes(h).sum())
    exp_bytes = pay + META_BYTES * len(h["keys"]) + 4.0 * nv + 8.0 * (nb + 1)
    look_bytes = 9.0 * n  # (bitmap, value) in, one byte out: the lookups' unavoidable traffic
    roof = {"bound": "hbm", "achieved": round(look_bytes / (ms_look / 1e3) / 1e9, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(look_bytes / (ms_look / 1e3) / 1e9 / HBM_PEAK_GBS, 5), "traffic": None,
            "kernel": "k_contains", "mean_launch_ms": round(ms_look, 4), "launches": args.steps,
            "bytes_per_launch": int(look_bytes),
            "note": "9 B per lookup; the key and container searches run in cache (latency-bound)"}
    export_roof = {"bound": "hbm", "achieved": round(exp_bytes / (ms_exp / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                   "unit": "GB/s", "frac": round(exp_bytes / (ms_exp / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                   "kernel": "k_export_values (+ sizing kernels; one call)", "mean_call_ms": round(ms_exp, 4),
                   "bytes_per_call": int(exp_bytes)}
    cpu = None
    if not args.no_cpu_baseline:
        ms_ = min(n, 1000000)
        nt = cpu_threads()
        chunk = max(1, ms_ // (4 * nt))
        tasks = [(lambda s0=s0: oracle.contains_many(bs.values, bs.offsets, ids[s0:s0 + chunk], xs[s0:s0 + chunk]))
                 for s0 in range(0, ms_, chunk)]
        cpu = cpu_baseline_tasks(tasks, float(ms_), "lookups/s", f"{ms_} of the lookups (binary search over the "
                                 f"sorted uint32 list)", args.cpu_seconds)
    _line("membership lookups/s (batched contains); export values/s beside it", round(n / dt, 1), "lookups/s",
          args, dt * 1e3,
          {"workload": f"access: {nb} mixed bitmaps over [0, 2^26) ({len(bs.values)} values); {n} random "
                       f"(bitmap, value) lookups, half members; export of the whole pool to sorted uint32",
           "bitmaps": nb, "lookups": n, "parallelism": "single GPU"},
          {"export_values_per_s": round(nv / dte, 1), "export_ms": round(dte * 1e3, 4), "export_values": nv,
           "export_roofline": export_roof}, roof, cpu)


def bench_canonical(args):
    """Canonicalisation (Section 1: the least-memory container of every chunk;
    Section 5.1: inputs run-optimised): a pool of --canon-bitmaps mixed bitmaps
    stored in random well-formed forms (arrays of any length, bitsets of any
    cardinality, runs cut into touching runs) rebuilt in P1 form.
    value = algorithmic input bytes / time."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth
    from tests import rgtest

    ctx = rg.Context(0)
    nb = args.canon_bitmaps
    bs = synth.mixed_small(n_bitmaps=nb, seed=synth.SEED_BASE + 10)
    sets = [bs[i] for i in range(nb)]
    a = rgtest.noncanonical_arrays(sets, np.random.default_rng(synth.SEED_BASE + 11))
    P = rg.Pool.from_host_arrays(a)
    out = rg.canonicalize(ctx, P)
    torch.cuda.synchronize()
    dig = rg.rg_pool_digest(ctx, out.as_pool()).cpu().numpy().view(np.uint64)
    for i in range(nb):
        assert int(dig[i]) == oracle.digest(sets[i]), i
    n_in = len(a["keys"])
    pay_in = float(container_payload_bytes(a).sum())
    in_bytes = pay_in + META_BYTES * n_in
    say(f"{nb} bitmaps, {n_in} containers in random forms ({np.bincount(a['types'], minlength=4)[1:].tolist()} "
        f"array/bitset/run): canonical forms match the oracle's fingerprints")

    def step():
        ctx.check(rg.lib().rg_pool_canonicalize(ctx.h, rg.ctypes.byref(P.c), rg.ctypes.byref(out.c), None))

    dt = time_steps(step, args.steps, args.warmup)
    rg.profile_enable(ctx, True)
    rg.profile_reset(ctx)
    time_steps(step, args.steps, 0)
    prof = rg.profile_read(ctx)
    rg.profile_enable(ctx, False)
    out_pay, out_n = result_payload_bytes(out)
    ms, launches = _kway_eval_ms(prof)
    roof = None
    if launches:
        per = pay_in + out_pay
        mean_s = ms / launches / 1e3
        roof = {"bound": "hbm", "achieved": round(per / mean_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(per / mean_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_kw_small + k_kw_bb + k_kw_eval (k-way evaluation step, one-bitmap unions)",
                "mean_launch_ms": round(mean_s * 1e3, 4), "launches": int(launches), "bytes_per_launch": int(per)}
    cpu = None
    if not args.no_cpu_baseline:
        nt = cpu_threads()
        chunk = max(1, nb // (4 * nt))
        tasks = [(lambda s0=s0: [oracle.containers(v) for v in sets[s0:s0 + chunk]]) for s0 in range(0, nb, chunk)]
        cpu = cpu_baseline_tasks(tasks, in_bytes, "GB/s", f"the P1 container view of all {nb} bitmaps from their "
                                 f"sorted lists", args.cpu_seconds)
    _line("input GB/s of device canonicalisation (non-P1 pool to P1)", round(in_bytes / dt / 1e9, 2), "GB/s", args,
          dt * 1e3,
          {"workload": f"canonical: {nb} mixed bitmaps over [0, 2^26) stored in random well-formed forms "
                       f"(1/3 arrays of any length, 1/3 bitsets, 1/3 runs cut into touching runs), rebuilt in P1 "
                       f"form", "bitmaps": nb, "parallelism": "single GPU"},
          {"containers_in": n_in, "containers_out": out_n, "containers_per_s": round(n_in / dt, 1)}, roof, cpu)


def bench_inplace(args):
    """In-place operations (Section 3.2: bits set, cleared, flipped with the
    cardinality kept; Section 5.9's wide unions partly in place): --acc mutable
    bitmaps, each changed by a fixed cycle of op= with bitmaps of a mixed pool
    (union, intersection, symmetric difference, difference), every result and
    cardinality checked against the oracle's fold after the timed steps. A step
    is one cycle, each of its operations applied to all bitmaps in one batched
    call (rg_mpool_op_batch); one call per operation (rg_mpool_op) is timed
    beside it. value = operations/s of the batched calls."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    ctx = rg.Context(0)
    bs = synth.mixed_small(n_bitmaps=100, seed=synth.SEED_BASE + 12)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    h = rg.Pool.host_arrays(bs.values, bs.offsets)[3]
    bb = h["bm_begin"].astype(np.int64)
    pay = container_payload_bytes(h)
    na = args.acc
    M = rg.MutablePool(ctx, na, na * 1100)
    state = []
    for b in range(na):
        M.assign(b, P, b)
        state.append(bs[b])
    rng = np.random.default_rng(synth.SEED_BASE + 13)
    cycle = [("or", int(s)) for s in rng.integers(0, 100, 4)] + [("and", int(rng.integers(0, 100)))] + \
            [("xor", int(rng.integers(0, 100))), ("andnot", int(rng.integers(0, 100)))] + \
            [("or", int(s)) for s in rng.integers(0, 100, 1)]
    ops_per_step = na * len(cycle)
    step_bytes = float(sum(pay[bb[s]:bb[s + 1]].sum() + META_BYTES * (bb[s + 1] - bb[s]) for _, s in cycle)) * na
    applied = 0
    targets = np.arange(na, dtype=np.uint32)

    def step_single():
        nonlocal applied
        for op, s in cycle:
            for b in range(na):
                M.op(op, b, P, s)
        applied += 1

    def step():
        nonlocal applied
        for op, s in cycle:
            M.op_batch([op] * na, targets, P, [s] * na)
        applied += 1

    dt_single = time_steps(step_single, args.steps, args.warmup)
    dt = time_steps(step, args.steps, args.warmup)
    st, free = M.status()
    assert st == rg.RG_OK, st
    for _ in range(applied):
        for op, s in cycle:
            state = [oracle.op(op, x, bs[s]) for x in state]
    out = M.export()
    hh = out.as_pool().to_host()
    from tests import rgtest
    cards = M.cards().cpu().numpy().view(np.uint64)
    for b in range(na):
        got, _ = rgtest.decode_bitmap(hh, b)
        assert np.array_equal(got, state[b]) and int(cards[b]) == len(state[b]), b
    say(f"{na} bitmaps after {applied} cycles of {len(cycle)} in-place ops each match the oracle's fold "
        f"({free} free slots)")
    ms_op = _event_ms(lambda: M.op_batch(["or"] * na, targets, P, [cycle[0][1]] * na), 20)
    roof = {"bound": "hbm", "achieved": round(step_bytes / dt / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(step_bytes / dt / 1e9 / HBM_PEAK_GBS, 5), "traffic": None,
            "kernel": "rg_mpool_op_batch (classify, capacity check, drop, evaluate, insert: six launches per batch)",
            "mean_call_ms": round(ms_op, 4), "bytes_per_step": int(step_bytes),
            "note": "bytes: payload + metadata of the B operands; mean_call_ms: one batched union of every bitmap"}
    cpu = None
    if not args.no_cpu_baseline:
        lists = [bs[b] for b in range(na)]

        def fold(x=lists):
            for op, s in cycle:
                x = [oracle.op(op, y, bs[s]) for y in x]

        cpu = cpu_baseline_tasks([fold], float(ops_per_step), "ops/s", f"one cycle of the {ops_per_step} "
                                 f"operations on the initial bitmaps (two-pointer merges into new lists)",
                                 args.cpu_seconds)
    _line("in-place operations/s (A op= B with maintained cardinality, batched)", round(ops_per_step / dt, 1), "ops/s",
          args,
          dt * 1e3,
          {"workload": f"inplace: {na} mutable bitmaps (starting as mixed bitmaps over [0, 2^26)), each changed by "
                       f"a cycle of {len(cycle)} op= (or x5, and, xor, andnot) with bitmaps of a 100-bitmap mixed "
                       f"pool", "accumulators": na, "parallelism": "single GPU"},
          {"ops_per_step": ops_per_step, "input_gb_per_s": round(step_bytes / dt / 1e9, 3),
           "one_call_per_op_ops_per_s": round(ops_per_step / dt_single, 1)}, roof, cpu)


# ---------------------------------------------------------------- HBM byte counters

TRAFFIC_SOURCES = ("rg_match.hip", "rg_count_dev.h", "rg_finalize.h", "rg_internal.h")


def source_hash():
    """Hash of the sources of the dominant kernel (the counter summary records it)."""
    import hashlib

    h = hashlib.sha256()
    digests = []
    for f in TRAFFIC_SOURCES:
        digests.append(hashlib.sha256(open(os.path.join(ROOT, "paper_1709_07821_amd", "csrc", f), "rb").read())
                       .hexdigest())
    h.update("".join(digests).encode())
    return h.hexdigest()[:16]


def measured_traffic(summary="k_count_fused_dense_bitsets.md"):
    """HBM bytes per fused count launch from a committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources have changed since it was taken."""
    prof = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(prof):
        return None
    text = open(prof).read()
    tb = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("traffic_bytes_per_launch:")]
    hv = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("source_hash:")]
    if not tb or not hv:
        return None
    return int(tb[0]) if source_hash() == hv[0] else None


if __name__ == "__main__":
    main()
