"""Benchmark: Roaring set operations on the dense-bitset workload.

Workload (bitset-bandwidth): 2e4 bitmaps, each with 256 bitset containers
(keys 0..255, 8 KiB each, bit density U(0.2, 0.8)), about 42 GB resident in
HBM, generated on the device; 1e4 random pairs (ia != ib). One step runs, for
each of AND, OR, XOR, ANDNOT, the count-only form (fused op + popcount,
|A op B| per pair) over all pairs, plus the Jaccard index per pair.

value = algorithmic input bytes of the step / step time (GB/s), the metric's
"input GB/s"; container-pairs/s is reported beside it. Inputs are resident in
HBM before timing starts.

The dominant kernel's roofline entry is measured live: the library brackets
each launch of its bitset-bitset kernel with HIP events on the launch stream
(rg_profile_*), and achieved = algorithmic bytes per launch / mean launch time.

cpu_baseline: the CPU oracle (plain two-pointer merges over sorted uint32
lists) timed on a bounded sample of the same pairs, rank 0 only.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
META_BYTES = 19  # key u16 + type u8 + card u32 + size u32 + off u64 per container


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--bitmaps", type=int, default=20000)
    ap.add_argument("--keys", type=int, default=256)
    ap.add_argument("--pairs", type=int, default=10000)
    ap.add_argument("--cpu-pairs", type=int, default=48, help="pairs in the oracle timing sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", type=int, default=2, help="pairs checked against the oracle before timing")
    ap.add_argument("--workload", choices=("dense", "dense-mat", "batched", "serve"), default="dense",
                    help="dense: the bitset-bandwidth headline; batched: many uneven pairs, plan vs per-pair; "
                         "serve: k-way queries under Poisson arrivals, batched server vs one query at a time")
    ap.add_argument("--index", type=int, default=4000, help="serve: bitmaps in the index")
    ap.add_argument("--rates", default="2000,5000,10000,20000,50000", help="serve: arrival rates (queries/s)")
    ap.add_argument("--duration", type=float, default=2.0, help="serve: seconds of arrivals per rate")
    ap.add_argument("--max-batch", type=int, default=256, help="serve: most queries per step (batched mode)")
    ap.add_argument("--pool", type=int, default=16384, help="batched: bitmaps in the pool")
    ap.add_argument("--batched-pairs", type=int, default=1000000, help="batched: random pairs per step")
    ap.add_argument("--per-pair-sample", type=int, default=500, help="batched: pairs timed one call each")
    ap.add_argument("--dispatch-pairs", type=int, default=300, help="batched: pairs whose costs train the dispatcher")
    ap.add_argument("--dispatch-epochs", type=int, default=10, help="batched: dispatcher training epochs")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES bytes (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is designed (keys partition the universe), not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_07821_amd as rg
    import synth

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
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "dense-mat":
        return bench_dense_mat(args)
    if args.workload == "serve":
        return bench_serve(args)
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
    print(f"# generated {nb} x {nk} bitsets ({words.numel() * 8 / 1e9:.1f} GB) in {time.time() - t0:.1f} s",
          file=sys.stderr, flush=True)
    ia, ib = synth.random_pairs(nb, npairs, seed=synth.DENSE_SEED)
    tia = torch.from_numpy(ia.view(np.int32)).to(dev)
    tib = torch.from_numpy(ib.view(np.int32)).to(dev)
    cards = {op: torch.zeros(npairs, dtype=torch.int64, device=dev) for op in rg.OPS}
    jacc = torch.zeros(npairs, dtype=torch.float64, device=dev)

    def step():
        for op in ("and", "or", "xor", "andnot"):
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
        print(f"# {args.check} pairs x 4 ops match the oracle", file=sys.stderr, flush=True)

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
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_count_fused", "mean_launch_ms": round(mean_s * 1e3, 4),
                "launches": int(k["launches"]), "bytes_per_launch": int(alg_bytes)}

    if roof is not None:
        roof["traffic"] = measured_traffic()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(ia, ib, nk, args.cpu_pairs)

    line = {
        "metric": "input GB/s and container-pairs/sec for AND/OR/XOR/ANDNOT+card (% HBM peak)",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "dense-bitset pairs: 2e4 bitmaps x 256 bitset containers (U(0.2,0.8) density), "
                               "1e4 random pairs, |A op B| for AND/OR/XOR/ANDNOT + Jaccard",
                   "bitmaps": nb, "keys_per_bitmap": nk, "pairs": npairs, "parallelism": "single GPU"},
        "container_pairs_per_s": round(cps, 1),
        "pct_hbm_peak": round(100 * value / HBM_PEAK_GBS, 2),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


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
    for op in rg.OPS:
        arenas[op], _, _ = rg.batch(ctx, op, P, P, tia, tib, materialize=True, card=True)
    torch.cuda.synchronize()
    # correctness gate: two pairs of every op against the oracle (fingerprints)
    for op in rg.OPS:
        dig = rg.rg_pool_digest(ctx, arenas[op].as_pool()).cpu().numpy().view(np.uint64)
        for p in range(2):
            exp = oracle.op(op, synth.dense_bitmap_values(int(ia[p]), nk), synth.dense_bitmap_values(int(ib[p]), nk))
            assert int(dig[p]) == oracle.digest(exp), (op, p)
    print(f"# {nb} x {nk} bitsets, {npairs} pairs; 2 pairs x 4 ops match the oracle", file=sys.stderr, flush=True)
    out_bytes = {op: int(arenas[op].c.payload_used) for op in rg.OPS}

    def step():
        for op in rg.OPS:
            rg.batch(ctx, op, P, P, tia, tib, materialize=True, card=True, out=arenas[op])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
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


def bench_batched(args):
    """Many uneven pairs: |A n B| and Jaccard for every pair of a random pair list
    over a pool of mixed bitmaps (lognormal cardinality, median 1e4, sigma 2,
    clipped to [10, 1e7], over [0, 2^32), 40/30/30 sparse/dense/run with a
    256-key hot set). Three executions of the same step, same results:
    one library call per pair; one batched call (host-synchronised waves);
    a plan (persistent work-stealing kernel, autotuned, replayed as a hipGraph)."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    dev = torch.device("cuda:0")
    ctx = rg.Context(0)
    seed = synth.SEED_BASE + 3
    t0 = time.time()
    hot = synth.hot_keys(seed, 256, 1 << 16)
    cards = [synth.lognormal_card(i, 1e4, 2.0, 10, 10 ** 7, seed) for i in range(args.pool)]
    sets = []
    for i in range(args.pool):
        sets.append(synth.mixed_bitmap(seed, i, cards[i], 32, hot))
        if (i + 1) % 4096 == 0:
            print(f"# generated {i + 1} of {args.pool} bitmaps, {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    bs = synth.BitmapSet.from_list(sets)
    del sets
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    ia, ib = synth.random_pairs(args.pool, args.batched_pairs, seed)
    n = len(ia)
    tia = torch.from_numpy(ia.view(np.int32)).to(dev)
    tib = torch.from_numpy(ib.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    print(f"# pool of {args.pool} bitmaps, {len(bs.values)} values, {P.c.n_containers} containers, "
          f"{n} pairs, built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    # eager batched call; also gives the matched container pairs (profile items)
    rg.profile_enable(ctx, True)
    rg.profile_reset(ctx)
    _, c_e, j_e = rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True)
    torch.cuda.synchronize()
    matched = sum(v["items"] for v in rg.profile_read(ctx).values())
    rg.profile_enable(ctx, False)
    c_e, j_e = c_e.cpu().numpy().view(np.uint64), j_e.cpu().numpy()
    for p in range(0, n, max(1, n // 16)):
        a, b = bs[int(ia[p])], bs[int(ib[p])]
        assert int(c_e[p]) == oracle.count("and", a, b) and j_e[p] == oracle.jaccard(a, b), p
    print(f"# 16 sampled pairs match the oracle; {matched} matched container pairs per step",
          file=sys.stderr, flush=True)

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps

    eager_s = timed(lambda: rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True),
                    args.steps, 1)
    print(f"# eager batched: {eager_s * 1e3:.2f} ms/step", file=sys.stderr, flush=True)
    # the same eager call on a pool that carries packed metadata records
    # (rg_pool_pack_meta); the plans below reuse them
    t_p = time.perf_counter()
    P.pack_meta(ctx)
    torch.cuda.synchronize()
    pack_s = time.perf_counter() - t_p
    eager_packed_s = timed(lambda: rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True),
                           args.steps, 1)
    _, c_p, j_p = rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True)
    torch.cuda.synchronize()
    assert np.array_equal(c_p.cpu().numpy().view(np.uint64), c_e) and np.array_equal(j_p.cpu().numpy(), j_e)
    print(f"# eager batched, packed metadata: {eager_packed_s * 1e3:.2f} ms/step (packing once: "
          f"{pack_s * 1e3:.1f} ms), results equal", file=sys.stderr, flush=True)

    # plan: tuned, captured, replayed on a side stream
    st = torch.cuda.Stream()
    pl = rg.Plan(ctx, "and", P, P, tia, tib, card=True, jaccard=True, stream=st)
    pl.tune(stream=st, reps=1)
    pl.capture(st)
    torch.cuda.synchronize()

    def run_plan():
        pl.execute(stream=st)

    plan_s = timed(run_plan, args.steps, args.warmup)
    assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), c_e)
    assert np.array_equal(pl.jacc.cpu().numpy(), j_e)
    info = pl.info()
    print(f"# plan (graph, {info}): {plan_s * 1e3:.2f} ms/step, results equal to the eager call",
          file=sys.stderr, flush=True)

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
    print(f"# dispatcher: {int(M.any(1).sum())} sampled container pairs, loss {losses[0]:.3f} -> {losses[-1]:.3f}, "
          f"{time.perf_counter() - t_s:.1f} s", file=sys.stderr, flush=True)
    pl2 = rg.Plan(ctx, "and", P, P, tia, tib, card=True, jaccard=True, stream=st)
    pl2.tune(stream=st, reps=1)
    pl2.capture(st)
    torch.cuda.synchronize()
    learned_s = timed(lambda: pl2.execute(stream=st), args.steps, args.warmup)
    assert np.array_equal(pl2.cards.cpu().numpy().view(np.uint64), c_e)
    assert np.array_equal(pl2.jacc.cpu().numpy(), j_e)
    info2 = pl2.info()
    pl2.close()
    ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)
    print(f"# plan with learned dispatch ({info2}): {learned_s * 1e3:.2f} ms/step, results equal",
          file=sys.stderr, flush=True)

    # one call per pair, on a sample
    k = min(args.per_pair_sample, n)
    one_c = torch.zeros(1, dtype=torch.int64, device=dev)
    one_j = torch.zeros(1, dtype=torch.float64, device=dev)
    flags = rg.RG_FLAG_CARD | rg.RG_FLAG_JACCARD

    def per_pair():
        for p in range(k):
            ctx.check(rg.roaring_batch(ctx, "and", P, P, tia[p:p + 1], tib[p:p + 1], flags, None, one_c, one_j))

    pp_s = timed(per_pair, 1, 0) / k * n
    print(f"# one call per pair: {pp_s / n * 1e6:.1f} us/pair on {k} pairs -> {pp_s * 1e3:.1f} ms/step",
          file=sys.stderr, flush=True)
    pl.close()

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
    }
    print(json.dumps(line), flush=True)


def bench_serve(args):
    """k-way AND/OR queries over a device-resident index under open-loop Poisson
    arrivals. Index: mixed bitmaps over [0, 2^26) (40/30/30 sparse/dense/run,
    32-key hot set), cardinality lognormal (median 5e4, sigma 1, clipped to
    [1e3, 1e6]). Mix: 40 % k-AND, 40 % k-OR (both materialised), 20 %
    count-only (half AND, half OR); k uniform in 2..32; ids uniform without
    replacement. Each rate runs twice: the continuous-batching server (up to
    --max-batch queries per step, two steps in flight) and one query at a time."""
    import numpy as np
    import torch

    import oracle
    import paper_1709_07821_amd as rg
    import synth

    ctx = rg.Context(0)
    seed = synth.SEED_BASE + 4
    t0 = time.time()
    hot = synth.hot_keys(seed, 32, 1 << 10)
    cards = [synth.lognormal_card(i, 5e4, 1.0, 1000, 10 ** 6, seed) for i in range(args.index)]
    bs = synth.BitmapSet.from_list([synth.mixed_bitmap(seed, i, cards[i], 26, hot) for i in range(args.index)])
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    torch.cuda.synchronize()
    print(f"# index of {args.index} bitmaps, {len(bs.values)} values, {P.c.n_containers} containers, "
          f"built in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
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

    # correctness gate: a sample against the oracle
    sample = make_queries(12)
    srv = rg.Server(ctx, P, arena_bytes=4 << 30, max_batch=args.max_batch, max_inflight=2)
    _, c_s, d_s = srv.replay(sample, np.zeros(len(sample), np.uint64))
    srv.stop()
    for i, (op, ids, mat) in enumerate(sample):
        e = oracle.kway(op, [bs[int(j)] for j in ids])
        assert c_s[i] == len(e) and d_s[i] == (oracle.digest(e) if mat else 0), i
    print("# 12 sampled queries match the oracle", file=sys.stderr, flush=True)

    rows = []
    for lam in [float(x) for x in args.rates.split(",")]:
        n = max(1, int(lam * args.duration))
        qs = make_queries(n)
        gaps = rng.exponential(1.0 / lam, n)
        arrival = (np.cumsum(gaps) * 1e9).astype(np.uint64)
        row = {"rate_qps": lam, "queries": n}
        for mode, mb, mi in (("batched", args.max_batch, 2), ("one_at_a_time", 1, 1)):
            srv = rg.Server(ctx, P, arena_bytes=4 << 30, max_batch=mb, max_inflight=mi)
            t = time.perf_counter()
            lat, c, d = srv.replay(qs, arrival)
            wall = time.perf_counter() - t
            st = srv.stop()
            if mode == "batched":
                ref = (c, d)
            else:
                assert np.array_equal(c, ref[0]) and np.array_equal(d, ref[1]), "results differ between modes"
            row[mode] = {"achieved_qps": round(n / wall, 1), "p50_us": round(float(np.percentile(lat, 50)) / 1e3, 1),
                         "p99_us": round(float(np.percentile(lat, 99)) / 1e3, 1),
                         "mean_batch": round(st["mean_batch"], 2), "steps": st["steps"]}
            print(f"# rate {lam:.0f}/s {mode}: {row[mode]}", file=sys.stderr, flush=True)
        rows.append(row)
    best = max(r["batched"]["achieved_qps"] for r in rows)
    line = {
        "metric": "queries/sec and p50/p99 latency, k-way AND/OR serving (continuous batching)",
        "value": best, "unit": "queries/s", "n_gpus": 1, "steps": len(rows), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"serving: index of {args.index} mixed bitmaps over [0, 2^26) (lognormal card, median "
                               f"5e4, sigma 1), Poisson arrivals, 40% k-AND / 40% k-OR materialised, 20% "
                               f"count-only, k in 2..32", "index": args.index, "duration_s": args.duration,
                   "parallelism": "single GPU"},
        "rates": rows,
    }
    print(json.dumps(line), flush=True)


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


def measured_traffic():
    """HBM bytes per fused count launch from the committed FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources have changed since it was taken."""
    prof = os.path.join(ROOT, "profiles", "k_count_fused_dense_bitsets.md")
    if not os.path.exists(prof):
        return None
    text = open(prof).read()
    tb = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("traffic_bytes_per_launch:")]
    hv = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("source_hash:")]
    if not tb or not hv:
        return None
    return int(tb[0]) if source_hash() == hv[0] else None


def cpu_baseline(ia, ib, nk, n_pairs):
    """The oracle, as it stands, on the first n_pairs pairs: 4 counts + Jaccard per pair."""
    import oracle
    import synth

    n_pairs = min(n_pairs, len(ia))
    sets = {}
    for p in range(n_pairs):
        for b in (int(ia[p]), int(ib[p])):
            if b not in sets:
                sets[b] = synth.dense_bitmap_values(b, nk)
    t0 = time.perf_counter()
    for p in range(n_pairs):
        a, b = sets[int(ia[p])], sets[int(ib[p])]
        for op in ("and", "or", "xor", "andnot"):
            oracle.count(op, a, b)
        oracle.jaccard(a, b)
    dt = time.perf_counter() - t0
    in_bytes = n_pairs * nk * 2 * (8192 + META_BYTES) * 4
    return {"value": round(in_bytes / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_pairs} of the pairs, 4 count-only ops + Jaccard each (two-pointer merges over "
                      f"sorted uint32), {dt:.1f} s"}


if __name__ == "__main__":
    main()
