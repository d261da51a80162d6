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
    ap.add_argument("--cpu-pairs", type=int, default=24, help="pairs in the oracle timing sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", type=int, default=2, help="pairs checked against the oracle before timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design in DESIGN.md, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1709_07821_amd as rg
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
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

    # dominant kernel: bitset-bitset, count-only form
    k = prof.get(("bb", False))
    roof = None
    if k and k["launches"]:
        per_launch_items = k["items"] / k["launches"]
        alg_bytes = per_launch_items * 2 * 8192
        mean_s = k["ms"] / k["launches"] / 1e3
        ach = alg_bytes / mean_s / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_bb<op, count-only>", "mean_launch_ms": round(mean_s * 1e3, 4),
                "launches": int(k["launches"]), "bytes_per_launch": int(alg_bytes)}

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
