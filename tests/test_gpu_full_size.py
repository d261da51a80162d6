"""Parity at the full sizes of the batched and serving workloads, in the
launch configuration bench.py times: the batched count (16 384 bitmaps, 1e6
pairs; eager call and a tuned plan) on 258 pairs spread over the list, and the
serving loop over the 1e5-bitmap index on 48 queries of the mix, against the
oracle (the bitmaps regenerated on the host for each sampled pair or query).
Every other pair of the batch is checked for plan = eager."""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import bench
import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rg():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1709_07821_amd as rg

    return rg


@pytest.fixture(scope="module")
def ctx(rg):
    c = rg.Context(0)
    yield c
    c.close()


def test_batched_full_size_sampled(rg, ctx):
    import torch

    n_pool, n_pairs = 16384, 1_000_000
    gen = bench.batched_pool_gen(n_pool)
    h = bench.build_pool_threaded(gen, n_pool)
    P = rg.Pool.from_host_arrays(h)
    del h
    ia, ib = synth.random_pairs(n_pool, n_pairs, synth.SEED_BASE + 3)
    tia = torch.from_numpy(ia.view(np.int32)).cuda()
    tib = torch.from_numpy(ib.view(np.int32)).cuda()
    _say(f"[full batched] pool of {n_pool} bitmaps, {P.c.n_containers} containers, {n_pairs} pairs")
    _, c_and, jac = rg.batch(ctx, "and", P, P, tia, tib, materialize=False, card=True, jaccard=True)
    _, c_xor, _ = rg.batch(ctx, "xor", P, P, tia, tib, materialize=False, card=True)
    pl = rg.Plan(ctx, "and", P, P, tia, tib, card=True, jaccard=True)
    pl.tune()
    pl.execute()
    ctx.sync()
    c_and = c_and.cpu().numpy().view(np.uint64)
    c_xor = c_xor.cpu().numpy().view(np.uint64)
    jac = jac.cpu().numpy()
    assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), c_and)
    assert np.array_equal(pl.jacc.cpu().numpy(), jac)
    pl.close()
    sample = np.unique(np.concatenate([[0, n_pairs - 1], np.linspace(0, n_pairs - 1, 256).astype(np.int64)]))

    def expect(p):
        a, b = gen(int(ia[p])), gen(int(ib[p]))
        return oracle.count("and", a, b), oracle.count("xor", a, b), oracle.jaccard(a, b)

    with ThreadPoolExecutor(16) as ex:
        exp = list(ex.map(expect, sample))
    for p, (ea, ex_, ej) in zip(sample, exp):
        assert int(c_and[p]) == ea and int(c_xor[p]) == ex_ and jac[p] == ej, p
    _say(f"[full batched] {len(sample)} sampled pairs match the oracle; plan = eager on all pairs")


def test_serve_full_index_sampled(rg, ctx):
    n_index = 100_000
    gen = bench.serve_index_gen(n_index)
    h = bench.build_pool_threaded(gen, n_index)
    P = rg.Pool.from_host_arrays(h)
    del h
    rng = np.random.default_rng(synth.SEED_BASE + 14)
    qs = []
    for i in range(48):
        k = int(rng.integers(2, 33))
        ids = rng.choice(n_index, size=k, replace=False).astype(np.uint32)
        qs.append((("and", "or")[i % 2], ids, i % 5 != 4))
    _say(f"[full serve] index of {n_index} bitmaps, {P.c.n_containers} containers, {len(qs)} queries")
    srv = rg.Server(ctx, P, arena_bytes=4 << 30, max_batch=256, max_inflight=2)
    try:
        _, cards, digs = srv.replay(qs, np.arange(len(qs), dtype=np.uint64) * 50_000, digest=True)
    finally:
        st = srv.stop()
    _say(f"[full serve] {st}")

    def expect(q):
        op, ids, mat = q
        e = oracle.kway(op, [gen(int(i)) for i in ids])
        return len(e), (oracle.digest(e) if mat else 0)

    with ThreadPoolExecutor(16) as ex:
        exp = list(ex.map(expect, qs))
    for i, (c, d) in enumerate(exp):
        assert int(cards[i]) == c and int(digs[i]) == d, i
