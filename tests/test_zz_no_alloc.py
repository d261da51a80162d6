"""roaring_batch_static, the count-only batch for callers that cannot
allocate: its scratch is the library's fixed device array. Its counts and
Jaccard values must equal roaring_batch's (bit for bit) and the oracle's, on
consecutive calls whose inputs shrink, with no change in free device memory."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import rgtest

pytestmark = pytest.mark.gpu

OPS = ("and", "or", "xor", "andnot")
FLAGS = 2 | 4  # RG_FLAG_CARD | RG_FLAG_JACCARD


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rg():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1709_07821_amd as rg

    return rg


def _t(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


class _Case:
    """One batch: pools, device pair arrays, roaring_batch's results for every
    operation, and output buffers for roaring_batch_static."""

    def __init__(self, rg, ctx, name, bs_a, bs_b, P, Q, ia, ib):
        import torch

        self.name, self.bs_a, self.bs_b, self.P, self.Q = name, bs_a, bs_b, P, Q
        self.ia, self.ib = np.asarray(ia, np.uint32), np.asarray(ib, np.uint32)
        self.tia, self.tib = _t(self.ia), _t(self.ib)
        n = len(self.ia)
        self.ref = {}
        for op in OPS:
            cards = torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda")
            jacc = torch.full((max(n, 1),), -1.0, dtype=torch.float64, device="cuda")
            ctx.check(rg.roaring_batch(ctx, op, P, Q, self.tia, self.tib, FLAGS, None, cards, jacc))
            ctx.sync()
            self.ref[op] = (cards[:n].cpu().numpy().view(np.uint64).copy(), jacc[:n].cpu().numpy().copy())
        self.cards = {op: torch.full((max(n, 1),), -1, dtype=torch.int64, device="cuda") for op in OPS}
        self.jacc = {op: torch.full((max(n, 1),), -1.0, dtype=torch.float64, device="cuda") for op in OPS}

    def run_static(self, rg, ctx, op):
        _say(f"[static] {self.name} op={op} pairs={len(self.ia)}")
        ctx.check(rg.roaring_batch_static(ctx, op, self.P, self.Q, self.tia, self.tib, FLAGS, self.cards[op],
                                          self.jacc[op]))
        ctx.sync()

    def check(self, op, n_oracle):
        n = len(self.ia)
        c1 = self.cards[op][:n].cpu().numpy().view(np.uint64)
        j1 = self.jacc[op][:n].cpu().numpy()
        c0, j0 = self.ref[op]
        assert np.array_equal(c0, c1), (self.name, op)
        assert np.array_equal(j0.view(np.uint64), j1.view(np.uint64)), (self.name, op)
        step = max(1, n // n_oracle)
        for p in range(0, n, step):
            a, b = self.bs_a[int(self.ia[p])], self.bs_b[int(self.ib[p])]
            assert int(c1[p]) == oracle.count(op, a, b), (self.name, op, p)
            assert j1[p] == oracle.jaccard(a, b), (self.name, op, p)


def test_static_matches_batch_on_shrinking_inputs(rg):
    """Consecutive static calls, each smaller than the one before (600 pairs of
    a mixed pool, every ordered pair of the edge sets, 23 pairs across two
    pools, one pair, none), against roaring_batch and the oracle; free device
    memory is the same before and after them."""
    import torch

    ctx = rg.Context(0)
    bs = synth.mixed_small(n_bitmaps=40, seed=71)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    es = synth.BitmapSet.from_list(rgtest.edge_sets())
    E = rg.Pool.from_sets(es.values, es.offsets)
    ia, ib = synth.random_pairs(len(bs), 600, seed=71)
    ka = np.repeat(np.arange(len(es), dtype=np.uint32), len(es))
    kb = np.tile(np.arange(len(es), dtype=np.uint32), len(es))
    ja = np.arange(23, dtype=np.uint32) % len(es)
    jb = (np.arange(23, dtype=np.uint32) * 7) % len(bs)
    cases = [_Case(rg, ctx, "mixed", bs, bs, P, P, ia, ib),
             _Case(rg, ctx, "edges", es, es, E, E, ka, kb),
             _Case(rg, ctx, "edges x mixed", es, bs, E, P, ja, jb),
             _Case(rg, ctx, "one pair", es, es, E, E, ka[5:6], kb[5:6])]
    empty = _t(ka[:0])
    sentinel = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    sentinel_j = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    # every static kernel once (code objects load on first use), then measure
    cases[-1].run_static(rg, ctx, "and")
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for op in OPS:
        for cs in cases:
            cs.run_static(rg, ctx, op)
        ctx.check(rg.roaring_batch_static(ctx, op, E, E, empty, empty, FLAGS, sentinel, sentinel_j))
        ctx.sync()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    assert int(sentinel[0]) == 7 and float(sentinel_j[0]) == 7.0  # zero pairs write nothing
    for op in OPS:
        for cs, n_or in zip(cases, (40, 10 ** 6, 23, 1)):
            cs.check(op, n_or)
    ctx.close()


def test_static_packs_metadata_in_its_array(rg):
    """Many pairs over a small pool: the call packs the pool's metadata records
    into the static array beside its per-pair scratch, as a roaring_batch call
    on the context's workspace does; then a smaller call over the same pool."""
    ctx = rg.Context(0)
    bs = synth.mixed_small(n_bitmaps=8, seed=72)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    ia, ib = synth.random_pairs(len(bs), 5000, seed=72)
    big = _Case(rg, ctx, "8 bitmaps", bs, bs, P, P, ia, ib)
    small = _Case(rg, ctx, "8 bitmaps", bs, bs, P, P, ia[:9], ib[:9])
    for op in OPS:
        big.run_static(rg, ctx, op)
        small.run_static(rg, ctx, op)
        big.check(op, 30)
        small.check(op, 9)
    ctx.close()


def test_static_rejects_what_it_cannot_take(rg):
    import torch

    ctx = rg.Context(0)
    bs = synth.mixed_small(n_bitmaps=4, seed=73)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    n = rg.RG_STATIC_MAX_PAIRS + 1
    ia = torch.zeros(n, dtype=torch.int32, device="cuda")
    cards = torch.zeros(n, dtype=torch.int64, device="cuda")
    assert rg.roaring_batch_static(ctx, "and", P, P, ia, ia, rg.RG_FLAG_CARD, cards) == rg.RG_ECAPACITY
    assert rg.roaring_batch_static(ctx, "and", P, P, ia[:4], ia[:4], rg.RG_FLAG_MATERIALIZE) == rg.RG_ENOTSUP
    assert rg.roaring_batch_static(ctx, "and", P, P, ia[:4], ia[:4], rg.RG_FLAG_CARD, None) == rg.RG_EINVAL
    # the largest call it takes still runs (all pairs (0, 0))
    ctx.check(rg.roaring_batch_static(ctx, "and", P, P, ia, ia, rg.RG_FLAG_CARD, cards,
                                      n_pairs=rg.RG_STATIC_MAX_PAIRS))
    ctx.sync()
    c = cards[:rg.RG_STATIC_MAX_PAIRS].cpu().numpy()
    assert np.all(c == len(bs[0]))
    ctx.close()
