"""Access to values on the GPU against the oracle: batched membership
(roaring_contains) and export to sorted uint32 values (roaring_to_uint32),
over every container kind, chunk edges, packed and unpacked pools, ranges of
bitmaps, and materialised results."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import rgtest

pytestmark = pytest.mark.gpu

EDGE_VALUES = np.array([0, 1, 63, 64, 65535, 65536, 65537, 131071, 2**31 - 1, 2**31, 2**32 - 2, 2**32 - 1],
                       np.uint32)


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


def _t(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def _queries(bs, rng, n_random):
    """Every member of every bitmap, its neighbours, the chunk edges for every
    bitmap, and random values."""
    ids, xs = [], []
    for b in range(len(bs)):
        v = bs[b].astype(np.int64)
        for d in (-1, 0, 1):
            q = v + d
            q = q[(q >= 0) & (q < 2**32)]
            ids.append(np.full(len(q), b, np.uint32))
            xs.append(q.astype(np.uint32))
        ids.append(np.full(len(EDGE_VALUES), b, np.uint32))
        xs.append(EDGE_VALUES)
    ids.append(rng.integers(0, len(bs), n_random).astype(np.uint32))
    xs.append(rng.integers(0, 2**32, n_random, dtype=np.uint64).astype(np.uint32))
    return np.concatenate(ids), np.concatenate(xs)


def _check_contains(rg, ctx, bs, P, label, n_random=20000, seed=3):
    rng = np.random.default_rng(seed)
    ids, xs = _queries(bs, rng, n_random)
    _say(f"[contains] {label}: {len(ids)} queries over {len(bs)} bitmaps")
    got = rg.contains(ctx, P, _t(ids), _t(xs)).cpu().numpy().astype(np.uint8)
    ctx.sync()
    exp = oracle.contains_many(bs.values, bs.offsets, ids, xs)
    bad = np.nonzero(got != exp)[0]
    assert len(bad) == 0, (label, [(int(ids[i]), int(xs[i]), int(got[i]), int(exp[i])) for i in bad[:5]])


def test_contains_edge_sets(rg, ctx):
    bs = synth.BitmapSet.from_list(rgtest.edge_sets())
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    _check_contains(rg, ctx, bs, P, "edges")


def test_contains_mixed_packed_and_unpacked(rg, ctx):
    """The same queries on a mixed pool with and without packed metadata
    records (arrays of at most four values are then read from the record)."""
    bs = synth.mixed_small(n_bitmaps=24, seed=44)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    _check_contains(rg, ctx, bs, P, "mixed")
    P.pack_meta(ctx)
    _check_contains(rg, ctx, bs, P, "mixed-packed")
    tiny = synth.BitmapSet.from_list([np.array([3, 70000, 2**32 - 1], np.uint32),
                                      np.array([5 * 65536 + i for i in (0, 1, 9, 65535)], np.uint32),
                                      np.zeros(0, np.uint32)])
    T = rg.Pool.from_sets(tiny.values, tiny.offsets)
    T.pack_meta(ctx)
    _check_contains(rg, ctx, tiny, T, "inline-records")


def test_contains_bad_id_reported(rg, ctx):
    import torch

    bs = synth.mixed_small(n_bitmaps=3, seed=45)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    ids = np.array([0, 7, 2], np.uint32)
    xs = np.array([int(bs[0][0]), 5, int(bs[2][-1])], np.uint32)
    out = torch.full((3,), 9, dtype=torch.uint8, device="cuda")
    assert rg.roaring_contains(ctx, P, _t(ids), _t(xs), out) == rg.RG_OK
    with pytest.raises(rg.RoaringError):
        ctx.sync()
    assert out.cpu().numpy().tolist() == [1, 0, 1]


def _check_export(rg, ctx, bs, P, b0, n, label):
    _say(f"[export] {label}: bitmaps {b0}..{b0 + n}")
    offs, vals = rg.to_uint32(ctx, P, b0, n)
    offs = offs.cpu().numpy().astype(np.uint64)
    vals = vals.cpu().numpy().view(np.uint32)
    base = int(bs.offsets[b0])
    assert np.array_equal(offs, bs.offsets[b0:b0 + n + 1] - np.uint64(base)), label
    assert np.array_equal(vals, bs.values[base:int(bs.offsets[b0 + n])]), label


def test_export_edge_and_mixed(rg, ctx):
    es = synth.BitmapSet.from_list(rgtest.edge_sets())
    E = rg.Pool.from_sets(es.values, es.offsets)
    _check_export(rg, ctx, es, E, 0, len(es), "edges")
    for b in range(len(es)):
        _check_export(rg, ctx, es, E, b, 1, f"edges[{b}]")
    _check_export(rg, ctx, es, E, 3, 0, "empty range")
    bs = synth.mixed_small(n_bitmaps=30, seed=46)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    _check_export(rg, ctx, bs, P, 0, len(bs), "mixed")
    _check_export(rg, ctx, bs, P, 7, 11, "mixed[7:18]")


def test_export_capacity_and_range(rg, ctx):
    import torch

    bs = synth.mixed_small(n_bitmaps=5, seed=47)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    offs = torch.empty(6, dtype=torch.int64, device="cuda")
    vals = torch.empty(10, dtype=torch.int32, device="cuda")
    st, need = rg.roaring_to_uint32(ctx, P, 0, 5, offs, vals, 10)
    assert st == rg.RG_ECAPACITY and need == len(bs.values)
    st, _ = rg.roaring_to_uint32(ctx, P, 3, 3, offs, vals, 10)
    assert st == rg.RG_EINVAL


def test_export_of_materialised_results(rg, ctx):
    """Results of all four operations, exported from the output arena (a pool),
    equal the oracle's result lists."""
    bs = synth.mixed_small(n_bitmaps=16, seed=48)
    es = synth.BitmapSet.from_list(rgtest.edge_sets())
    sets = [bs[i] for i in range(len(bs))] + [es[i] for i in range(len(es))]
    al = synth.BitmapSet.from_list(sets)
    P = rg.Pool.from_sets(al.values, al.offsets)
    k = len(sets)
    ia = np.arange(k, dtype=np.uint32)
    ib = ((np.arange(k) * 5 + 3) % k).astype(np.uint32)
    for op in ("and", "or", "xor", "andnot"):
        out, _, _ = rg.batch(ctx, op, P, P, _t(ia), _t(ib), materialize=True)
        R = out.as_pool()
        offs, vals = rg.to_uint32(ctx, R, 0, k)
        offs = offs.cpu().numpy()
        vals = vals.cpu().numpy().view(np.uint32)
        for p in range(k):
            exp = oracle.op(op, sets[int(ia[p])], sets[int(ib[p])])
            assert np.array_equal(vals[offs[p]:offs[p + 1]], exp), (op, p)


def test_export_dense_bitsets(rg, ctx):
    """Bitset containers only (the dense workload's generator): values of a few
    bitmaps against the host twin of the generator."""
    import torch

    nb, nk = 6, 8
    words = torch.empty(nb * nk * 1024, dtype=torch.int64, device="cuda")
    synth.dense_bitsets_device(words.data_ptr(), 0, nb, nk, torch.cuda.current_stream().cuda_stream)
    P = rg.Pool.from_dense_words(ctx, words, nb, nk)
    offs, vals = rg.to_uint32(ctx, P, 0, nb)
    offs = offs.cpu().numpy()
    vals = vals.cpu().numpy().view(np.uint32)
    for b in range(nb):
        assert np.array_equal(vals[offs[b]:offs[b + 1]], synth.dense_bitmap_values(b, nk)), b
