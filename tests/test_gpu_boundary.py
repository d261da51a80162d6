"""The C-ABI conventions on the GPU: count-only calls that never wait for the
device (errors reported by rg_sync), calls on a caller-owned workspace
(no device allocation, RG_ECAPACITY when it is too small), the host form of
the Jaccard index, and calls that share the context's workspace from two
streams."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp
from tests import rgtest

pytestmark = pytest.mark.gpu

OPS = ("and", "or", "xor", "andnot")


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


def test_async_count_reports_bad_index_through_sync(rg):
    import torch

    ctx = rg.Context(0)
    bs = synth.mixed_small(n_bitmaps=4, seed=21)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    ia = np.array([0, 9, 2], np.uint32)  # 9 is outside the pool
    ib = np.array([1, 1, 3], np.uint32)
    cards = torch.full((3,), 7, dtype=torch.int64, device="cuda")
    jacc = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    st = rg.roaring_batch(ctx, "and", P, P, _t(ia), _t(ib), rg.RG_FLAG_CARD | rg.RG_FLAG_JACCARD, None, cards, jacc)
    assert st == rg.RG_OK  # the call does not wait for the device
    with pytest.raises(rg.RoaringError) as e:
        ctx.sync()
    assert e.value.status == rg.RG_EINVAL
    ctx.sync()  # the flag was cleared
    c = cards.cpu().numpy()
    j = jacc.cpu().numpy()
    assert c[1] == 0 and j[1] == 0.0
    for p in (0, 2):
        a, b = bs[int(ia[p])], bs[int(ib[p])]
        assert c[p] == oracle.count("and", a, b) and j[p] == oracle.jaccard(a, b)
    # a materialising call checks the indices itself
    out = rg.OutArena(3, 1 << 12, 1 << 20)
    assert rg.roaring_batch(ctx, "and", P, P, _t(ia), _t(ib), rg.RG_FLAG_MATERIALIZE, out) == rg.RG_EINVAL
    ctx.close()


def test_jaccard_host(rg):
    ctx = rg.Context(0)
    sets = rgtest.edge_sets()
    bs = synth.BitmapSet.from_list(sets)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    for a in range(len(sets)):
        for b in (0, 1, 9, len(sets) - 1):
            assert rg.roaring_jaccard_host(ctx, P, a, P, b) == oracle.jaccard(sets[a], sets[b]), (a, b)
    ctx.close()


def _mixed_case():
    bs = synth.mixed_small(n_bitmaps=40, seed=33)
    ia, ib = synth.random_pairs(len(bs), 300, seed=33)
    return bs, ia, ib


def test_caller_workspace_count_only_no_growth(rg):
    """Count-only batches on a workspace of exactly rg_workspace_size bytes give
    the oracle's counts and leave the device's free memory unchanged; a
    256-byte workspace is RG_ECAPACITY."""
    import torch

    ctx = rg.Context(0)
    bs, ia, ib = _mixed_case()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    flags = rg.RG_FLAG_CARD | rg.RG_FLAG_JACCARD
    need = ctx.workspace_size("and", flags, P, P, len(ia))
    assert need > 0 and need % 256 == 0
    cards = torch.zeros(len(ia), dtype=torch.int64, device="cuda")
    jacc = torch.zeros(len(ia), dtype=torch.float64, device="cuda")
    # every kernel once on the context's own workspace (code objects load on first use)
    for op in OPS:
        ctx.check(rg.roaring_batch(ctx, op, P, P, tia, tib, flags, None, cards, jacc))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ctx.set_workspace(small)
    assert rg.roaring_batch(ctx, "and", P, P, tia, tib, flags, None, cards, jacc) == rg.RG_ECAPACITY
    ctx.set_workspace(ws)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = {}
    for op in OPS:
        cards.zero_()
        ctx.check(rg.roaring_batch(ctx, op, P, P, tia, tib, flags, None, cards, jacc))
        ctx.sync()
        got[op] = (cards.cpu().numpy().view(np.uint64).copy(), jacc.cpu().numpy().copy())
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    for op in OPS:
        exp, _, jexp = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_jaccard=True)
        assert np.array_equal(got[op][0], exp), op
        assert np.array_equal(got[op][1], jexp), op
    ctx.set_workspace(None)
    ctx.close()


@pytest.mark.parametrize("op", OPS)
def test_caller_workspace_materialised_minimum(rg, op):
    """A materialising batch on the least workspace rg_workspace_size reports
    runs in several waves and builds the oracle's results."""
    import torch

    ctx = rg.Context(0)
    bs, ia, ib = _mixed_case()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    flags = rg.RG_FLAG_MATERIALIZE | rg.RG_FLAG_CARD
    need = ctx.workspace_size(op, flags, P, P, len(ia))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    ctx.set_workspace(ws)
    out, cards, _ = rg.batch(ctx, op, P, P, tia, tib, materialize=True, card=True)
    torch.cuda.synchronize()
    res = out.as_pool()
    assert rg.rg_pool_validate(ctx, res) == 0
    dig = rg.rg_pool_digest(ctx, res).cpu().numpy().view(np.uint64)
    exp_c, exp_d, _ = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_digest=True)
    assert np.array_equal(cards.cpu().numpy().view(np.uint64), exp_c)
    assert np.array_equal(dig, exp_d)
    ctx.set_workspace(None)
    ctx.close()


def test_workspace_shared_across_streams(rg):
    """A count-only batch on one stream and a dispatcher gradient on another,
    issued back to back in both orders, share the context's workspace: both
    results stay right (counts against the oracle, gradient against the fp64
    reference)."""
    import torch

    ctx = rg.Context(0)
    bs, ia, ib = _mixed_case()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    exp, _, _ = oracle.pairs("xor", bs.values, bs.offsets, bs.values, bs.offsets, ia, ib)
    rng = np.random.default_rng(5)
    n = 4000
    p = rng.normal(0.0, 0.3, mlp.N_PARAMS).astype(np.float32)
    x = rng.normal(0.0, 1.0, (n, 12)).astype(np.float32)
    t = rng.normal(0.0, 1.0, (n, 6)).astype(np.float32)
    m = (rng.random((n, 6)) < 0.7).astype(np.uint8)
    tp, tx, tt, tm = (torch.from_numpy(a).cuda() for a in (p, x, t, m))
    g0 = mlp.grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), m.astype(np.float64))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for order in (0, 1):
        cards = torch.zeros(len(ia), dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()  # inputs and outputs are ready before the two streams start
        calls = [lambda: ctx.check(rg.roaring_batch(ctx, "xor", P, P, tia, tib, rg.RG_FLAG_CARD, None, cards,
                                                    None, s1)),
                 lambda: rg.mlp_grad(ctx, tp, tx, tt, tm, stream=s2)]
        res = [None, None]
        for i in ((0, 1) if order == 0 else (1, 0)):
            res[i] = calls[i]()
        torch.cuda.synchronize()
        assert np.array_equal(cards.cpu().numpy().view(np.uint64), exp), order
        g = res[1][0].cpu().numpy().astype(np.float64)
        assert np.abs(g - g0).max() <= 1e-4 * np.abs(g0).max() + 1e-7, order
    ctx.close()


def test_materialised_calls_ignore_stale_workspace(rg):
    """Materialising calls write every workspace slot they later read: on a
    caller workspace filled with random bytes, then with 0xFF bytes, all four
    operations give the oracle's results, one pool and two. (The first design
    of materialised union and symmetric difference placed each key at its
    merged position and left the slot after every matched key unwritten, so
    those slots held what an earlier call had left there.)"""
    import torch

    ctx = rg.Context(0)
    bs = synth.mixed_small(n_bitmaps=30, seed=34)
    es = synth.BitmapSet.from_list(rgtest.edge_sets())
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    E = rg.Pool.from_sets(es.values, es.offsets)
    ia, ib = synth.random_pairs(len(bs), 200, seed=34)
    ja = (np.arange(60) % len(es)).astype(np.uint32)
    jb = (np.arange(60) * 7 % len(bs)).astype(np.uint32)
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(35)
    for fill in ("random", "ones"):
        for (A, B, xa, xb, sa, sb) in ((P, P, ia, ib, bs, bs), (E, P, ja, jb, es, bs)):
            for op in OPS:
                if fill == "random":
                    ws.random_(0, 256, generator=gen)
                else:
                    ws.fill_(255)
                torch.cuda.synchronize()
                ctx.set_workspace(ws)
                _say(f"[stale workspace] {fill} op={op} pairs={len(xa)}")
                out, cards, jacc = rg.batch(ctx, op, A, B, _t(xa), _t(xb), materialize=True, card=True,
                                            jaccard=True)
                torch.cuda.synchronize()
                ctx.set_workspace(None)
                dig = rg.rg_pool_digest(ctx, out.as_pool()).cpu().numpy().view(np.uint64)
                c = cards.cpu().numpy().view(np.uint64)
                j = jacc.cpu().numpy()
                ec, ed, ej = oracle.pairs(op, sa.values, sa.offsets, sb.values, sb.offsets, xa, xb, want_digest=True,
                                          want_jaccard=True)
                assert np.array_equal(dig[:len(xa)], ed), (fill, op)
                assert np.array_equal(c, ec) and np.array_equal(j, ej), (fill, op)
    ctx.close()


def test_inconsistent_cardinality_is_a_capacity_error(rg):
    """A caller-built pool whose stored cardinality understates a container's
    values: materialised union through the k-way kernels finds the result
    longer than its slot at the end of the arena and fails with
    RG_ECAPACITY instead of writing past it."""
    import torch

    vals = np.arange(1000, 1200, 2, dtype=np.uint32)  # one array container of 100 values (100 runs)
    n, nc, pb, h = rg.Pool.host_arrays(vals, np.array([0, len(vals)], np.uint64))
    h["card"][0] = 50                       # understated
    h["bm_card"][0] = 50
    h["bm_wbytes"][0] = 112                 # roundup16(2 * 50)
    e = rg.Pool.host_arrays(np.zeros(0, np.uint32), np.array([0, 0], np.uint64))[3]
    A = rg.Pool.from_host_arrays(h)
    B = rg.Pool.from_host_arrays(e)
    ctx = rg.Context(0)
    out = rg.OutArena(1, 1, 112)
    ia = _t(np.array([0], np.uint32))
    st = rg.roaring_batch(ctx, "or", A, B, ia, ia, rg.RG_FLAG_MATERIALIZE, out)
    assert st == rg.RG_ECAPACITY, st
    torch.cuda.synchronize()
    ctx.close()
