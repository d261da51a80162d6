"""Batched plans on the GPU: persistent work-stealing execution, hipGraph
capture and replay, autotuning - all against the oracle and the eager path."""
import sys

import numpy as np
import pytest

import oracle
import synth
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


@pytest.fixture(scope="module")
def ctx(rg):
    c = rg.Context(0)
    yield c
    c.close()


def _t(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def _expect(bs, ia, ib, op):
    card = np.array([oracle.count(op, bs[int(x)], bs[int(y)]) for x, y in zip(ia, ib)], np.uint64)
    jac = np.array([oracle.jaccard(bs[int(x)], bs[int(y)]) for x, y in zip(ia, ib)])
    return card, jac


def _workloads():
    sets = rgtest.edge_sets()
    k = len(sets)
    yield "edges", synth.BitmapSet.from_list(sets), np.repeat(np.arange(k), k), np.tile(np.arange(k), k)
    bs = synth.mixed_small()
    ia, ib = synth.consecutive_pairs(len(bs))
    yield "mixed", bs, ia, ib
    bs, ia, ib = synth.array_stress(n_pairs=4000)
    yield "array-stress", bs, ia, ib


@pytest.mark.parametrize("which", ["edges", "mixed", "array-stress"])
def test_plan_matches_oracle(rg, ctx, which):
    import torch

    name, bs, ia, ib = next(w for w in _workloads() if w[0] == which)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    for op in OPS:
        _say(f"[plan {name}] op={op} pairs={len(ia)}")
        card, jac = _expect(bs, ia, ib, op)
        pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True)
        for rep in range(2):
            pl.cards.zero_()
            pl.jacc.zero_()
            pl.execute()
            torch.cuda.synchronize()
            assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), card), (name, op, rep)
            assert np.array_equal(pl.jacc.cpu().numpy(), jac), (name, op, rep)
        pl.close()


def test_plan_graph_replays_match_eager(rg, ctx):
    """Capture once on a side stream; replay several times with eager work and
    synchronisations in between; every replay equals the eager result."""
    import torch

    bs = synth.mixed_small(n_bitmaps=40, seed=21)
    ia, ib = synth.random_pairs(len(bs), 300, seed=21)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    for op in ("and", "xor"):
        _, eager_cards, eager_jacc = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True, jaccard=True)
        torch.cuda.synchronize()
        eager_cards = eager_cards.cpu().numpy().copy()
        eager_jacc = eager_jacc.cpu().numpy().copy()
        card, jac = _expect(bs, ia, ib, op)
        assert np.array_equal(eager_cards.view(np.uint64), card)
        side = torch.cuda.Stream()
        pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True, stream=side)
        torch.cuda.synchronize()
        pl.capture(side)
        assert pl.info()["graph"]
        for rep in range(4):
            pl.cards.zero_()
            pl.jacc.zero_()
            torch.cuda.synchronize()
            with torch.cuda.stream(side):
                pl.execute(side)
            side.synchronize()
            assert np.array_equal(pl.cards.cpu().numpy(), eager_cards), (op, rep)
            assert np.array_equal(pl.jacc.cpu().numpy(), eager_jacc), (op, rep)
            # eager work between replays
            rg.batch(ctx, "or", P, P, tia, tib, materialize=False, card=True)
            torch.cuda.synchronize()
        pl.close()


def test_plan_tune_keeps_results(rg, ctx):
    import torch

    bs, ia, ib = synth.array_stress(n_pairs=2000)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    card, jac = _expect(bs, ia, ib, "and")
    pl = rg.Plan(ctx, "and", P, P, tia, tib, card=True, jaccard=True)
    pl.tune(reps=1)
    info = pl.info()
    _say(f"[tune] chose {info}")
    pl.cards.zero_()
    pl.execute()
    torch.cuda.synchronize()
    assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), card)
    assert np.array_equal(pl.jacc.cpu().numpy(), jac)
    for g, r, tm in [(256, 8, 0), (4096, 1000, 64), (512, 32, 4096)]:
        pl.set(g, r, tm)
        pl.cards.zero_()
        pl.execute()
        torch.cuda.synchronize()
        assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), card), (g, r, tm)
    pl.close()


def test_plan_tune_cache(rg, ctx, tmp_path):
    """A tuned setting is stored in the JSON cache under the plan's key and
    applied to the next plan of the same shape without tuning; results equal."""
    import json

    import torch

    bs, ia, ib = synth.array_stress(n_pairs=1500)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    card, jac = _expect(bs, ia, ib, "xor")
    cache = str(tmp_path / "tune.json")
    pl = rg.Plan(ctx, "xor", P, P, tia, tib, card=True, jaccard=True)
    pl.tune(reps=1, cache=cache)
    chosen = pl.info()
    pl.close()
    table = json.load(open(cache))
    assert len(table) == 1
    stored = next(iter(table.values()))
    assert stored == {k: chosen[k] for k in ("grid", "gallop_ratio", "thread_max")}
    # a different setting is stored by hand: the next plan must take it from the cache
    key = next(iter(table))
    table[key] = {"grid": 256, "gallop_ratio": 8, "thread_max": 16}
    json.dump(table, open(cache, "w"))
    pl2 = rg.Plan(ctx, "xor", P, P, tia, tib, card=True, jaccard=True)
    pl2.tune(reps=1, cache=cache)
    info = pl2.info()
    assert (info["grid"], info["gallop_ratio"], info["thread_max"]) == (256, 8, 16)
    pl2.execute()
    torch.cuda.synchronize()
    assert np.array_equal(pl2.cards.cpu().numpy().view(np.uint64), card)
    assert np.array_equal(pl2.jacc.cpu().numpy(), jac)
    pl2.close()


def test_plan_two_pools(rg, ctx):
    """A plan whose pairs take A from one pool and B from another (each pool's
    container metadata packed separately) gives the oracle's counts."""
    import torch

    a_bs = synth.mixed_small(n_bitmaps=10, seed=31)
    b_bs = synth.BitmapSet.from_list(rgtest.edge_sets())
    A = rg.Pool.from_sets(a_bs.values, a_bs.offsets)
    B = rg.Pool.from_sets(b_bs.values, b_bs.offsets)
    ia = np.repeat(np.arange(len(a_bs)), len(b_bs)).astype(np.uint32)
    ib = np.tile(np.arange(len(b_bs)), len(a_bs)).astype(np.uint32)
    for op in OPS:
        exp, _, jexp = oracle.pairs(op, a_bs.values, a_bs.offsets, b_bs.values, b_bs.offsets, ia, ib,
                                    want_jaccard=True)
        pl = rg.Plan(ctx, op, A, B, _t(ia), _t(ib), card=True, jaccard=True)
        pl.execute()
        torch.cuda.synchronize()
        assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), exp), op
        assert np.array_equal(pl.jacc.cpu().numpy(), jexp), op
        pl.close()


def test_plan_errors(rg, ctx):
    import torch

    bs = synth.mixed_small(n_bitmaps=3, seed=22)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    with pytest.raises(rg.RoaringError):
        rg.Plan(ctx, "and", P, P, _t(np.array([0, 9], np.uint32)), _t(np.array([1, 1], np.uint32)))


def _uneven_pool(n_bitmaps=256, n_pairs=3000):
    """The shape of the batched uneven workload at a size the oracle checks in
    seconds: cardinalities lognormal (median 1e4, sigma 2, clipped to
    [10, 1e7]) over [0, 2^32), the mixed recipe with a 256-key hot set, random
    pairs."""
    seed = synth.SEED_BASE + 3
    hot = synth.hot_keys(seed, 256, 1 << 16)
    sets = [synth.mixed_bitmap(seed, i, synth.lognormal_card(i, 1e4, 2.0, 10, 10 ** 7, seed), 32, hot)
            for i in range(n_bitmaps)]
    bs = synth.BitmapSet.from_list(sets)
    ia, ib = synth.random_pairs(n_bitmaps, n_pairs, seed)
    return bs, ia, ib


def test_uneven_shape_eager_and_plan_match_oracle(rg, ctx):
    """Every pair's count and Jaccard index, from the eager batched call and
    from a plan (executed and replayed as a graph), equal the oracle's."""
    import torch

    bs, ia, ib = _uneven_pool()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    stream = torch.cuda.Stream()
    for op in OPS:
        _say(f"[uneven] op={op} pairs={len(ia)} values={len(bs.values)}")
        card, _, jac = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_jaccard=True)
        _, c, j = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True, jaccard=True)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().view(np.uint64), card), op
        assert np.array_equal(j.cpu().numpy(), jac), op
        pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True)
        with torch.cuda.stream(stream):
            pl.capture(stream)
            for rep in range(2):
                pl.cards.zero_()
                pl.jacc.zero_()
                pl.execute(stream)
                stream.synchronize()
                assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), card), (op, rep)
                assert np.array_equal(pl.jacc.cpu().numpy(), jac), (op, rep)
        pl.close()


def _check_mat_result(rg, ctx, label, op, bs, ia, ib, pool, cards, jacc, full=True):
    """Every pair's result bitmap against the oracle: fingerprint, and when full
    the decoded values and container metadata; counts and Jaccard index."""
    assert rg.rg_pool_validate(ctx, pool) == 0, (label, op)
    dig = rg.rg_pool_digest(ctx, pool).cpu().numpy().view(np.uint64)
    c = cards.cpu().numpy().view(np.uint64)
    j = jacc.cpu().numpy()
    card_e, dig_e, jac_e = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_digest=True,
                                        want_jaccard=True)
    assert np.array_equal(dig[:len(ia)], dig_e), (label, op)
    assert np.array_equal(c, card_e) and np.array_equal(j, jac_e), (label, op)
    if full:
        h = pool.to_host()
        for p in range(len(ia)):
            exp = oracle.op(op, bs[int(ia[p])], bs[int(ib[p])])
            got, meta = rgtest.decode_bitmap(h, p)
            assert np.array_equal(got, exp), (label, op, p)
            assert meta == rgtest.oracle_meta(oracle, exp), (label, op, p)


@pytest.mark.parametrize("which", ["edges", "mixed", "array-stress"])
def test_materialising_plan_replays_match_oracle(rg, ctx, which):
    """A materialising plan captured in a hipGraph and replayed three times,
    with eager calls of the same context in between and the arena wiped before
    each replay: every replay's results equal the oracle's."""
    import torch

    label, bs, ia, ib = [w for w in _workloads() if w[0] == which][0]
    ia, ib = ia.astype(np.uint32), ib.astype(np.uint32)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    stream = torch.cuda.Stream()
    for op in OPS:
        _say(f"[mat plan {label}] op={op} pairs={len(ia)}")
        pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True, materialize=True, stream=stream)
        with torch.cuda.stream(stream):
            pl.capture(stream)
            for rep in range(3):
                for t in (pl.out.keys, pl.out.types, pl.out.card, pl.out.payload, pl.out.bm_begin):
                    t.fill_(0x55)
                pl.cards.zero_()
                pl.jacc.zero_()
                pl.execute(stream)
                stream.synchronize()
                # an eager call of the same context between replays
                _, c2, _ = rg.batch(ctx, "xor", P, P, tia, tib, materialize=False, card=True)
                torch.cuda.synchronize()
                R = pl.result(stream)
                _check_mat_result(rg, ctx, label, op, bs, ia, ib, R, pl.cards, pl.jacc, full=rep == 0)
        pl.close()


def test_materialising_plan_in_waves_uneven_shape(rg, ctx):
    """The batched uneven shape materialised in arena-sized waves: the wave size
    cut so that the plan runs in many waves, every pair's fingerprint, count and
    Jaccard index against the oracle, for all four operations, and equal to the
    eager materialising call."""
    import torch

    bs, ia, ib = _uneven_pool(n_bitmaps=128, n_pairs=600)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    stream = torch.cuda.Stream()
    ctx.set_wave_slots(20000)
    try:
        for op in OPS:
            pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True, materialize=True, stream=stream)
            info = pl.info()
            _say(f"[mat plan uneven] op={op} pairs={len(ia)} {info}")
            assert info["waves"] > 3
            with torch.cuda.stream(stream):
                pl.capture(stream)
                for rep in range(2):
                    pl.execute(stream)
                    stream.synchronize()
                    R = pl.result(stream)
                    _check_mat_result(rg, ctx, "uneven", op, bs, ia, ib, R, pl.cards, pl.jacc, full=False)
            out, _, _ = rg.batch(ctx, op, P, P, tia, tib, materialize=True)
            torch.cuda.synchronize()
            d_eager = rg.rg_pool_digest(ctx, out.as_pool()).cpu().numpy()
            d_plan = rg.rg_pool_digest(ctx, R).cpu().numpy()
            assert np.array_equal(d_eager, d_plan), op
            pl.close()
    finally:
        ctx.set_wave_slots(1 << 24)


def test_materialising_plan_errors(rg, ctx):
    bs = synth.mixed_small(n_bitmaps=5, seed=61)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    with pytest.raises(rg.RoaringError):  # pair index outside the pool
        rg.Plan(ctx, "or", P, P, _t(np.array([0, 9], np.uint32)), _t(np.array([1, 1], np.uint32)), materialize=True)
    ia, ib = _t(np.array([0, 1], np.uint32)), _t(np.array([1, 2], np.uint32))
    out = rg.OutArena(2, 1, 16)
    import ctypes

    h = ctypes.c_void_p()
    st = rg.lib().rg_plan_create_mat(ctx.h, 1, ctypes.byref(P.c), ctypes.byref(P.c), rg._ptr(ia), rg._ptr(ib), 2,
                                     rg.RG_FLAG_MATERIALIZE, ctypes.byref(out.c), None, None, ctypes.byref(h), None)
    assert st == rg.RG_ECAPACITY and out.c.needed_containers > 1 and out.c.needed_payload_bytes > 16
