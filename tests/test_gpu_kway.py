"""k-way intersection / union (roaring_multi) and the serving loop on the GPU,
against the oracle's left fold (k-way semantics as defined for the serving
workload: AND / OR of k bitmaps of one pool)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import rgtest

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


def overlapping_sets(n=24, seed=7):
    """Bitmaps that share most of their content, so that k-way intersections
    are non-empty and cross every container type: each is one of two mixed base
    bitmaps (two thirds use the first), whole for every fourth bitmap (runs
    intact) and otherwise thinned to a seeded 85 %, plus a few private values."""
    hot = synth.hot_keys(seed, 16, 1 << 10)
    bases = [synth.mixed_bitmap(seed, i, 40000, 26, hot) for i in range(2)]
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        b = bases[1 if i % 3 == 0 else 0]
        keep = b if i % 4 == 0 else b[rng.random(len(b)) < 0.85]
        extra = rng.integers(0, 1 << 26, 500).astype(np.uint32)
        out.append(np.unique(np.concatenate([keep, extra])).astype(np.uint32))
    return synth.BitmapSet.from_list(out)


def _queries(n_bitmaps, n, seed, kmax=8, ops=("and", "or")):
    rng = np.random.default_rng(seed)
    qs = []
    for i in range(n):
        k = int(rng.integers(1, kmax + 1))
        ids = rng.choice(n_bitmaps, size=k, replace=(i % 4 == 0)).astype(np.uint32)
        qs.append((ops[i % len(ops)], ids))
    return qs


def _workload(which):
    if which == "overlapping":
        return overlapping_sets()
    if which == "edges":
        return synth.BitmapSet.from_list(rgtest.edge_sets())
    return synth.mixed_small(n_bitmaps=30)


@pytest.mark.parametrize("kidx", [False, True], ids=["search", "key-index"])
@pytest.mark.parametrize("which", ["overlapping", "edges", "mixed"])
def test_multi_matches_oracle(rg, ctx, which, kidx):
    import torch

    bs = _workload(which)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    if kidx:
        P.key_index(ctx)
    qs = _queries(len(bs), 16, seed=11)
    # symmetric difference (parity of k) and difference (first minus the others)
    qs += _queries(len(bs), 8, seed=12, kmax=5, ops=("xor", "andnot"))
    # k at the limit: 256 ids (repeats allowed)
    qs.append(("and", np.resize(np.arange(min(3, len(bs)), dtype=np.uint32), 256)))
    qs.append(("or", np.resize(np.arange(len(bs), dtype=np.uint32), 256)))
    n_nonempty_and = 0
    for op, ids in qs:
        _say(f"[multi {which}] op={op} k={len(ids)}")
        exp = oracle.kway(op, [bs[int(i)] for i in ids])
        n_nonempty_and += op == "and" and len(exp) > 0
        tids = torch.from_numpy(ids.view(np.int32)).cuda()
        out, card = rg.multi(ctx, op, P, tids, materialize=True, card=True)
        torch.cuda.synchronize()
        assert int(card[0].item()) == len(exp), (which, op, ids)
        res = out.as_pool()
        assert rg.rg_pool_validate(ctx, res) == 0
        assert int(rg.rg_pool_digest(ctx, res).cpu().numpy().view(np.uint64)[0]) == oracle.digest(exp)
        h = res.to_host()
        got, meta = rgtest.decode_bitmap(h, 0)
        assert np.array_equal(got, exp), (which, op, ids)
        assert meta == rgtest.oracle_meta(oracle, exp), (which, op, ids)
        _, card2 = rg.multi(ctx, op, P, tids, materialize=False, card=True)
        assert int(card2[0].item()) == len(exp)
    if which == "overlapping":
        assert n_nonempty_and >= 3  # the workload does exercise non-empty intersections


def test_multi_errors(rg, ctx):
    import torch

    bs = synth.mixed_small(n_bitmaps=4, seed=5)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    card = torch.zeros(1, dtype=torch.int64, device="cuda")

    def call(op, ids, flags=rg.RG_FLAG_CARD):
        t = torch.tensor(np.asarray(ids, np.uint32).view(np.int32), device="cuda")
        return rg.roaring_multi(ctx, op, P, t, flags, None, card)

    assert call(7, [0, 1]) == rg.RG_EINVAL
    assert call("and", [0, 9]) == rg.RG_EINVAL
    assert call("and", [0] * 257) == rg.RG_EINVAL
    assert call("or", [0, 1], flags=0) == rg.RG_EINVAL
    out = rg.OutArena(1, 0, 0, "cuda")
    out.c.cap_containers = 0
    out.c.cap_payload_bytes = 0
    t = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    assert rg.roaring_multi(ctx, "or", P, t, rg.RG_FLAG_MATERIALIZE, out, None) == rg.RG_ECAPACITY
    assert out.c.needed_containers > 0 and out.c.needed_payload_bytes > 0


def _expect(bs, qs):
    res = []
    for op, ids, mat in qs:
        e = oracle.kway(op, [bs[int(i)] for i in ids])
        res.append((len(e), oracle.digest(e) if mat else 0))
    return res


def test_server_results_alone_and_in_mix(rg, ctx):
    """Each query's result (cardinality, container-form fingerprint) is the
    oracle's, whether it runs alone (one query per step) or in the mix."""
    bs = overlapping_sets()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    base = _queries(len(bs), 48, seed=23, kmax=12)
    qs = [(op, ids, i % 5 != 4) for i, (op, ids) in enumerate(base)]
    exp = _expect(bs, qs)
    # alone: one query per step, one step in flight
    alone = rg.Server(ctx, P, arena_bytes=256 << 20, max_batch=1, max_inflight=1)
    lat, cards, dig = alone.replay(qs, np.zeros(len(qs), np.uint64), digest=True)
    st = alone.stop()
    _say(f"[serve alone] {st}")
    assert st["steps"] == len(qs)
    for i, (c, d) in enumerate(exp):
        assert cards[i] == c and dig[i] == d, ("alone", i)
    # in the mix: all arrive at once, batched, two steps in flight
    mix = rg.Server(ctx, P, arena_bytes=256 << 20, max_batch=16, max_inflight=2)
    lat2, cards2, dig2 = mix.replay(qs, np.zeros(len(qs), np.uint64), digest=True)
    st2 = mix.stop()
    _say(f"[serve mix] {st2}")
    assert st2["mean_batch"] > 1.0
    assert np.array_equal(cards2, cards) and np.array_equal(dig2, dig)
    # spread arrivals (continuous batching while steps run)
    mix = rg.Server(ctx, P, arena_bytes=256 << 20, max_batch=8, max_inflight=2)
    lat3, cards3, dig3 = mix.replay(qs, np.arange(len(qs), dtype=np.uint64) * 20000, digest=True)
    st3 = mix.stop()
    _say(f"[serve spread] {st3} p50={np.percentile(lat3, 50) / 1e3:.1f}us p99={np.percentile(lat3, 99) / 1e3:.1f}us")
    assert np.array_equal(cards3, cards) and np.array_equal(dig3, dig)


def test_server_digest_only_when_asked(rg, ctx):
    """Fingerprints are computed for the queries that ask for them (and
    only the steps holding such a query run the fingerprint kernel); the
    others read 0, with the same cardinalities."""
    bs = overlapping_sets(n=12, seed=5)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    qs = [(op, ids, True) for op, ids in _queries(len(bs), 24, seed=29, kmax=6)]
    exp = _expect(bs, qs)
    srv = rg.Server(ctx, P, arena_bytes=64 << 20, max_batch=8, max_inflight=2)
    try:
        _, cards, dig = srv.replay(qs, np.zeros(len(qs), np.uint64))
        assert [int(c) for c in cards] == [e[0] for e in exp]
        assert not dig.any()
        tickets = [srv.submit(op, ids, materialize=m, digest=i % 2 == 0) for i, (op, ids, m) in enumerate(qs)]
        for i, t in enumerate(tickets):
            r = srv.poll(t)
            assert r.done and r.status == 0 and r.card == exp[i][0], i
            assert r.digest == (exp[i][1] if i % 2 == 0 else 0), i
            srv.release(t)
    finally:
        srv.stop()


def test_server_views_and_small_arena(rg, ctx):
    """Materialised results are readable through the view until released; an
    arena that holds only a few queries at a time still serves every query."""
    import torch

    bs = overlapping_sets(n=12, seed=3)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    qs = [(op, ids, True) for op, ids in _queries(len(bs), 20, seed=31, kmax=6)]
    exp = _expect(bs, qs)
    srv = rg.Server(ctx, P, arena_bytes=8 << 20, max_batch=4, max_inflight=2)
    try:
        tickets = [srv.submit(op, ids, materialize=m, digest=True) for op, ids, m in qs]
        for i, t in enumerate(tickets):
            r = srv.poll(t, wait=True)
            assert r.done and r.status == 0 and r.card == exp[i][0] and r.digest == exp[i][1], i
            if i < 6 and r.n_containers:
                # the view is a window into the step's arrays: its containers need
                # not start at 0 (query i of a step)
                view = rg.Pool.from_view(r.view)
                assert int(rg.rg_pool_digest(ctx, view).cpu().numpy().view(np.uint64)[0]) == exp[i][1]
                torch.cuda.synchronize()
            srv.release(t)
    finally:
        st = srv.stop()
    _say(f"[serve small arena] {st}")
    assert st["queries"] == len(qs)
    with pytest.raises(rg.RoaringError):
        srv2 = rg.Server(ctx, P, arena_bytes=1 << 20, max_batch=4, max_inflight=2)
        try:
            srv2.submit("or", np.resize(np.arange(12, dtype=np.uint32), 256), materialize=True)
        finally:
            srv2.stop()


def test_server_all_ops_while_context_busy(rg, ctx):
    """Queries of all four operations, served while the owner of the context
    keeps making pairwise calls on it: both sides give the oracle's results."""
    import torch

    bs = overlapping_sets(n=16, seed=8)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    qs = [(op, ids, i % 3 != 2) for i, (op, ids) in
          enumerate(_queries(len(bs), 40, seed=41, kmax=7, ops=("and", "or", "xor", "andnot")))]
    exp = _expect(bs, qs)
    ia = np.arange(0, 15, dtype=np.uint32)
    ib = np.arange(1, 16, dtype=np.uint32)
    tia = torch.from_numpy(ia.view(np.int32)).cuda()
    tib = torch.from_numpy(ib.view(np.int32)).cuda()
    srv = rg.Server(ctx, P, arena_bytes=64 << 20, max_batch=8, max_inflight=2)
    try:
        tickets = [srv.submit(op, ids, materialize=m, digest=True) for op, ids, m in qs]
        for rep in range(3):
            for op in ("and", "or", "xor", "andnot"):
                _, c, _ = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True)
                torch.cuda.synchronize()
                c = c.cpu().numpy().view(np.uint64)
                for p in range(len(ia)):
                    assert int(c[p]) == oracle.count(op, bs[int(ia[p])], bs[int(ib[p])]), (rep, op, p)
        for i, t in enumerate(tickets):
            r = srv.poll(t, wait=True)
            assert r.done and r.status == 0 and r.card == exp[i][0] and r.digest == exp[i][1], (i, qs[i][0])
            srv.release(t)
    finally:
        st = srv.stop()
    _say(f"[serve all ops, busy context] {st}")


def _kway_bounds(op, sets):
    """The result bounds of a k-way query written out from the bitmaps: keys
    between the extreme first and last keys (union, symmetric difference) or
    the inner ones (intersection), capped by the key counts; payload bytes
    capped by 8 KiB per container."""
    keys = [np.unique(np.asarray(v, np.uint64) >> np.uint64(16)) for v in sets]
    wb = []
    for v in sets:
        c = oracle.containers(np.asarray(v, np.uint32))
        wb.append(int(sum(((min(8192, 2 * int(x)) + 15) // 16) * 16 for x in c["card"])))
    nk = [len(k) for k in keys]
    nonempty = [k for k in keys if len(k)]
    if op == "and":
        kb = 0
        if all(nk):
            lo, hi = max(int(k[0]) for k in keys), min(int(k[-1]) for k in keys)
            kb = min(min(nk), hi - lo + 1) if hi >= lo else 0
        pb = min(wb)
    elif op == "andnot":
        kb, pb = nk[0], wb[0]
    else:
        kb = min(sum(nk), max(int(k[-1]) for k in nonempty) - min(int(k[0]) for k in nonempty) + 1) if nonempty else 0
        pb = sum(wb)
    return kb, min(pb, kb * 8192)


def span_sets():
    """Bitmaps built to exercise the key bounds (first and last key of each
    bitmap: intersections of overlapping, disjoint and empty key ranges, unions
    reaching key 65535) and the split key passes (unions of more than 4096 keys,
    intersections of more than four bitmaps)."""
    rng = np.random.default_rng(31)

    def over(keys, per_key):
        keys = np.asarray(keys, np.uint32)
        lows = rng.integers(0, 65536, (len(keys), per_key)).astype(np.uint32)
        return np.unique(((keys[:, None] << np.uint32(16)) | lows).ravel())

    sets = [
        over(np.arange(10, 21), 300),         # 0: keys 10..20
        over(np.arange(15, 31), 5000),        # 1: keys 15..30 (bitsets)
        over(np.arange(40, 51), 50),          # 2: keys 40..50
        np.zeros(0, np.uint32),               # 3: empty
        over(np.arange(65530, 65536), 20),    # 4: keys 65530..65535
        over(np.arange(0, 6), 20),            # 5: keys 0..5
    ]
    # 6..11: 3000 keys each, one to three values per key, sharing half their keys
    common = rng.choice(65536, 1500, replace=False)
    for i in range(6):
        own = rng.choice(65536, 1500, replace=False)
        sets.append(np.unique(np.concatenate([over(common, 1 + i % 3), over(own, 1)])))
    return synth.BitmapSet.from_list(sets)


@pytest.mark.parametrize("kidx", [False, True], ids=["search", "key-index"])
def test_multi_key_spans_and_split_passes(rg, ctx, kidx):
    import torch

    bs = span_sets()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    if kidx:
        P.key_index(ctx)
    u = lambda *ids: np.array(ids, np.uint32)
    big = np.arange(6, 12, dtype=np.uint32)
    qs = [
        ("and", u(0, 1, 1)), ("and", u(0, 2, 1)), ("and", u(0, 3, 1)), ("and", u(1, 0, 1, 0, 1)),
        ("or", u(4, 5, 0)), ("xor", u(4, 5, 4)), ("or", u(3, 3, 3)), ("or", u(3, 4, 3)),
        ("or", big), ("xor", np.concatenate([big, big[:1]])), ("and", np.concatenate([big, big[:2]])),
        ("and", np.concatenate([big, big[:3]])), ("andnot", u(6, 7, 8)), ("and", np.resize(big, 256)),
        ("or", np.resize(np.arange(12, dtype=np.uint32), 256)), ("xor", np.resize(big, 255)),
    ]
    for op, ids in qs:
        _say(f"[spans kidx={kidx}] op={op} k={len(ids)}")
        exp = oracle.kway(op, [bs[int(i)] for i in ids])
        tids = torch.from_numpy(ids.view(np.int32)).cuda()
        out, card = rg.multi(ctx, op, P, tids, materialize=True, card=True)
        torch.cuda.synchronize()
        assert int(card[0].item()) == len(exp), (op, ids)
        # the arena the call asked for: result-container and payload bounds
        # from each bitmap's key count, first and last key and payload bound
        kb, pb = _kway_bounds(op, [bs[int(i)] for i in ids])
        assert (int(out.c.needed_containers), int(out.c.needed_payload_bytes)) == (kb, pb), (op, ids)
        h = out.as_pool().to_host()
        got, meta = rgtest.decode_bitmap(h, 0)
        assert np.array_equal(got, exp), (op, ids)
        assert meta == rgtest.oracle_meta(oracle, exp), (op, ids)
    # the same queries through the server, batched (several split queries per step)
    sq = [(op, ids, i % 3 != 2) for i, (op, ids) in enumerate(qs)]
    exp = _expect(bs, sq)
    srv = rg.Server(ctx, P, arena_bytes=256 << 20, max_batch=8, max_inflight=2)
    _, cards, dig = srv.replay(sq, np.zeros(len(sq), np.uint64), digest=True)
    st = srv.stop()
    _say(f"[spans serve] {st}")
    for i, (c, d) in enumerate(exp):
        assert cards[i] == c and dig[i] == d, i


@pytest.mark.parametrize("kidx", [False, True], ids=["search", "key-index"])
def test_server_wave_fold_large_steps(rg, ctx, kidx):
    """Steps of more than 8192 slots fold unions and symmetric differences of up
    to 64 bitmaps one wave per result key (k_kw_wave): 64 such queries (k from
    3 to 64, materialised and count-only) in steps of up to 64, against the
    oracle, and the same queries one at a time (workgroup evaluation)."""
    bs = overlapping_sets(n=40, seed=17)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    if kidx:
        P.key_index(ctx)
    rng = np.random.default_rng(41)
    qs = []
    for i in range(64):
        k = int(rng.integers(3, 65))
        ids = rng.choice(len(bs), size=k, replace=k > len(bs)).astype(np.uint32)
        qs.append((("or", "xor")[i % 2], ids, i % 3 != 2))
    exp = _expect(bs, qs)
    big = rg.Server(ctx, P, arena_bytes=512 << 20, max_batch=64, max_inflight=1)
    _, cards, dig = big.replay(qs, np.zeros(len(qs), np.uint64), digest=True)
    st = big.stop()
    _say(f"[wave fold kidx={kidx}] {st}")
    assert st["mean_batch"] > 8  # most queries ran in large steps
    for i, (c, d) in enumerate(exp):
        assert cards[i] == c and dig[i] == d, ("batched", i)
    one = rg.Server(ctx, P, arena_bytes=512 << 20, max_batch=1, max_inflight=1)
    _, cards1, dig1 = one.replay(qs, np.zeros(len(qs), np.uint64), digest=True)
    one.stop()
    assert np.array_equal(cards1, cards) and np.array_equal(dig1, dig)
