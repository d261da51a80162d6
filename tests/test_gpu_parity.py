"""GPU parity: every operation, through the C ABI, against the CPU oracle,
element by element (values, container keys/types/cards/sizes, counts,
Jaccard bit-for-bit, fingerprints)."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import rgtest

pytestmark = pytest.mark.gpu

OPS = ("and", "or", "xor", "andnot")
# every operation is materialised (OR/XOR/ANDNOT through the k-way path)
MAT_OPS = ("and", "or", "xor", "andnot")


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


def check_batch(rg, ctx, bs, ia, ib, ops=OPS, bs_b=None, label="", key_index=(False, False)):
    """Run each op on pairs (ia[p] of bs, ib[p] of bs_b) and compare everything
    with the oracle. key_index: whether the A and the B pool carry key-presence
    indexes."""
    import torch

    bs_b = bs if bs_b is None else bs_b
    A = rg.Pool.from_sets(bs.values, bs.offsets)
    B = A if bs_b is bs else rg.Pool.from_sets(bs_b.values, bs_b.offsets)
    if key_index[0]:
        A.key_index(ctx)
    if key_index[1] and B is not A:
        B.key_index(ctx)
    assert rg.rg_pool_validate(ctx, A) == 0
    assert rg.rg_pool_validate(ctx, B) == 0
    tia, tib = _t(ia), _t(ib)
    n = len(ia)
    for op in ops:
        mat = op in MAT_OPS
        _say(f"[{label}] op={op} pairs={n} materialise={mat}")
        _, cards2, jacc2 = rg.batch(ctx, op, A, B, tia, tib, materialize=False, card=True, jaccard=True)
        if mat:
            out, cards, jacc = rg.batch(ctx, op, A, B, tia, tib, materialize=True, card=True, jaccard=True)
        torch.cuda.synchronize()
        cards2 = cards2.cpu().numpy().view(np.uint64)
        jacc2 = jacc2.cpu().numpy()
        if mat:
            res = out.as_pool()
            assert rg.rg_pool_validate(ctx, res) == 0, "result violates the container rules"
            dig = rg.rg_pool_digest(ctx, res).cpu().numpy().view(np.uint64)
            h = res.to_host()
            cards = cards.cpu().numpy().view(np.uint64)
            jacc = jacc.cpu().numpy()
        for p in range(n):
            a, b = bs[int(ia[p])], bs_b[int(ib[p])]
            exp = oracle.op(op, a, b)
            j = oracle.jaccard(a, b)
            assert int(cards2[p]) == len(exp), (label, op, p)
            assert jacc2[p] == j, (label, op, p, jacc2[p], j)
            if not mat:
                continue
            got, meta = rgtest.decode_bitmap(h, p)
            assert np.array_equal(got, exp), (label, op, p)
            assert meta == rgtest.oracle_meta(oracle, exp), (label, op, p)
            assert int(h["bm_card"][p]) == len(exp)
            assert int(cards[p]) == len(exp), (label, op, p)
            assert jacc[p] == j, (label, op, p, jacc[p], j)
            assert int(dig[p]) == oracle.digest(exp), (label, op, p)


def test_edge_sets_all_pairs(rg, ctx):
    sets = rgtest.edge_sets()
    bs = synth.BitmapSet.from_list(sets)
    k = len(sets)
    ia = np.repeat(np.arange(k), k).astype(np.uint32)
    ib = np.tile(np.arange(k), k).astype(np.uint32)
    check_batch(rg, ctx, bs, ia, ib, label="edges")


def test_mixed_small_consecutive(rg, ctx):
    bs = synth.mixed_small()
    ia, ib = synth.consecutive_pairs(len(bs))
    check_batch(rg, ctx, bs, ia, ib, label="mixed")


@pytest.mark.parametrize("variant", ["generic", "merge", "gallop", "probe", "runmerge", "thread"])
def test_forced_variants_same_result(rg, ctx, variant):
    bs = synth.mixed_small(n_bitmaps=30)
    ia, ib = synth.consecutive_pairs(len(bs))
    ctx.set_dispatch(rg.RG_DISPATCH_FIXED, rg.VARIANTS[variant])
    try:
        check_batch(rg, ctx, bs, ia, ib, label=f"forced-{variant}")
        sets = rgtest.edge_sets()
        eb = synth.BitmapSet.from_list(sets)
        k = len(sets)
        check_batch(rg, ctx, eb, np.repeat(np.arange(k), k).astype(np.uint32),
                    np.tile(np.arange(k), k).astype(np.uint32), label=f"forced-edges-{variant}")
    finally:
        ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)


def test_array_stress_sample(rg, ctx):
    bs, ia, ib = synth.array_stress(n_pairs=3000)
    check_batch(rg, ctx, bs, ia, ib, label="array-stress")


def test_two_pools_and_repeats(rg, ctx):
    a = synth.mixed_small(n_bitmaps=8, seed=5)
    b = synth.mixed_small(n_bitmaps=6, seed=6)
    ia = np.array([0, 1, 2, 7, 7, 3, 0], np.uint32)
    ib = np.array([5, 0, 2, 1, 1, 3, 0], np.uint32)
    check_batch(rg, ctx, a, ia, ib, bs_b=b, label="two-pools")


def test_single_pair_entry_points(rg, ctx):
    import torch

    bs = synth.mixed_small(n_bitmaps=4, seed=11)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    dj = torch.zeros(1, dtype=torch.float64, device="cuda")
    for op in OPS:
        for (x, y) in [(0, 1), (2, 3), (1, 1)]:
            exp = oracle.op(op, bs[x], bs[y])
            ctx.check(getattr(rg, f"roaring_{op}_cardinality")(ctx, P, x, P, y, d))
            torch.cuda.synchronize()
            assert int(d.item()) == len(exp)
            probe = rg.OutArena(1, 0, 0)
            probe.c.cap_containers = 0
            probe.c.cap_payload_bytes = 0
            st = getattr(rg, f"roaring_{op}")(ctx, P, x, P, y, probe)
            assert st in (rg.RG_ECAPACITY, rg.RG_OK)
            out = rg.OutArena(1, probe.c.needed_containers, probe.c.needed_payload_bytes)
            ctx.check(getattr(rg, f"roaring_{op}")(ctx, P, x, P, y, out))
            torch.cuda.synchronize()
            got, meta = rgtest.decode_bitmap(out.as_pool().to_host(), 0)
            assert np.array_equal(got, exp) and meta == rgtest.oracle_meta(oracle, exp)
        ctx.check(rg.roaring_jaccard(ctx, P, 0, P, 1, dj))
        torch.cuda.synchronize()
        assert dj.item() == oracle.jaccard(bs[0], bs[1])


def test_errors(rg, ctx):
    import torch

    bs = synth.mixed_small(n_bitmaps=3, seed=12)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    d = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert rg.roaring_and_cardinality(ctx, P, 3, P, 0, d) == rg.RG_EINVAL
    ia = _t(np.array([0, 5], np.uint32))
    ib = _t(np.array([1, 1], np.uint32))
    cards = torch.zeros(2, dtype=torch.int64, device="cuda")
    # count-only batches do not wait for the device: the bad index is reported by rg_sync
    assert rg.roaring_batch(ctx, "and", P, P, ia, ib, rg.RG_FLAG_CARD, None, cards) == rg.RG_OK
    with pytest.raises(rg.RoaringError):
        ctx.sync()
    out = rg.OutArena(1, 1, 16)
    assert rg.roaring_and(ctx, P, 0, P, 1, out) == rg.RG_ECAPACITY
    assert out.c.needed_containers > 1 and out.c.needed_payload_bytes > 16
    assert rg.roaring_batch(ctx, 7, P, P, ia, ib, rg.RG_FLAG_CARD, None, cards) == rg.RG_EINVAL


def test_empty_batch(rg, ctx):
    bs = synth.mixed_small(n_bitmaps=3, seed=13)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    e = _t(np.zeros(0, np.uint32))
    out, cards, jacc = rg.batch(ctx, "and", P, P, e, e, materialize=True, card=True, jaccard=True)
    assert out.c.n_containers == 0


def test_dense_generator_device_matches_host(rg, ctx):
    import torch

    w = torch.empty(3 * 4 * 1024, dtype=torch.int64, device="cuda")
    synth.dense_bitsets_device(w.data_ptr(), 17, 3, 4, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    host = w.cpu().numpy().view(np.uint64).reshape(3, 4, 1024)
    for b in range(3):
        for k in range(4):
            assert np.array_equal(host[b, k], synth.dense_container(17 + b, k))


def test_dense_bitsets_reduced(rg, ctx):
    """Bitset-bandwidth workload at reduced scale: 24 bitmaps x 256 bitsets."""
    import torch

    nb, nk = 24, 256
    w = torch.empty(nb * nk * 1024, dtype=torch.int64, device="cuda")
    synth.dense_bitsets_device(w.data_ptr(), 0, nb, nk, torch.cuda.current_stream().cuda_stream)
    P = rg.Pool.from_dense_words(ctx, w, nb, nk)
    assert rg.rg_pool_validate(ctx, P) == 0
    ia, ib = synth.random_pairs(nb, 12, seed=synth.DENSE_SEED)
    vals = {b: synth.dense_bitmap_values(int(b), nk) for b in set(ia.tolist()) | set(ib.tolist())}
    for op in OPS:
        mat = op in MAT_OPS
        _say(f"[dense-reduced] op={op} materialise={mat}")
        _, cards2, jacc = rg.batch(ctx, op, P, P, _t(ia), _t(ib), materialize=False, card=True, jaccard=True)
        if mat:
            out, cards, _ = rg.batch(ctx, op, P, P, _t(ia), _t(ib), materialize=True, card=True)
        torch.cuda.synchronize()
        cards2 = cards2.cpu().numpy().view(np.uint64)
        jacc = jacc.cpu().numpy()
        if mat:
            res = out.as_pool()
            assert rg.rg_pool_validate(ctx, res) == 0
            dig = rg.rg_pool_digest(ctx, res).cpu().numpy().view(np.uint64)
            h = res.to_host()
            cards = cards.cpu().numpy().view(np.uint64)
        for p in range(len(ia)):
            a, b = vals[int(ia[p])], vals[int(ib[p])]
            n_exp = oracle.count(op, a, b)
            assert int(cards2[p]) == n_exp
            assert jacc[p] == oracle.jaccard(a, b)
            if mat:
                assert int(cards[p]) == n_exp
            if mat and p < 3:
                exp = oracle.op(op, a, b)
                got, meta = rgtest.decode_bitmap(h, p)
                assert np.array_equal(got, exp)
                assert meta == rgtest.oracle_meta(oracle, exp)
                assert int(dig[p]) == oracle.digest(exp)


def test_materialised_two_pools_different_layouts(rg, ctx):
    """Materialised OR/XOR/ANDNOT between two different pools (the A side and
    the B side of each pair come from different pools)."""
    import torch

    a_bs = synth.mixed_small(n_bitmaps=6, seed=14)
    b_bs = synth.BitmapSet.from_list(rgtest.edge_sets())
    A = rg.Pool.from_sets(a_bs.values, a_bs.offsets)
    B = rg.Pool.from_sets(b_bs.values, b_bs.offsets)
    ia = np.repeat(np.arange(len(a_bs)), len(b_bs)).astype(np.uint32)
    ib = np.tile(np.arange(len(b_bs)), len(a_bs)).astype(np.uint32)
    for op in ("or", "xor", "andnot"):
        _say(f"[two-pools-mat] op={op} pairs={len(ia)}")
        out, cards, jacc = rg.batch(ctx, op, A, B, _t(ia), _t(ib), materialize=True, card=True, jaccard=True)
        torch.cuda.synchronize()
        res = out.as_pool()
        assert rg.rg_pool_validate(ctx, res) == 0
        dig = rg.rg_pool_digest(ctx, res).cpu().numpy().view(np.uint64)
        cards = cards.cpu().numpy().view(np.uint64)
        jacc = jacc.cpu().numpy()
        for p in range(len(ia)):
            a, b = a_bs[int(ia[p])], b_bs[int(ib[p])]
            exp = oracle.op(op, a, b)
            assert int(cards[p]) == len(exp) and int(dig[p]) == oracle.digest(exp), (op, p)
            assert jacc[p] == oracle.jaccard(a, b)



def _popcount_table():
    import torch

    t = torch.zeros(256, dtype=torch.int32)
    for v in range(256):
        t[v] = bin(v).count("1")
    return t


def test_dense_bitsets_full_size_sampled(rg, ctx):
    """The bitset-bandwidth workload at full size, in the launch configuration the
    bench times (2e4 bitmaps x 256 bitsets, 1e4 random pairs, count-only batched
    calls). Three checks: (1) 64 pairs spread over the list (first, last, every
    157th) against the oracle for all four counts and the Jaccard index; (2)
    every pair's intersection count against a popcount of the AND of the two
    bitmaps' words computed by torch (byte table lookups; no library code);
    (3) every pair's four counts are consistent with the Section 5.9 identities
    (a self-consistency check of the count conversion only: the library derives
    the other counts from the intersection). A materialised batch of sampled
    pairs is decoded and fingerprinted against the oracle."""
    import concurrent.futures as cf

    import torch

    nb, nk, npairs = 20000, 256, 10000
    w = torch.empty(nb * nk * 1024, dtype=torch.int64, device="cuda")
    for b0 in range(0, nb, 1000):
        synth.dense_bitsets_device(w.data_ptr() + b0 * nk * 8192, b0, min(1000, nb - b0), nk,
                                   torch.cuda.current_stream().cuda_stream)
    P = rg.Pool.from_dense_words(ctx, w, nb, nk)
    ia, ib = synth.random_pairs(nb, npairs, seed=synth.DENSE_SEED)
    tia, tib = _t(ia), _t(ib)
    cards = {}
    for op in OPS:
        _, c, j = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True, jaccard=True)
        torch.cuda.synchronize()
        cards[op] = c.cpu().numpy().view(np.uint64).astype(np.int64)
        jac = j.cpu().numpy()
    # (1) oracle on 64 spread pairs (ctypes calls release the GIL: a thread pool)
    sample = sorted(set([0, npairs - 1] + list(range(157, npairs - 1, 157))))
    assert len(sample) >= 64

    def oracle_pair(p):
        a = synth.dense_bitmap_values(int(ia[p]), nk)
        b = synth.dense_bitmap_values(int(ib[p]), nk)
        return p, {op: oracle.count(op, a, b) for op in OPS}, oracle.jaccard(a, b)

    _say(f"[dense-full] oracle on {len(sample)} pairs")
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        for p, exp, jexp in ex.map(oracle_pair, sample):
            for op in OPS:
                assert int(cards[op][p]) == exp[op], (op, p)
            assert jac[p] == jexp, p
    # (2) every pair's |A n B| by torch: AND of the words, byte popcount table, sum
    _say("[dense-full] torch popcount of every pair")
    tab = _popcount_table().cuda()
    wv = w.view(nb, nk * 1024)
    got = np.zeros(npairs, np.int64)
    for p0 in range(0, npairs, 50):
        p1 = min(npairs, p0 + 50)
        x = wv[tia[p0:p1].long()] & wv[tib[p0:p1].long()]
        got[p0:p1] = tab[x.view(torch.uint8).long()].sum(dim=1).cpu().numpy()
    assert np.array_equal(cards["and"], got)
    # (3) self-consistency of the derived counts with the stored totals
    tot = P.bm_card.cpu().numpy()
    na, nb_ = tot[ia], tot[ib]
    assert np.array_equal(cards["or"] + cards["and"], na + nb_)
    assert np.array_equal(cards["xor"], na + nb_ - 2 * cards["and"])
    assert np.array_equal(cards["andnot"], na - cards["and"])
    mat_sample = [0, 1, npairs // 2, npairs - 1]
    sia, sib = _t(ia[mat_sample]), _t(ib[mat_sample])
    for op in OPS:
        out, mc, _ = rg.batch(ctx, op, P, P, sia, sib, materialize=True, card=True)
        torch.cuda.synchronize()
        res = out.as_pool()
        assert rg.rg_pool_validate(ctx, res) == 0
        dig = rg.rg_pool_digest(ctx, res).cpu().numpy().view(np.uint64)
        for q, p in enumerate(mat_sample[:2]):
            a = synth.dense_bitmap_values(int(ia[p]), nk)
            b = synth.dense_bitmap_values(int(ib[p]), nk)
            exp = oracle.op(op, a, b)
            assert int(dig[q]) == oracle.digest(exp), (op, p)
    del w, P
    torch.cuda.empty_cache()


def test_array_stress_full_size_sampled(rg, ctx):
    """Array-array stress at full size (1e5 pairs): counts of every pair satisfy
    the identities; 200 sampled pairs equal the oracle for all four operations."""
    import torch

    bs, ia, ib = synth.array_stress()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    cards = {}
    for op in OPS:
        _, c, _ = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True)
        torch.cuda.synchronize()
        cards[op] = c.cpu().numpy().view(np.uint64).astype(np.int64)
    tot = P.bm_card.cpu().numpy()
    assert np.array_equal(cards["or"] + cards["and"], tot[ia] + tot[ib])
    rng = np.random.default_rng(9)
    for p in rng.choice(len(ia), 200, replace=False):
        a, b = bs[int(ia[p])], bs[int(ib[p])]
        for op in OPS:
            assert int(cards[op][p]) == oracle.count(op, a, b), (op, p)


def _key_matching_layouts():
    """Bitmaps that stress key matching: eight with every one of the 65536 keys
    (one value per key, so each pair of them matches 65536 containers and the
    staged key window overflows), every third key with two values, a single
    value, an empty bitmap, and scattered values over the whole universe."""
    sets = []
    k = np.arange(65536, dtype=np.uint64)
    for i in range(8):
        sets.append((k * 65536 + (((k * 2654435761) >> (i + 7)) & 3)).astype(np.uint32))
    k3 = np.arange(0, 65536, 3, dtype=np.uint64)
    sets.append(np.sort(np.concatenate([k3 * 65536 + 5, k3 * 65536 + (k3 & 0xFFFF)])).astype(np.uint32))
    sets.append(np.array([7 * 65536 + 7], np.uint32))
    sets.append(np.zeros(0, np.uint32))
    rng = np.random.default_rng(5)
    sets.append(np.unique(rng.integers(0, 1 << 32, 5000, dtype=np.uint64)).astype(np.uint32))
    return synth.BitmapSet.from_list([np.unique(s) for s in sets])


def test_key_matching_block_layouts(rg, ctx):
    """Pairs of 65536-key bitmaps (more than 2^24 candidate slots: two waves of
    the materialising path, one launch of the fused count kernel;
    blocks inside one pair with no staged window) interleaved with empty,
    one-key and small pairs (blocks spanning many pairs, pairs without
    candidates); every count and Jaccard index, eager and as a plan, equals
    the oracle, and materialised intersections of a sample decode to it."""
    import torch

    bs = _key_matching_layouts()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    rng = np.random.default_rng(17)
    big = [(int(a), int(b)) for a, b in rng.integers(0, 8, (260, 2))]
    small = [(int(a), int(b)) for a, b in rng.integers(0, len(bs), (120, 2))]
    pairs = big + small
    order = rng.permutation(len(pairs))
    ia = np.array([pairs[i][0] for i in order], np.uint32)
    ib = np.array([pairs[i][1] for i in order], np.uint32)
    tia, tib = _t(ia), _t(ib)
    for op in OPS:
        _say(f"[key-matching] op={op} pairs={len(ia)}")
        exp, _, jexp = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_jaccard=True)
        _, c, j = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True, jaccard=True)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().view(np.uint64), exp), op
        assert np.array_equal(j.cpu().numpy(), jexp), op
        pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True)
        assert pl.info()["slots"] > 1 << 24
        pl.execute()
        torch.cuda.synchronize()
        assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), exp), op
        assert np.array_equal(pl.jacc.cpu().numpy(), jexp), op
        pl.close()
    sample = np.array([0, 1, len(ia) - 1] + [p for p in range(len(ia)) if ia[p] >= 8][:3])
    out, mc, _ = rg.batch(ctx, "and", P, P, _t(ia[sample]), _t(ib[sample]), materialize=True, card=True)
    torch.cuda.synchronize()
    res = out.as_pool()
    assert rg.rg_pool_validate(ctx, res) == 0
    h = res.to_host()
    for q, p in enumerate(sample):
        e = oracle.op("and", bs[int(ia[p])], bs[int(ib[p])])
        got, meta = rgtest.decode_bitmap(h, q)
        assert np.array_equal(got, e), p
        assert meta == rgtest.oracle_meta(oracle, e), p


@pytest.mark.parametrize("which", ["edges", "array-stress"])
def test_packed_metadata_same_results(rg, ctx, which):
    """A pool carrying packed metadata records (rg_pool_pack_meta) gives the
    oracle's counts, Jaccard indices and materialised intersections, eagerly and
    through a plan that reuses the records."""
    import torch

    if which == "edges":
        bs = synth.BitmapSet.from_list(rgtest.edge_sets())
        k = len(bs)
        ia, ib = np.repeat(np.arange(k), k).astype(np.uint32), np.tile(np.arange(k), k).astype(np.uint32)
    else:
        bs, ia, ib = synth.array_stress(n_pairs=3000)
    P = rg.Pool.from_sets(bs.values, bs.offsets).pack_meta(ctx)
    torch.cuda.synchronize()
    tia, tib = _t(ia), _t(ib)
    for op in OPS:
        _say(f"[packed {which}] op={op}")
        exp, _, jexp = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_jaccard=True)
        _, c, j = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True, jaccard=True)
        pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True)
        pl.execute()
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().view(np.uint64), exp), op
        assert np.array_equal(j.cpu().numpy(), jexp), op
        assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), exp), op
        pl.close()
    n = min(len(ia), 40)
    out, mc, _ = rg.batch(ctx, "and", P, P, _t(ia[:n]), _t(ib[:n]), materialize=True, card=True)
    torch.cuda.synchronize()
    h = out.as_pool().to_host()
    for p in range(n):
        e = oracle.op("and", bs[int(ia[p])], bs[int(ib[p])])
        got, meta = rgtest.decode_bitmap(h, p)
        assert np.array_equal(got, e) and meta == rgtest.oracle_meta(oracle, e), p


def test_array_stress_full_size_materialised(rg, ctx):
    """Array-array stress at full size (1e5 pairs) materialised for all four
    operations: every pair's cardinality and container-form fingerprint equal
    the oracle's (union and symmetric difference results above 4096 values
    become bitsets or runs by P1); a sample of results is decoded in full."""
    import torch

    bs, ia, ib = synth.array_stress()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    tia, tib = _t(ia), _t(ib)
    for op in OPS:
        _say(f"[array-stress full mat] op={op}")
        card, dig, _ = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_digest=True)
        out, c, _ = rg.batch(ctx, op, P, P, tia, tib, materialize=True, card=True)
        torch.cuda.synchronize()
        res = out.as_pool()
        assert rg.rg_pool_validate(ctx, res) == 0
        assert np.array_equal(c.cpu().numpy().view(np.uint64), card), op
        assert np.array_equal(rg.rg_pool_digest(ctx, res).cpu().numpy().view(np.uint64), dig), op
        h = res.to_host()
        for p in np.random.default_rng(3).choice(len(ia), 20, replace=False):
            e = oracle.op(op, bs[int(ia[p])], bs[int(ib[p])])
            got, meta = rgtest.decode_bitmap(h, int(p))
            assert np.array_equal(got, e) and meta == rgtest.oracle_meta(oracle, e), (op, p)
        del out, res, h


def test_key_index_layout_and_matching(rg, ctx):
    """The key-presence index (rg_pool_key_index) holds every key's bit and each
    word's rank, as a numpy construction of the same layout; pools carrying it
    (keys found by bit test and popcount, in LDS for single-pair blocks and in
    global memory otherwise) give the oracle's counts and Jaccard indices,
    eagerly and through a plan, with and without packed records."""
    import torch

    sets = rgtest.edge_sets() + [synth.mixed_small(n_bitmaps=16, seed=91)[i] for i in range(16)]
    bs = synth.BitmapSet.from_list(sets)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    P.key_index(ctx)
    torch.cuda.synchronize()
    kx = P.kidx.cpu().numpy().reshape(len(bs), rg.RG_KEY_INDEX_BYTES)
    h = P.to_host()
    for b in range(len(bs)):
        keys = h["keys"][int(h["bm_begin"][b]):int(h["bm_begin"][b + 1])].astype(np.int64)
        words = np.zeros(1024, np.uint64)
        np.bitwise_or.at(words, keys >> 6, np.left_shift(np.uint64(1), (keys & 63).astype(np.uint64)))
        pc = np.array([bin(int(w)).count("1") for w in words], np.int64)
        ranks = (np.cumsum(pc) - pc).astype(np.uint16)
        assert np.array_equal(kx[b, :8192].view(np.uint64), words), b
        assert np.array_equal(kx[b, 8192:].view(np.uint16), ranks), b
    k = len(sets)
    ia = np.repeat(np.arange(k), k).astype(np.uint32)
    ib = np.tile(np.arange(k), k).astype(np.uint32)
    tia, tib = _t(ia), _t(ib)
    for packed in (False, True):
        if packed:
            P.pack_meta(ctx)
        for op in OPS:
            _say(f"[key index] packed={packed} op={op} pairs={len(ia)}")
            exp, _, jexp = oracle.pairs(op, bs.values, bs.offsets, bs.values, bs.offsets, ia, ib, want_jaccard=True)
            _, c, j = rg.batch(ctx, op, P, P, tia, tib, materialize=False, card=True, jaccard=True)
            torch.cuda.synchronize()
            assert np.array_equal(c.cpu().numpy().view(np.uint64), exp), (packed, op)
            assert np.array_equal(j.cpu().numpy(), jexp), (packed, op)
            pl = rg.Plan(ctx, op, P, P, tia, tib, card=True, jaccard=True)
            pl.execute()
            torch.cuda.synchronize()
            assert np.array_equal(pl.cards.cpu().numpy().view(np.uint64), exp), (packed, op)
            assert np.array_equal(pl.jacc.cpu().numpy(), jexp), (packed, op)
            pl.close()
    # the 65536-key layouts with an index (single-pair blocks staged in LDS)
    lb = _key_matching_layouts()
    L = rg.Pool.from_sets(lb.values, lb.offsets)
    L.key_index(ctx)
    rng = np.random.default_rng(92)
    xa = rng.integers(0, len(lb), 300).astype(np.uint32)
    xb = rng.integers(0, len(lb), 300).astype(np.uint32)
    for op in OPS:
        exp, _, jexp = oracle.pairs(op, lb.values, lb.offsets, lb.values, lb.offsets, xa, xb, want_jaccard=True)
        _, c, j = rg.batch(ctx, op, L, L, _t(xa), _t(xb), materialize=False, card=True, jaccard=True)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy().view(np.uint64), exp), op
        assert np.array_equal(j.cpu().numpy(), jexp), op


@pytest.mark.parametrize("which", ["edges", "mixed"])
def test_materialised_with_key_index(rg, ctx, which):
    """Pools that carry key-presence indexes: the k-way kernels of union,
    symmetric difference and difference take their key sets from the presence
    words and find containers by bit test and rank; one pool, and an indexed
    pool against one without."""
    bs = synth.BitmapSet.from_list(rgtest.edge_sets()) if which == "edges" else synth.mixed_small(n_bitmaps=24, seed=95)
    k = len(bs)
    rng = np.random.default_rng(96)
    ia = rng.integers(0, k, 120).astype(np.uint32)
    ib = rng.integers(0, k, 120).astype(np.uint32)
    check_batch(rg, ctx, bs, ia, ib, label=f"kidx-{which}", key_index=(True, True))
    other = synth.mixed_small(n_bitmaps=12, seed=97)
    ib2 = rng.integers(0, len(other), 120).astype(np.uint32)
    check_batch(rg, ctx, bs, ia, ib2, bs_b=other, label=f"kidx-{which}-A", key_index=(True, False))
    check_batch(rg, ctx, other, ib2, ia, bs_b=bs, label=f"kidx-{which}-B", key_index=(False, True))


def test_materialised_many_empty_pairs(rg, ctx):
    """Far more pairs than candidate slots (2e5 pairs of empty bitmaps around
    a few non-empty ones): the device scan of the pair offsets runs over every
    pair, so its workspace is sized by the pair count as well as the slots."""
    import torch

    rng = np.random.default_rng(98)
    sets = [np.zeros(0, np.uint32), np.unique(rng.integers(0, 1 << 20, 300)).astype(np.uint32),
            np.unique(rng.integers(0, 1 << 20, 50)).astype(np.uint32)]
    bs = synth.BitmapSet.from_list(sets)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    n = 200_000
    ia = np.zeros(n, np.uint32)
    ib = np.zeros(n, np.uint32)
    ia[[0, 77_777, n - 1]] = [1, 2, 1]
    ib[[0, 77_777, n - 1]] = [2, 1, 1]
    for op in OPS:
        _say(f"[many empty] op={op} pairs={n}")
        out, cards, _ = rg.batch(ctx, op, P, P, _t(ia), _t(ib), materialize=True, card=True)
        torch.cuda.synchronize()
        c = cards.cpu().numpy().view(np.uint64)
        h = out.as_pool().to_host()
        for p in (0, 1, 77_777, n - 2, n - 1):
            exp = oracle.op(op, sets[int(ia[p])], sets[int(ib[p])])
            assert int(c[p]) == len(exp), (op, p)
            got, meta = rgtest.decode_bitmap(h, p)
            assert np.array_equal(got, exp) and meta == rgtest.oracle_meta(oracle, exp), (op, p)
        assert int(c.astype(np.int64).sum()) == sum(len(oracle.op(op, sets[int(ia[p])], sets[int(ib[p])]))
                                                    for p in (0, 77_777, n - 1))
