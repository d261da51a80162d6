"""In-place operations on mutable bitmaps (rg_mpool_*): sequences of A op= B
against the oracle's fold of the same operations, the maintained
cardinalities, the slot accounting of the device allocator, the capacity
check that leaves a bitmap untouched, a wide union built in place, and
batches of operations on distinct bitmaps (rg_mpool_op_batch) against the
same fold."""
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


def _sources():
    sets = rgtest.edge_sets() + [synth.mixed_small(n_bitmaps=24, seed=81)[i] for i in range(24)]
    return sets, synth.BitmapSet.from_list(sets)


def _check(rg, ctx, M, expected, label):
    out = M.export()
    h = out.as_pool().to_host()
    assert rg.rg_pool_validate(ctx, out.as_pool()) == 0, label
    cards = M.cards().cpu().numpy().view(np.uint64)
    n_cont = 0
    for b, exp in enumerate(expected):
        got, meta = rgtest.decode_bitmap(h, b)
        assert np.array_equal(got, exp), (label, b)
        assert meta == rgtest.oracle_meta(oracle, exp), (label, b)
        assert int(cards[b]) == len(exp), (label, b)
        assert int(h["bm_card"][b]) == len(exp), (label, b)
        n_cont += len(meta)
    st, free = M.status()
    assert st == rg.RG_OK and free == M.n_slots - n_cont, (label, free, n_cont)


def test_inplace_sequences_match_oracle(rg, ctx):
    sets, bs = _sources()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    rng = np.random.default_rng(82)
    nb = 4
    M = rg.MutablePool(ctx, nb, 20000)
    expected = []
    for b in range(nb):
        s = int(rng.integers(len(sets)))
        M.assign(b, P, s)
        expected.append(sets[s])
    _check(rg, ctx, M, expected, "assign")
    for step in range(40):
        b = int(rng.integers(nb))
        op = OPS[int(rng.integers(4))]
        s = int(rng.integers(len(sets)))
        M.op(op, b, P, s)
        expected[b] = oracle.op(op, expected[b], sets[s])
        if step % 4 == 3:
            _say(f"[mutable] step {step}: {[len(e) for e in expected]}")
            _check(rg, ctx, M, expected, f"step {step}")
    # every operation with itself: A & A = A, A | A = A, A ^ A = {}, A \\ A = {}
    for b in range(nb):
        out = M.export(b, 1)
        R = out.as_pool()
        for op in OPS:
            M.op(op, b, R, 0)
            expected[b] = oracle.op(op, expected[b], expected[b])
        _check(rg, ctx, M, expected, f"self {b}")
    for b in range(nb):
        M.clear(b)
        expected[b] = np.zeros(0, np.uint32)
    _check(rg, ctx, M, expected, "cleared")
    M.close()


def test_inplace_capacity_skip(rg, ctx):
    """With too few free slots, a union that must insert keys is skipped as a
    whole (the bitmap keeps its value) and reported once."""
    a = np.arange(0, 5 * 65536, 7, dtype=np.uint32)                       # keys 0..4
    b = np.arange(3 * 65536, 30 * 65536, 11, dtype=np.uint32)             # keys 3..29
    bs = synth.BitmapSet.from_list([a, b])
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    M = rg.MutablePool(ctx, 1, 12)
    M.assign(0, P, 0)
    M.op("or", 0, P, 1)  # needs 25 new slots, 7 are free
    st, free = M.status()
    assert st == rg.RG_ECAPACITY and free == 7
    st, free = M.status()
    assert st == rg.RG_OK  # reported once
    _check(rg, ctx, M, [a], "after skip")
    M.op("and", 0, P, 1)  # needs no slot: keys 3, 4 stay
    _check(rg, ctx, M, [oracle.op("and", a, b)], "and")
    M.close()


def test_wide_union_in_place(rg, ctx):
    """An accumulator built by folding 40 bitmaps into it in place equals the
    oracle's k-way union; its cardinality is maintained throughout."""
    bs = synth.mixed_small(n_bitmaps=40, seed=83)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    M = rg.MutablePool(ctx, 1, 4096)
    for i in range(40):
        M.op("or", 0, P, i)
    _check(rg, ctx, M, [oracle.kway("or", [bs[i] for i in range(40)])], "wide union")
    for i in range(0, 40, 3):
        M.op("andnot", 0, P, i)
    exp = oracle.kway("or", [bs[i] for i in range(40)])
    for i in range(0, 40, 3):
        exp = oracle.op("andnot", exp, bs[i])
    _check(rg, ctx, M, [exp], "wide union minus")
    M.close()


def test_batches_match_oracle(rg, ctx):
    """Batches mixing all four operations (including symmetric differences
    that empty keys and intersections that drop them), batches of more than
    64 operations, and a bitmap's own value as operand, against the oracle."""
    sets, bs = _sources()
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    rng = np.random.default_rng(84)
    nb = 80
    M = rg.MutablePool(ctx, nb, 100000)  # the fold peaks near 80 000 containers with a batch's insertions
    expected = []
    for b in range(nb):
        s = int(rng.integers(len(sets)))
        M.assign(b, P, s)
        expected.append(sets[s])
    for rnd in range(6):
        n = int(rng.integers(1, nb + 1))
        bms = rng.permutation(nb)[:n]
        ops = [OPS[int(rng.integers(4))] for _ in range(n)]
        srcs = [int(rng.integers(len(sets))) for _ in range(n)]
        M.op_batch(ops, bms, P, srcs)
        for op, b, s in zip(ops, bms, srcs):
            expected[b] = oracle.op(op, expected[b], sets[s])
        _say(f"[mutable batch] round {rnd}: {n} operations")
        _check(rg, ctx, M, expected, f"batch {rnd}")
    # every bitmap with a copy of itself: xor empties every key, then or restores
    out = M.export()
    R = out.as_pool()
    M.op_batch(["xor"] * nb, np.arange(nb), R, np.arange(nb))
    _check(rg, ctx, M, [np.zeros(0, np.uint32)] * nb, "xor self")
    M.op_batch(["or"] * nb, np.arange(nb), R, np.arange(nb))
    _check(rg, ctx, M, expected, "or back")
    M.close()


def test_batch_capacity_and_errors(rg, ctx):
    """A batch whose insertions exceed the free slots is skipped as a whole;
    a bitmap named twice in one call is refused."""
    a = np.arange(0, 5 * 65536, 7, dtype=np.uint32)        # keys 0..4
    b = np.arange(3 * 65536, 30 * 65536, 11, dtype=np.uint32)  # keys 3..29
    bs = synth.BitmapSet.from_list([a, b])
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    M = rg.MutablePool(ctx, 2, 20)
    M.assign(0, P, 0)
    M.assign(1, P, 0)  # 10 slots in use, 10 free
    M.op_batch(["or", "and"], [0, 1], P, [1, 1])  # the union needs 25 new slots
    st, free = M.status()
    assert st == rg.RG_ECAPACITY and free == 10
    _check(rg, ctx, M, [a, a], "batch skipped")
    M.op_batch(["and", "andnot"], [0, 1], P, [1, 1])
    _check(rg, ctx, M, [oracle.op("and", a, b), oracle.op("andnot", a, b)], "and, andnot")
    with pytest.raises(rg.RoaringError):
        M.op_batch(["or", "or"], [0, 0], P, [0, 1])
    M.close()
