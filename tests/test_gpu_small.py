"""The one-wave kernels of materialised results (pairs with an array side;
pairs of bitsets): containers built to hit each of their cases - merges at and
just past the value limit, merges whose second operand cannot start aligned,
results that come out as runs across many 64-value rounds, absent sides,
array-bitset and array-run filters in both operand orders, full 4096-value
arrays, bitset pairs whose results are bitsets, arrays, runs or empty, lone
bitsets and lone run containers - against the oracle, through the eager call
(binned intersection and k-way path) and a materialising plan, and the same
pairs with the one-wave kernels switched off."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import rgtest
from tests.test_gpu_parity import check_batch

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


def _chunk(key, lows):
    return (np.uint32(key) << np.uint32(16)) | np.asarray(lows, np.uint32)


def case_sets():
    """Two bitmaps whose chunks pair up as listed; (A, B) per key."""
    rng = np.random.default_rng(91)
    ev = np.arange(0, 65536, 2)
    parts = {
        # small random arrays: merges of about 200 values, few runs
        0: (np.unique(rng.integers(0, 4000, 100)), np.unique(rng.integers(0, 4000, 100))),
        # 2000 evens + 2096 odds = 4096 values: union is one run 0..4191
        1: (ev[:2048 - 48], ev[:2096] + 1),
        # 2049 + 2048 = 4097 values: past the merge limit (intersection and difference still filter)
        2: (ev[:2049], ev[:2048] + 1),
        # array against a bitset
        3: (np.unique(rng.integers(0, 65536, 3000)), np.unique(rng.integers(0, 65536, 9000))),
        # runs (100 runs of 20) against an array inside them and around them
        4: (np.concatenate([np.arange(s, s + 20) for s in range(0, 4000, 40)]),
            np.unique(rng.integers(0, 4200, 500))),
        # value pairs {4i, 4i+1} and {4i+1, 4i+2}: union in runs of three
        5: (np.sort(np.concatenate([np.arange(0, 2000, 4), np.arange(1, 2000, 4)])),
            np.sort(np.concatenate([np.arange(1, 2000, 4), np.arange(2, 2000, 4)]))),
        # only in A / only in B
        6: (np.unique(rng.integers(0, 65536, 37)), None),
        7: (None, np.unique(rng.integers(0, 65536, 70))),
        # the chunk's last value on both sides
        8: (np.array([65535]), np.array([65535])),
        # two full-size arrays, every 16th value, offset by 0 and 8 / 16
        9: (np.arange(0, 65536, 16), np.arange(0, 65536, 16)[::2]),
        # a bitset against an array
        10: (np.unique(rng.integers(0, 65536, 6000)), np.unique(rng.integers(0, 65536, 1500))),
        # an array against 1500 runs of one value and a gap (staged runs)
        11: (np.unique(rng.integers(0, 6000, 800)), np.concatenate([np.arange(s, s + 3) for s in range(0, 6000, 4)])),
        # an array against 2047 runs (the most a run container of more than 4096 values has)
        12: (np.unique(rng.integers(0, 65536, 4096)),
             np.concatenate([np.arange(s, s + 3) for s in range(0, 2047 * 32, 32)])),
        # pairs {4i, 4i+1}: the intersection with its shifted copy gives singletons
        13: (np.sort(np.concatenate([np.arange(0, 8000, 4), np.arange(1, 8000, 4)])),
             np.sort(np.concatenate([np.arange(1, 8000, 4), np.arange(2, 8000, 4)]))),
        # two random bitsets: bitset results, and an intersection that is an array
        14: (np.unique(rng.integers(0, 65536, 11000)), np.unique(rng.integers(0, 65536, 11000))),
        # a bitset and itself less ten values: difference and symmetric difference of ten values
        15: (bs15 := np.unique(rng.integers(0, 65536, 7000)), np.delete(bs15, np.arange(0, 5000, 500))),
        # a bitset only in A, a bitset only in B
        16: (np.unique(rng.integers(0, 65536, 9000)), None),
        17: (None, np.unique(rng.integers(0, 65536, 9000))),
        # evens and odds below 20000 (bitsets): union and symmetric difference are one run
        18: (np.arange(0, 20000, 2), np.arange(1, 20000, 2)),
        # evens below 40000 and the odds less every 13th: 1539 runs over 38462 values
        19: (np.arange(0, 40000, 2), np.delete(np.arange(1, 40000, 2), np.arange(0, 20000, 13))),
        # a run container only in A, one only in B (copied in P1 form)
        20: (np.concatenate([np.arange(s, s + 20) for s in range(0, 4000, 40)]), None),
        21: (None, np.arange(100, 60000)),
        # 2001 + 2095 = 4096 values: the second array cannot start 16-byte aligned
        # in the wave's 4096 staging entries (staged value by value)
        22: (ev[:2001], ev[:2095] + 1),
    }
    a, b = [], []
    for key, (pa, pb) in parts.items():
        if pa is not None:
            a.append(_chunk(key, pa))
        if pb is not None:
            b.append(_chunk(key, pb))
    return np.concatenate(a), np.concatenate(b)


def _check_types(rg):
    """The chunks have the container types the cases are named for."""
    a, b = case_sets()
    ca, cb = oracle.containers(a), oracle.containers(b)
    ta = dict(zip(ca["keys"].tolist(), ca["types"].tolist()))
    tb = dict(zip(cb["keys"].tolist(), cb["types"].tolist()))
    A, B, R = rgtest.ARRAY, rgtest.BITSET, rgtest.RUN
    assert ta[3] == A and tb[3] == B
    assert ta[4] == R and tb[4] == A
    assert ta[5] == A and tb[5] == A
    assert ta[10] == B and tb[10] == A
    assert ta[11] == A and tb[11] == R
    assert ta[12] == A and tb[12] == R and int(cb["runs"][cb["keys"].tolist().index(12)]) == 2047
    assert ta[9] == A and int(ca["card"][ca["keys"].tolist().index(9)]) == 4096
    for key in (14, 15, 18, 19):
        assert ta[key] == B and tb[key] == B, key
    assert ta[16] == B and tb[17] == B
    assert ta[20] == R and tb[21] == R


def test_cases_against_oracle(rg, ctx):
    _check_types(rg)
    a, b = case_sets()
    bs = synth.BitmapSet.from_list([a, b, np.zeros(0, np.uint32), a[::5].copy()])
    ia = np.array([0, 1, 0, 1, 2, 0, 3, 0], np.uint32)
    ib = np.array([1, 0, 0, 1, 0, 2, 0, 3], np.uint32)
    check_batch(rg, ctx, bs, ia, ib, ops=OPS, label="small-cases")


def test_cases_without_the_wave_kernels(rg, ctx):
    """Forcing the generic variant turns the one-wave kernels off: the same
    results."""
    a, b = case_sets()
    bs = synth.BitmapSet.from_list([a, b])
    ctx.set_dispatch(rg.RG_DISPATCH_FIXED, rg.VARIANTS["generic"])
    try:
        check_batch(rg, ctx, bs, np.array([0, 1], np.uint32), np.array([1, 0], np.uint32), label="small-off")
    finally:
        ctx.set_dispatch(rg.RG_DISPATCH_HEURISTIC)


def test_materialising_plan_on_cases(rg, ctx):
    import torch

    a, b = case_sets()
    sets = [a, b, a[::3].copy(), b[::7].copy()]
    bs = synth.BitmapSet.from_list(sets)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    ia = np.array([0, 1, 2, 3, 0, 2], np.uint32)
    ib = np.array([1, 0, 3, 2, 3, 1], np.uint32)
    tia = torch.from_numpy(ia.view(np.int32)).cuda()
    tib = torch.from_numpy(ib.view(np.int32)).cuda()
    for op in OPS:
        _say(f"[small-plan] op={op}")
        pl = rg.Plan(ctx, op, P, P, tia, tib, materialize=True, card=True, jaccard=True)
        for rep in range(2):
            pl.execute()
            ctx.sync()
            res = pl.result()
            assert rg.rg_pool_validate(ctx, res) == 0
            h = res.to_host()
            for p in range(len(ia)):
                exp = oracle.op(op, sets[int(ia[p])], sets[int(ib[p])])
                got, meta = rgtest.decode_bitmap(h, p)
                assert np.array_equal(got, exp), (op, rep, p)
                assert meta == rgtest.oracle_meta(oracle, exp), (op, rep, p)
        pl.close()


def test_random_small_arrays(rg, ctx):
    """Array stress pairs and mixed pools: sizes over the whole range."""
    bs, ia, ib = synth.array_stress(n_pairs=1500, seed=92)
    check_batch(rg, ctx, bs, ia, ib, label="small-stress")
    ms = synth.mixed_small(n_bitmaps=40, seed=93)
    rng = np.random.default_rng(94)
    check_batch(rg, ctx, ms, rng.integers(0, 40, 200).astype(np.uint32), rng.integers(0, 40, 200).astype(np.uint32),
                label="small-mixed")
