"""Device-side canonicalisation (rg_pool_canonicalize) and the well-formed
check (rg_pool_check): pools whose containers are valid but not in the
least-memory form come out in P1 form, equal to the oracle's container view
and fingerprint, value for value."""
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


def _extreme_sets():
    """Chunks whose non-canonical forms are the largest allowed: a full chunk,
    a chunk with one value, and half a chunk (alternate values)."""
    return [np.arange(0, 65536, dtype=np.uint32),
            np.array([4 * 65536 + 65535], np.uint32),
            np.arange(6 * 65536, 7 * 65536, 2, dtype=np.uint32),
            np.concatenate([np.arange(9 * 65536, 9 * 65536 + 5000), np.arange(9 * 65536 + 7000, 10 * 65536)]
                           ).astype(np.uint32)]


def _extreme_arrays():
    """Host arrays of _extreme_sets in forms P1 never picks: the full chunk as
    65536 touching one-value runs, the single value as a bitset, alternate
    values as a 32768-value array, the last set as an array of 63536 values."""
    sets = _extreme_sets()
    chunks, keys, types, card, size, offs = [], [], [], [], [], []
    bm_begin, bm_card, bm_wbytes = [0], [], []
    pos = 0

    def add(key, t, c, sz, pl):
        nonlocal pos
        keys.append(key)
        types.append(t)
        card.append(c)
        size.append(sz)
        offs.append(pos)
        padded = pl + b"\0" * ((-len(pl)) % 16)
        chunks.append(padded)
        pos += len(padded)

    add(0, rgtest.RUN, 65536, 65536, np.stack([np.arange(65536), np.zeros(65536)], 1).astype(np.uint16).tobytes())
    w = np.zeros(1024, np.uint64)
    w[1023] = np.uint64(1) << np.uint64(63)
    add(4, rgtest.BITSET, 1, 1024, w.tobytes())
    add(6, rgtest.ARRAY, 32768, 32768, np.arange(0, 65536, 2).astype(np.uint16).tobytes())
    low = (sets[3] & 0xFFFF).astype(np.uint16)
    add(9, rgtest.ARRAY, len(low), len(low), low.tobytes())
    for i, v in enumerate(sets):
        bm_begin.append(i + 1)
        bm_card.append(len(v))
        bm_wbytes.append(8192 if len(v) > 4096 else (2 * len(v) + 15) & ~15)
    return sets, {"bm_begin": np.array(bm_begin, np.uint64), "keys": np.array(keys, np.uint16),
                  "types": np.array(types, np.uint8), "card": np.array(card, np.uint32),
                  "size": np.array(size, np.uint32), "off": np.array(offs, np.uint64),
                  "payload": np.frombuffer(b"".join(chunks), np.uint8).copy(),
                  "bm_card": np.array(bm_card, np.uint64), "bm_wbytes": np.array(bm_wbytes, np.uint64)}


def _check_canonical(rg, ctx, sets, P, label):
    assert rg.rg_pool_check(ctx, P, 0) == 0, label
    out = rg.canonicalize(ctx, P)
    R = out.as_pool()
    assert rg.rg_pool_validate(ctx, R) == 0, label
    h = R.to_host()
    dig = rg.rg_pool_digest(ctx, R).cpu().numpy().view(np.uint64)
    for b, v in enumerate(sets):
        got, meta = rgtest.decode_bitmap(h, b)
        assert np.array_equal(got, v), (label, b)
        assert meta == rgtest.oracle_meta(oracle, v), (label, b)
        assert int(dig[b]) == oracle.digest(v), (label, b)
    return R


def test_canonicalize_random_forms(rg, ctx):
    rng = np.random.default_rng(17)
    for label, sets in (("edges", rgtest.edge_sets()),
                        ("mixed", [synth.mixed_small(n_bitmaps=20, seed=51)[i] for i in range(20)])):
        for rep in range(2):
            a = rgtest.noncanonical_arrays(sets, rng)
            P = rg.Pool.from_host_arrays(a)
            _say(f"[canonical] {label} rep {rep}: {len(a['keys'])} containers, types {np.bincount(a['types'])}")
            assert rg.rg_pool_check(ctx, P, rg.RG_RULES_P1) > 0, label  # some forms are not P1
            _check_canonical(rg, ctx, sets, P, f"{label}-{rep}")


def test_canonicalize_extreme_forms(rg, ctx):
    sets, a = _extreme_arrays()
    P = rg.Pool.from_host_arrays(a)
    assert rg.rg_pool_check(ctx, P, rg.RG_RULES_P1) == 4
    _check_canonical(rg, ctx, sets, P, "extreme")


def test_canonical_pool_is_unchanged(rg, ctx):
    """A pool already in P1 form comes back with the same containers."""
    bs = synth.mixed_small(n_bitmaps=12, seed=52)
    P = rg.Pool.from_sets(bs.values, bs.offsets)
    R = _check_canonical(rg, ctx, [bs[i] for i in range(len(bs))], P, "canonical")
    h0, h1 = P.to_host(), R.to_host()
    for k in ("bm_begin", "keys", "types", "card", "size", "bm_card"):
        assert np.array_equal(h0[k], h1[k]), k


def test_recount_and_ops_after_canonicalize(rg, ctx):
    """rg_pool_recount on a non-canonical pool gives the builder's counts; the
    canonical pool's pairwise counts and Jaccard equal the oracle's."""
    import torch

    rng = np.random.default_rng(18)
    sets = [synth.mixed_small(n_bitmaps=10, seed=53)[i] for i in range(10)] + rgtest.edge_sets()
    a = rgtest.noncanonical_arrays(sets, rng)
    P = rg.Pool.from_host_arrays(a)
    card0, bmc0, bmw0 = P.card.clone(), P.bm_card.clone(), P.bm_wbytes.clone()
    P.card.zero_()
    P.bm_card.zero_()
    P.bm_wbytes.zero_()
    rg.rg_pool_recount(ctx, P)
    torch.cuda.synchronize()
    assert torch.equal(P.card, card0) and torch.equal(P.bm_card, bmc0) and torch.equal(P.bm_wbytes, bmw0)
    R = rg.canonicalize(ctx, P).as_pool()
    n = len(sets)
    ia = np.arange(n, dtype=np.uint32)
    ib = ((np.arange(n) * 7 + 2) % n).astype(np.uint32)
    tia = torch.from_numpy(ia.view(np.int32)).cuda()
    tib = torch.from_numpy(ib.view(np.int32)).cuda()
    for op in ("and", "or", "xor", "andnot"):
        _, c, j = rg.batch(ctx, op, R, R, tia, tib, materialize=False, card=True, jaccard=True)
        ctx.sync()
        c = c.cpu().numpy()
        j = j.cpu().numpy()
        for p in range(n):
            A, B = sets[int(ia[p])], sets[int(ib[p])]
            assert int(c[p]) == oracle.count(op, A, B) and j[p] == oracle.jaccard(A, B), (op, p)


def test_check_finds_malformed_containers(rg, ctx):
    """Overlapping runs, an unsorted array and a wrong cardinality are not
    well-formed; each is one offending container."""
    rng = np.random.default_rng(19)
    sets = [np.arange(100, 200, dtype=np.uint32), np.array([70000, 70005, 70010], np.uint32),
            np.arange(3 * 65536, 3 * 65536 + 50, dtype=np.uint32)]
    a = rgtest.noncanonical_arrays(sets, rng, p_array=0.0, p_bitset=0.0)  # all runs
    P = rg.Pool.from_host_arrays(a)
    assert rg.rg_pool_check(ctx, P, 0) == 0
    bad = {k: v.copy() for k, v in a.items()}
    # container 0: two runs that overlap ([100, 149] and [140, 199])
    bad["size"][0] = 2
    pl = np.array([100, 49, 140, 59], np.uint16).tobytes()
    o = int(bad["off"][0])
    assert int(a["off"][1]) - o >= 16
    bad["payload"][o:o + 8] = np.frombuffer(pl, np.uint8)
    # container 1 as an array out of order
    o1 = int(bad["off"][1])
    bad["types"][1] = rgtest.ARRAY
    bad["size"][1] = 3
    bad["payload"][o1:o1 + 6] = np.frombuffer(np.array([5, 0, 10], np.uint16).tobytes(), np.uint8)
    # container 2 with a cardinality one too high (its bitmap's totals follow)
    bad["card"][2] += 1
    bad["bm_card"][2] += 1
    Q = rg.Pool.from_host_arrays(bad)
    assert rg.rg_pool_check(ctx, Q, 0) == 3
