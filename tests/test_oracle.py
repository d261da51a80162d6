"""Pins for the CPU oracle: brute force on tiny universes, library special cases,
identities, the paper's worked examples and the container-size rules."""
import json
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")

# Boundary-straddling values: chunk edges, word edges, the 2^31 and 2^32 ends.
BOUNDARY = sorted({0, 1, 63, 64, 4095, 4096, 65535, 65536, 65537, 70000, 131071, 3 * 65536 + 5,
                   2**31 - 1, 2**31, 2**32 - 2, 2**32 - 1})


def _from_mask(mask, vals):
    return np.array([v for j, v in enumerate(vals) if mask >> j & 1], dtype=np.uint32)


MASK_OPS = {"and": lambda a, b: a & b, "or": lambda a, b: a | b, "xor": lambda a, b: a ^ b,
            "andnot": lambda a, b: a & ~b}


def _check_mask_pair(ma, mb, vals):
    A, B = _from_mask(ma, vals), _from_mask(mb, vals)
    for name, f in MASK_OPS.items():
        m = f(ma, mb) & ((1 << len(vals)) - 1)
        exp = _from_mask(m, vals)
        got = oracle.op(name, A, B)
        assert np.array_equal(got, exp), (name, ma, mb)
        assert oracle.count(name, A, B) == bin(m).count("1")


def test_bruteforce_exhaustive_8():
    """Every pair of subsets of 8 boundary values, all four operations."""
    vals = [0, 63, 64, 65535, 65536, 131071, 2**31, 2**32 - 1]
    for ma in range(256):
        for mb in range(256):
            _check_mask_pair(ma, mb, vals)


def test_bruteforce_random_16():
    rng = random.Random(1709)
    for _ in range(3000):
        _check_mask_pair(rng.getrandbits(16), rng.getrandbits(16), BOUNDARY)


def _rand_set(rng, n, hi):
    return np.unique(rng.integers(0, hi, size=n, dtype=np.uint64)).astype(np.uint32)


@pytest.mark.parametrize("seed", range(12))
def test_numpy_set_routines(seed):
    """Special case that reduces to library routines (the sorted-vector baseline
    of Section 5.1 uses the standard set algorithms)."""
    rng = np.random.default_rng(seed)
    hi = [50, 1 << 16, 1 << 20, 1 << 32][seed % 4]
    a = _rand_set(rng, int(rng.integers(0, 3000)), hi)
    b = _rand_set(rng, int(rng.integers(0, 3000)), hi)
    assert np.array_equal(oracle.op("and", a, b), np.intersect1d(a, b))
    assert np.array_equal(oracle.op("or", a, b), np.union1d(a, b))
    assert np.array_equal(oracle.op("andnot", a, b), np.setdiff1d(a, b))
    assert np.array_equal(oracle.op("xor", a, b), np.setxor1d(a, b))
    sa, sb = set(a.tolist()), set(b.tolist())
    assert oracle.count("and", a, b) == len(sa & sb)
    assert oracle.count("or", a, b) == len(sa | sb)
    assert oracle.count("xor", a, b) == len(sa ^ sb)
    assert oracle.count("andnot", a, b) == len(sa - sb)


@pytest.mark.parametrize("seed", range(8))
def test_identities(seed):
    """Section 5.9 cardinality identities and set-algebra invariants."""
    rng = np.random.default_rng(100 + seed)
    a = _rand_set(rng, 5000, 1 << 18)
    b = _rand_set(rng, 4000, 1 << 18)
    i, u = oracle.count("and", a, b), oracle.count("or", a, b)
    assert u + i == len(a) + len(b)
    assert oracle.count("andnot", a, b) == len(a) - i
    assert oracle.count("xor", a, b) == len(a) + len(b) - 2 * i
    assert np.array_equal(oracle.op("xor", a, b),
                          oracle.op("andnot", oracle.op("or", a, b), oracle.op("and", a, b)))
    assert np.array_equal(oracle.op("and", oracle.op("and", a, b), a), oracle.op("and", a, b))
    for name in ("and", "or", "xor"):
        assert np.array_equal(oracle.op(name, a, b), oracle.op(name, b, a))
    assert np.array_equal(oracle.op("and", a, a), a)
    assert np.array_equal(oracle.op("or", a, a), a)
    assert len(oracle.op("xor", a, a)) == 0
    assert len(oracle.op("andnot", a, a)) == 0
    e = np.zeros(0, np.uint32)
    assert np.array_equal(oracle.op("or", a, e), a)
    assert len(oracle.op("and", a, e)) == 0
    assert np.array_equal(oracle.op("andnot", a, e), a)
    assert np.array_equal(oracle.op("xor", e, a), a)


def test_jaccard_rounding_and_edges():
    """J = |A n B| / |A u B| (Section 5.9); Python's int/int true division is
    correctly rounded, so it pins the single binary64 division."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        a = _rand_set(rng, int(rng.integers(1, 500)), 700)
        b = _rand_set(rng, int(rng.integers(1, 500)), 700)
        i = len(set(a.tolist()) & set(b.tolist()))
        u = len(set(a.tolist()) | set(b.tolist()))
        assert oracle.jaccard(a, b) == i / u == float(Fraction(i, u))
    e = np.zeros(0, np.uint32)
    assert oracle.jaccard(e, e) == 1.0
    assert oracle.jaccard([1, 2, 3], [2, 3, 4]) == 0.5
    assert oracle.jaccard([1, 2], [3]) == 0.0
    assert oracle.jaccard([5], e) == 0.0
    assert oracle.jaccard([1, 2, 3], [1, 2, 3]) == 1.0


def test_kway_fold():
    rng = np.random.default_rng(3)
    lists = [_rand_set(rng, 2000, 1 << 14) for _ in range(7)]
    sets = [set(l.tolist()) for l in lists]
    assert np.array_equal(oracle.kway("and", lists), np.array(sorted(set.intersection(*sets)), np.uint32))
    assert np.array_equal(oracle.kway("or", lists), np.array(sorted(set.union(*sets)), np.uint32))
    assert np.array_equal(oracle.kway("or", lists[::-1]), oracle.kway("or", lists))
    assert np.array_equal(oracle.kway("and", lists[3:] + lists[:3]), oracle.kway("and", lists))
    assert np.array_equal(oracle.kway("and", lists[:1]), lists[0])
    # symmetric difference of k sets: the values in an odd number of them
    counts = {}
    for st in sets:
        for v in st:
            counts[v] = counts.get(v, 0) + 1
    odd = sorted(v for v, c in counts.items() if c % 2 == 1)
    assert np.array_equal(oracle.kway("xor", lists), np.array(odd, np.uint32))
    # disjoint inputs: the symmetric difference is the whole union (largest possible result)
    disjoint = [np.arange(i * 3000, i * 3000 + 2500, dtype=np.uint32) for i in range(6)]
    assert len(oracle.kway("xor", disjoint)) == 6 * 2500
    # difference of k sets: the first minus all the others
    assert np.array_equal(oracle.kway("andnot", lists),
                          np.array(sorted(sets[0].difference(*sets[1:])), np.uint32))


# ----------------------------------------------------------------- containers

def test_p1_boundary_table():
    g = json.load(open(os.path.join(GOLD, "p1_boundaries.json")))
    names = {"array": oracle.ARRAY, "bitset": oracle.BITSET, "run": oracle.RUN}
    for c, r, t in g["rows"]:
        assert oracle.type_of(c, r) == names[t], (c, r, t)


def test_p1_is_least_memory_allowed_form():
    """Section 1: a type is allowed only under the size rules, and the type is
    picked to minimise memory (array 2c bytes, bitset 8 KiB, run 4r bytes)."""
    for c in list(range(1, 200)) + list(range(4000, 4200)) + [8191, 8192, 30000, 65535, 65536]:
        for r in sorted({1, 2, 3, c // 2 - 1, c // 2, c // 2 + 1, 2046, 2047, 2048, 2049, c}):
            if r < 1 or r > c or r > (c + 1) // 1 or (c == 65536 and r > 1) or r > 32768:
                continue
            allowed = {}
            if c >= 4097:
                allowed[oracle.BITSET] = 8192
            if c <= 4096:
                allowed[oracle.ARRAY] = 2 * c
            if (c > 4096 and r <= 2047) or (c <= 4096 and 2 * r < c):
                allowed[oracle.RUN] = 4 * r
            best = min(allowed, key=lambda t: allowed[t])
            assert sorted(allowed.values()).count(allowed[best]) == 1, "no ties"
            assert oracle.type_of(c, r) == best, (c, r)


def _fig1_set():
    g = json.load(open(os.path.join(GOLD, "fig1_bitmap.json")))
    rec = g["set_recipe"]
    vals = [62 * i for i in range(rec["multiples_of_62_first_n"])]
    for lo, hi in rec["half_open_intervals"]:
        vals += list(range(lo, hi))
    lo, hi = rec["even_values_in"]
    vals += list(range(lo, hi, 2))
    return g, np.array(sorted(vals), dtype=np.uint32)


def test_fig1_container_view():
    g, v = _fig1_set()
    cv = oracle.containers(v)
    names = {"array": oracle.ARRAY, "bitset": oracle.BITSET, "run": oracle.RUN}
    assert len(v) == g["total_card"]
    assert cv["keys"].tolist() == [c["key"] for c in g["containers"]]
    assert cv["types"].tolist() == [names[c["type"]] for c in g["containers"]]
    assert cv["card"].tolist() == [c["card"] for c in g["containers"]]
    # array container: 1000 sorted 16-bit values, 2 bytes each
    assert 2 * int(cv["card"][0]) == g["array_payload_bytes"]
    w = oracle.serialise(v, 0)
    assert int(w[1]) == 1000 and int(w[2]) & 0xFFFF == 0 and (int(w[2 + 999 // 4]) >> 48) & 0xFFFF == 61938
    # run container: <start, length-1> pairs
    w = oracle.serialise(v, 1)
    runs = g["containers"][1]["runs_start_lenminus1"]
    assert int(w[0]) == 1 | (3 << 16) | (300 << 32)
    assert int(w[1]) == len(runs)
    got = []
    for i in range(len(runs)):
        p = (int(w[2 + i // 2]) >> (32 * (i % 2))) & 0xFFFFFFFF
        got.append([p & 0xFFFF, p >> 16])
    assert got == runs
    # bitset container: value x at bit x & 63 of word x >> 6 (Section 3.2)
    w = oracle.serialise(v, 2)
    assert len(w) == 2 + 1024
    assert all(int(x) == 0x5555555555555555 for x in w[2:])


def test_difference_example():
    g = json.load(open(os.path.join(GOLD, "difference_example.json")))
    assert oracle.op("andnot", g["A"], g["B"]).tolist() == g["A_minus_B"]
    # the block masks of the worked example
    A = g["A"]
    masks = []
    for blk in (g["B"][:4], g["B"][4:]):
        masks.append(sum(1 << i for i, x in enumerate(A) if x in blk))
    assert masks == g["block_masks"]
    m = masks[0] | masks[1]
    assert m == g["ored_mask"]
    assert [x for i, x in enumerate(A) if not m >> i & 1] == g["A_minus_B"]


def test_dedup_example():
    g = json.load(open(os.path.join(GOLD, "dedup_example.json")))
    assert sorted(g["A"] + g["B"]) == g["merged_with_duplicates"]
    assert oracle.op("or", g["A"], g["B"]).tolist() == g["union"]
    assert oracle.op("xor", g["A"], g["B"]).tolist() == g["xor"]


def test_containers_runs_and_types():
    # c = 4097 values with r = 2047 runs -> run; add one isolated value -> r = 2048 -> bitset
    vals = []
    x = 0
    per = [2] * 2046 + [4097 - 2 * 2046]
    for k in per:
        vals += list(range(x, x + k))
        x += k + 1
    v = np.array(vals, np.uint32)
    cv = oracle.containers(v)
    assert cv["card"].tolist() == [4097] and cv["runs"].tolist() == [2047]
    assert cv["types"].tolist() == [oracle.RUN]
    v2 = np.array(vals[:-1] + [65535], np.uint32)  # still 4097 values, one more run
    cv2 = oracle.containers(v2)
    assert cv2["card"].tolist() == [4097] and cv2["runs"].tolist() == [2048]
    assert cv2["types"].tolist() == [oracle.BITSET]
    full = np.arange(65536 * 3, 65536 * 4, dtype=np.uint32)
    cv3 = oracle.containers(full)
    assert cv3["keys"].tolist() == [3] and cv3["types"].tolist() == [oracle.RUN] and cv3["runs"].tolist() == [1]
    w = oracle.serialise(full, 0)
    assert int(w[2]) == 0 | (65535 << 16)
    assert oracle.containers(np.zeros(0, np.uint32))["keys"].size == 0


def test_containers_match_python_grouping():
    rng = np.random.default_rng(11)
    v = np.unique(np.concatenate([rng.integers(0, 1 << 20, 20000), np.arange(300000, 340000)])).astype(np.uint32)
    cv = oracle.containers(v)
    keys = sorted(set((v >> 16).tolist()))
    assert cv["keys"].tolist() == keys
    for i, k in enumerate(keys):
        chunk = v[(v >> 16) == k]
        assert int(cv["card"][i]) == len(chunk)
        runs = 1 + int(np.count_nonzero(np.diff(chunk.astype(np.int64)) != 1))
        assert int(cv["runs"][i]) == runs


def test_digest_properties():
    rng = np.random.default_rng(5)
    v = np.unique(rng.integers(0, 1 << 22, 50000)).astype(np.uint32)
    d = oracle.digest(v)
    assert d == oracle.digest(v.copy())
    # additive over containers: the digest of a set is the sum of its chunks' digests
    s = 0
    for k in np.unique(v >> 16):
        s = (s + oracle.digest(v[(v >> 16) == k])) % (1 << 64)
    assert s == d
    # one value more or less changes it
    assert oracle.digest(v[1:]) != d
    w = np.unique(np.append(v, np.uint32(12345678))).astype(np.uint32)
    if len(w) != len(v):
        assert oracle.digest(w) != d
    assert oracle.digest(np.zeros(0, np.uint32)) == 0


def test_pairs_loop():
    rng = np.random.default_rng(9)
    lists = [_rand_set(rng, int(rng.integers(0, 3000)), 1 << 18) for _ in range(10)]
    offs = np.zeros(11, np.uint64)
    offs[1:] = np.cumsum([len(l) for l in lists])
    vals = np.concatenate(lists).astype(np.uint32)
    ia = np.arange(9, dtype=np.uint32)
    ib = ia + 1
    for name in oracle.OPS:
        card, dig, jac = oracle.pairs(name, vals, offs, vals, offs, ia, ib, True, True, True)
        for p in range(9):
            r = oracle.op(name, lists[p], lists[p + 1])
            assert int(card[p]) == len(r)
            assert int(dig[p]) == oracle.digest(r)
            assert jac[p] == oracle.jaccard(lists[p], lists[p + 1])


def test_contains_bruteforce_subsets():
    """Membership against the subset's defining mask: every subset of 8
    boundary values, every boundary value and its neighbours as the query."""
    vals = [0, 63, 64, 65535, 65536, 131071, 2**31, 2**32 - 1]
    queries = sorted({q for v in vals for q in (v - 1, v, v + 1) if 0 <= q < 2**32})
    for m in range(256):
        A = _from_mask(m, vals)
        for q in queries:
            exp = q in vals and (m >> vals.index(q)) & 1 == 1
            assert oracle.contains(A, q) == exp, (m, q)


def test_contains_many_matches_python_sets():
    rng = np.random.default_rng(41)
    sets = [_rand_set(rng, n, hi) for n, hi in ((0, 10), (1, 2**32), (300, 70000), (5000, 2**20), (2000, 2**32))]
    offs = np.cumsum([0] + [len(s) for s in sets]).astype(np.uint64)
    vals = np.concatenate(sets).astype(np.uint32)
    ids = rng.integers(0, len(sets), 20000).astype(np.uint32)
    xs = np.where(rng.random(20000) < 0.5, rng.integers(0, 2**32, 20000, dtype=np.uint64),
                  np.concatenate([vals, vals, vals, vals, vals])[rng.integers(0, len(vals), 20000)]).astype(np.uint32)
    got = oracle.contains_many(vals, offs, ids, xs)
    py = [set(s.tolist()) for s in sets]
    exp = np.array([int(x) in py[i] for i, x in zip(ids.tolist(), xs.tolist())], np.uint8)
    assert np.array_equal(got, exp)
    assert got.sum() > 1000  # the sample holds members and non-members
