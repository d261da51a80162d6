"""Test helpers: an independent reader of the pool format (numpy), used to
turn GPU results back into sorted value lists for comparison with the oracle,
and shared case builders."""
import numpy as np

ARRAY, BITSET, RUN = 1, 2, 3


def decode_container(h, i):
    """Values (low 16 bits, as uint32) of container i of host pool arrays h."""
    t = int(h["types"][i])
    sz = int(h["size"][i])
    off = int(h["off"][i])
    pl = h["payload"]
    if t == ARRAY:
        return pl[off:off + 2 * sz].view(np.uint16).astype(np.uint32)
    if t == BITSET:
        words = pl[off:off + 8192].view(np.uint64)
        bits = np.unpackbits(words.view(np.uint8), bitorder="little")
        return np.nonzero(bits)[0].astype(np.uint32)
    if t == RUN:
        pr = pl[off:off + 4 * sz].view(np.uint16).reshape(-1, 2).astype(np.int64)
        parts = [np.arange(s, s + l + 1, dtype=np.int64) for s, l in pr]
        return (np.concatenate(parts) if parts else np.zeros(0, np.int64)).astype(np.uint32)
    raise AssertionError(f"bad container type {t}")


def decode_bitmap(h, b):
    """Sorted uint32 values of bitmap b, and its per-container (key, type, card, size)."""
    s, e = int(h["bm_begin"][b]), int(h["bm_begin"][b + 1])
    vals, meta = [], []
    for i in range(s, e):
        key = int(h["keys"][i])
        lo = decode_container(h, i)
        vals.append((np.uint32(key) << np.uint32(16)) | lo)
        meta.append((key, int(h["types"][i]), int(h["card"][i]), int(h["size"][i])))
    v = np.concatenate(vals).astype(np.uint32) if vals else np.zeros(0, np.uint32)
    return v, meta


def oracle_meta(oracle, v):
    """(key, type, card, size) per container from the oracle's container view."""
    cv = oracle.containers(v)
    out = []
    for k, t, c, r in zip(cv["keys"], cv["types"], cv["card"], cv["runs"]):
        t = int(t)
        size = int(c) if t == ARRAY else 1024 if t == BITSET else int(r)
        out.append((int(k), t, int(c), size))
    return out


def edge_sets():
    """Bitmaps that sit on the container-type boundaries and chunk edges."""
    sets = []
    sets.append(np.zeros(0, np.uint32))                                      # empty
    sets.append(np.arange(0, 65536, dtype=np.uint32))                        # full chunk -> 1 run
    sets.append(np.array([0, 65535, 65536, 131071, 2**32 - 1], np.uint32))    # chunk edges
    sets.append(np.arange(0, 8192, 2, dtype=np.uint32))                      # 4096 singletons -> array
    sets.append(np.arange(0, 8194, 2, dtype=np.uint32))                      # 4097 singletons -> bitset
    v = []
    x = 0
    for k in [2] * 2046 + [5]:                                               # c=4097, r=2047 -> run
        v += list(range(x, x + k))
        x += k + 1
    sets.append(np.array(v, np.uint32) + np.uint32(3 * 65536))
    v2 = v[:-1] + [65535]                                                    # c=4097, r=2048 -> bitset
    sets.append(np.array(v2, np.uint32) + np.uint32(3 * 65536))
    sets.append(np.arange(5 * 65536 + 100, 5 * 65536 + 103, dtype=np.uint32))  # c=3 r=1 -> run
    sets.append(np.array([7 * 65536 + 1, 7 * 65536 + 2], np.uint32))         # c=2 r=1 -> array
    rng = np.random.default_rng(99)
    sets.append(np.unique(np.concatenate([rng.integers(0, 1 << 20, 30000), np.arange(200000, 260000),
                                          rng.integers(300000, 300000 + 65536, 40000)])).astype(np.uint32))
    sets.append(np.unique(rng.integers(0, 1 << 32, 5000, dtype=np.uint64)).astype(np.uint32))
    sets.append(np.arange(65536 * 9, 65536 * 11, 3, dtype=np.uint32))        # 2 chunks, 21846 values each
    sets.append(np.concatenate([np.arange(65536 * 9, 65536 * 9 + 40000), np.arange(65536 * 10 + 7, 65536 * 11)]
                               ).astype(np.uint32))
    # Section 1 size-rule boundaries at and below 4096 values, one chunk each:
    # key 11: c=4096, r=2048 -> array (2r < c fails);  key 12: c=4096, r=2047 -> run;
    # key 13: c=5, r=2 -> run;  key 14: c=4, r=2 -> array;
    # key 15: c=4095, r=2047 (odd c, r=(c-1)/2) -> run;  key 16: c=4095, r=2048 -> array
    sets.append(np.concatenate([_chunk_runs(11, [2] * 2048), _chunk_runs(12, [2] * 2046 + [4]),
                                _chunk_runs(13, [3, 2]), _chunk_runs(14, [2, 2]),
                                _chunk_runs(15, [2] * 2046 + [3]), _chunk_runs(16, [2] * 2047 + [1])]))
    # its partner: the same keys on the other side of each boundary (key 11:
    # c=4096, r=2047; 12: c=4096, r=2048; 13: c=4, r=2; 14: c=5, r=2; 15: c=4095,
    # r=2048; 16: c=4095, r=2047); their union gives c=4097 with r=2047 (run)
    # and c=4096 with r=2047 (run), their intersection c=4095 with r=2048 (array)
    sets.append(np.concatenate([_chunk_runs(11, [2] * 2046 + [4]), _chunk_runs(12, [2] * 2048),
                                _chunk_runs(13, [2, 2]), _chunk_runs(14, [3, 2]),
                                _chunk_runs(15, [2] * 2047 + [1]), _chunk_runs(16, [2] * 2046 + [3])]))
    return sets


def _chunk_runs(key, lengths, gap=1):
    """Values of chunk `key`: runs of the given lengths starting at 0, separated
    by `gap` absent values (so the runs are maximal and their count is exact)."""
    v, x = [], 0
    for n in lengths:
        v.extend(range(x, x + n))
        x += n + gap
    assert x - gap <= 65536
    return (np.array(v, np.uint32) + np.uint32(key * 65536)).astype(np.uint32)


def noncanonical_arrays(sets, rng, p_array=0.34, p_bitset=0.33):
    """Host pool arrays (the pool format) holding the given sorted sets in
    well-formed but not necessarily least-memory containers: each chunk is
    stored, at random, as an array (any length), a bitset (any cardinality) or
    a run list whose maximal runs are cut at random points into touching runs.
    card, bm_card and bm_wbytes are consistent with the contents."""
    keys, types, card, size, offs, chunks = [], [], [], [], [], []
    bm_begin, bm_card, bm_wbytes = [0], [], []
    pos = 0
    for v in sets:
        v = np.asarray(v, dtype=np.uint32)
        hi = v >> np.uint32(16)
        tw = 0
        for key in np.unique(hi):
            low = (v[hi == key] & np.uint32(0xFFFF)).astype(np.int64)
            c = len(low)
            u = rng.random()
            if u < p_array:
                t, pl = ARRAY, low.astype(np.uint16).tobytes()
                sz = c
            elif u < p_array + p_bitset:
                w = np.zeros(1024, np.uint64)
                np.bitwise_or.at(w, low >> 6, np.left_shift(np.uint64(1), (low & 63).astype(np.uint64)))
                t, pl, sz = BITSET, w.tobytes(), 1024
            else:
                starts = np.concatenate([[0], np.nonzero(np.diff(low) != 1)[0] + 1])
                ends = np.concatenate([starts[1:], [c]])  # exclusive indices
                runs = []
                for s0, e0 in zip(starts, ends):
                    a, b = int(low[s0]), int(low[e0 - 1])
                    cuts = sorted(set(int(x) for x in rng.integers(a + 1, b + 1, size=rng.integers(0, 3)))) if b > a \
                        else []
                    pts = [a] + cuts + [b + 1]
                    for x, y in zip(pts[:-1], pts[1:]):
                        runs.append((x, y - x - 1))
                pr = np.array(runs, np.uint16).reshape(-1, 2)
                t, pl, sz = RUN, pr.tobytes(), len(runs)
            keys.append(int(key))
            types.append(t)
            card.append(c)
            size.append(sz)
            offs.append(pos)
            padded = pl + b"\0" * ((-len(pl)) % 16)
            chunks.append(padded)
            pos += len(padded)
            tw += (min(8192, 2 * c) + 15) & ~15
        bm_begin.append(len(keys))
        bm_card.append(len(v))
        bm_wbytes.append(tw)
    payload = np.frombuffer(b"".join(chunks) or b"\0" * 16, np.uint8).copy()
    return {"bm_begin": np.array(bm_begin, np.uint64), "keys": np.array(keys, np.uint16),
            "types": np.array(types, np.uint8), "card": np.array(card, np.uint32),
            "size": np.array(size, np.uint32), "off": np.array(offs, np.uint64), "payload": payload,
            "bm_card": np.array(bm_card, np.uint64), "bm_wbytes": np.array(bm_wbytes, np.uint64)}
