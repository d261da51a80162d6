"""CPU oracle - TEST INFRASTRUCTURE ONLY.

The plain definition of what the GPU library computes, written from the paper
(Lemire et al., arXiv:1709.07821) as two-pointer merges over sorted uint32
lists (oracle.c). Only tests/, the smoke check and the benchmark's CPU-baseline
leg may import it. It shares no code with the GPU library and does not import
it; the GPU library must never import or call this module.

Functions (all take strictly increasing uint32 numpy arrays):

* ``op(name, a, b)``      - result list of and/or/xor/andnot (Section 1 set ops)
* ``count(name, a, b)``   - result size only (Section 5.9, Fast Counts)
* ``jaccard(a, b)``       - |A n B| / |A u B| as one binary64 division; J(0/0) = 1
* ``kway(name, lists)``   - left fold of the two-way op (and/or)
* ``containers(v)``       - container view: key, P1 type, card, runs, first index
* ``type_of(c, r)``       - P1 type rule (Section 1 size rules, least memory)
* ``serialise(v, i)``     - words of container i in the fingerprint layout
* ``digest(v)``           - canonical fingerprint of the container form
* ``contains(v, x)``      - membership of one value (Section 1 random access)
* ``contains_many(values, offsets, ids, xs)`` - batched membership over a collection

Export to uint32 (Section 3.1, Section 5.5) has no function here: the oracle
holds every set as its sorted uint32 list, which is the expected export.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")

OPS = {"and": 0, "or": 1, "xor": 2, "andnot": 3}
ARRAY, BITSET, RUN = 1, 2, 3

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u16p = ctypes.POINTER(ctypes.c_uint16)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)
_lib = None


def build():
    import subprocess

    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", _LIB, os.path.join(_HERE, "oracle.c")],
                   check=True)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        for nm in ("ora_and", "ora_or", "ora_xor", "ora_andnot"):
            f = getattr(L, nm)
            f.restype = ctypes.c_uint64
            f.argtypes = [_u32p, ctypes.c_uint64, _u32p, ctypes.c_uint64, _u32p]
        L.ora_op.restype = ctypes.c_uint64
        L.ora_op.argtypes = [ctypes.c_int, _u32p, ctypes.c_uint64, _u32p, ctypes.c_uint64, _u32p]
        L.ora_jaccard.restype = ctypes.c_double
        L.ora_jaccard.argtypes = [_u32p, ctypes.c_uint64, _u32p, ctypes.c_uint64]
        L.ora_kway.restype = ctypes.c_uint64
        L.ora_kway.argtypes = [ctypes.c_int, ctypes.POINTER(_u32p), _u64p, ctypes.c_uint32, _u32p, _u32p]
        L.ora_type_of.restype = ctypes.c_int
        L.ora_type_of.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.ora_container_count.restype = ctypes.c_uint64
        L.ora_container_count.argtypes = [_u32p, ctypes.c_uint64]
        L.ora_containers.restype = None
        L.ora_containers.argtypes = [_u32p, ctypes.c_uint64, _u16p, _u8p, _u32p, _u32p, _u64p]
        L.ora_digest.restype = ctypes.c_uint64
        L.ora_digest.argtypes = [_u32p, ctypes.c_uint64]
        L.ora_pairs.restype = None
        L.ora_pairs.argtypes = [ctypes.c_int, _u32p, _u64p, _u32p, _u64p, _u32p, _u32p, ctypes.c_uint64,
                                _u64p, _u64p, _f64p, _u32p]
        L.ora_contains.restype = ctypes.c_int
        L.ora_contains.argtypes = [_u32p, ctypes.c_uint64, ctypes.c_uint32]
        L.ora_contains_many.restype = None
        L.ora_contains_many.argtypes = [_u32p, _u64p, _u32p, _u32p, ctypes.c_uint64, _u8p]
        L.ora_serialise.restype = ctypes.c_uint64
        L.ora_serialise.argtypes = [_u32p, ctypes.c_uint64, ctypes.c_uint64, _u64p]
        _lib = L
    return _lib


def _c32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(_u32p)


def op(name: str, a, b) -> np.ndarray:
    a, pa = _c32(a)
    b, pb = _c32(b)
    cap = len(a) + len(b) if name in ("or", "xor") else (len(a) if name == "andnot" else min(len(a), len(b)))
    out = np.zeros(max(cap, 1), dtype=np.uint32)
    n = _load().ora_op(OPS[name], pa, len(a), pb, len(b), out.ctypes.data_as(_u32p))
    return out[:n]


def count(name: str, a, b) -> int:
    a, pa = _c32(a)
    b, pb = _c32(b)
    return int(_load().ora_op(OPS[name], pa, len(a), pb, len(b), None))


def jaccard(a, b) -> float:
    a, pa = _c32(a)
    b, pb = _c32(b)
    return float(_load().ora_jaccard(pa, len(a), pb, len(b)))


def kway(name: str, lists) -> np.ndarray:
    arrs = [np.ascontiguousarray(l, dtype=np.uint32) for l in lists]
    k = len(arrs)
    if k == 0:
        return np.zeros(0, np.uint32)
    # a union or symmetric difference can hold every input value; an
    # intersection or difference at most the first input's
    cap = sum(len(a) for a in arrs) if name in ("or", "xor") else len(arrs[0])
    ptrs = (_u32p * k)(*[a.ctypes.data_as(_u32p) for a in arrs])
    lens = np.array([len(a) for a in arrs], dtype=np.uint64)
    out = np.zeros(max(cap, 1), np.uint32)
    tmp = np.zeros(max(cap, 1), np.uint32)
    n = _load().ora_kway(OPS[name], ptrs, lens.ctypes.data_as(_u64p), k, out.ctypes.data_as(_u32p),
                         tmp.ctypes.data_as(_u32p))
    return out[:n]


def type_of(c: int, r: int) -> int:
    return int(_load().ora_type_of(c, r))


def containers(v):
    """Container view of a sorted set: dict of numpy arrays keys/types/card/runs/first."""
    v, pv = _c32(v)
    L = _load()
    k = int(L.ora_container_count(pv, len(v)))
    keys = np.zeros(k, np.uint16)
    types = np.zeros(k, np.uint8)
    card = np.zeros(k, np.uint32)
    runs = np.zeros(k, np.uint32)
    first = np.zeros(k, np.uint64)
    L.ora_containers(pv, len(v), keys.ctypes.data_as(_u16p), types.ctypes.data_as(_u8p),
                     card.ctypes.data_as(_u32p), runs.ctypes.data_as(_u32p), first.ctypes.data_as(_u64p))
    return {"keys": keys, "types": types, "card": card, "runs": runs, "first": first}


def serialise(v, idx: int) -> np.ndarray:
    """Words of container number idx in the digest's serialised layout."""
    v, pv = _c32(v)
    w = np.zeros(1026, np.uint64)
    n = int(_load().ora_serialise(pv, len(v), idx, w.ctypes.data_as(_u64p)))
    return w[:n]


def digest(v) -> int:
    v, pv = _c32(v)
    return int(_load().ora_digest(pv, len(v)))


def pairs(name: str, va, oa, vb, ob, ia, ib, want_card=True, want_digest=False, want_jaccard=False):
    """Per-pair op over two collections (values + offsets); returns (card, digest, jaccard) arrays."""
    va, pva = _c32(va)
    vb, pvb = _c32(vb)
    oa = np.ascontiguousarray(oa, dtype=np.uint64)
    ob = np.ascontiguousarray(ob, dtype=np.uint64)
    ia, pia = _c32(ia)
    ib, pib = _c32(ib)
    n = len(ia)
    card = np.zeros(n, np.uint64) if want_card else None
    dig = np.zeros(n, np.uint64) if want_digest else None
    jac = np.zeros(n, np.float64) if want_jaccard else None
    maxa = int(np.max(np.diff(oa))) if len(oa) > 1 else 0
    maxb = int(np.max(np.diff(ob))) if len(ob) > 1 else 0
    tmp = np.zeros(max(maxa + maxb, 1), np.uint32)
    _load().ora_pairs(OPS[name], pva, oa.ctypes.data_as(_u64p), pvb, ob.ctypes.data_as(_u64p), pia, pib, n,
                      card.ctypes.data_as(_u64p) if card is not None else None,
                      dig.ctypes.data_as(_u64p) if dig is not None else None,
                      jac.ctypes.data_as(_f64p) if jac is not None else None, tmp.ctypes.data_as(_u32p))
    return card, dig, jac


def contains(v, x: int) -> bool:
    v, pv = _c32(v)
    return bool(_load().ora_contains(pv, len(v), int(x)))


def contains_many(values, offsets, ids, xs) -> np.ndarray:
    """out[i] = xs[i] in set ids[i] of the collection (values, offsets); uint8."""
    values, pv = _c32(values)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    ids, pi = _c32(ids)
    xs, px = _c32(xs)
    out = np.zeros(max(len(ids), 1), np.uint8)
    _load().ora_contains_many(pv, offsets.ctypes.data_as(_u64p), pi, px, len(ids), out.ctypes.data_as(_u8p))
    return out[:len(ids)]
