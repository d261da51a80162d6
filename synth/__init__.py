"""Seeded synthetic inputs shared by the GPU library's tests/bench and the oracle.

This module only draws integer sets (sorted uint32 value lists, or raw bitset
words for the dense-bitset workload). It holds none of the set-operation
arithmetic or container logic of either side. The generator is SplitMix64
used as a counter-based generator (see synth.c for the definition).

A collection of bitmaps is returned as ``BitmapSet(values, offsets)``: bitmap i
holds ``values[offsets[i]:offsets[i+1]]``, strictly increasing.

Workload recipes (sizes and distributions follow the paper's evaluation
shapes; the paper's own datasets are not available, these stand in for them):

* ``mixed_small``  - 100 bitmaps over [0, 2^26), 1k-50k values each, 40 %
  sparse / 30 % dense window / 30 % clustered runs, consecutive pairs.
* ``array_stress`` - 1e5 pairs of single-container bitmaps (key 0) whose sizes
  are truncated Zipf(1.2) on [1, 4096] with size ratio at most 1000.
* ``dense_bitsets`` - 2e4 bitmaps x 256 bitset containers at density
  U(0.2, 0.8), 1e4 random pairs; generated on the device, with a CPU twin that
  regenerates any bitmap on demand.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libsynth.so")
_LIB_GPU = os.path.join(_HERE, "libsynth_gpu.so")

SEED_BASE = 17090782

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_lib = None
_lib_gpu = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            from . import build as _b

            _b.build_cpu()
        L = ctypes.CDLL(_LIB)
        L.synth_mix64.restype = ctypes.c_uint64
        L.synth_mix64.argtypes = [ctypes.c_uint64]
        L.synth_rand.restype = ctypes.c_uint64
        L.synth_rand.argtypes = [ctypes.c_uint64] * 3
        L.synth_mixed_bitmap.restype = ctypes.c_uint64
        L.synth_mixed_bitmap.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                         _u32p, ctypes.c_uint32, _u32p]
        L.synth_hot_keys.restype = None
        L.synth_hot_keys.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u32p]
        L.synth_zipf_pair_sizes.restype = None
        L.synth_zipf_pair_sizes.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                            ctypes.c_uint32, ctypes.c_uint32, _u32p, _u32p]
        L.synth_distinct_u16.restype = None
        L.synth_distinct_u16.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u32p]
        L.synth_dense_container.restype = None
        L.synth_dense_container.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _u64p]
        L.synth_dense_bitmap_values.restype = ctypes.c_uint64
        L.synth_dense_bitmap_values.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _u32p]
        L.synth_random_pairs.restype = None
        L.synth_random_pairs.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         _u32p, _u32p]
        L.synth_lognormal_card.restype = ctypes.c_uint64
        L.synth_lognormal_card.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64]
        L.synth_sort_unique.restype = ctypes.c_uint64
        L.synth_sort_unique.argtypes = [_u32p, ctypes.c_uint64]
        _lib = L
    return _lib


def _p32(a):
    return a.ctypes.data_as(_u32p)


def _p64(a):
    return a.ctypes.data_as(_u64p)


def mix64(z: int) -> int:
    return int(_load().synth_mix64(z))


def rand(seed: int, stream: int, ctr: int) -> int:
    return int(_load().synth_rand(seed, stream, ctr))


@dataclass
class BitmapSet:
    values: np.ndarray   # uint32, concatenated sorted distinct values
    offsets: np.ndarray  # uint64 [n + 1]

    def __len__(self):
        return len(self.offsets) - 1

    def __getitem__(self, i):
        return self.values[int(self.offsets[i]):int(self.offsets[i + 1])]

    @staticmethod
    def from_list(lists):
        offs = np.zeros(len(lists) + 1, dtype=np.uint64)
        for i, l in enumerate(lists):
            offs[i + 1] = offs[i] + len(l)
        vals = np.concatenate([np.asarray(l, dtype=np.uint32) for l in lists]) if lists else np.zeros(0, np.uint32)
        return BitmapSet(vals.astype(np.uint32), offs)


def sort_unique(v) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(v, dtype=np.uint32)).copy()
    n = int(_load().synth_sort_unique(_p32(a), len(a)))
    return a[:n]


def hot_keys(seed: int, n_hot: int, n_chunks: int, stream: int = 1 << 42) -> np.ndarray:
    out = np.zeros(n_hot, dtype=np.uint32)
    _load().synth_hot_keys(seed, stream, n_hot, n_chunks, _p32(out))
    return out


def mixed_bitmap(seed: int, index: int, n_target: int, ulog2: int, hot: np.ndarray) -> np.ndarray:
    hot = np.ascontiguousarray(hot, dtype=np.uint32)
    out = np.zeros(max(n_target, 1), dtype=np.uint32)
    n = _load().synth_mixed_bitmap(seed, index, n_target, ulog2, _p32(hot), len(hot), _p32(out))
    return out[:n].copy()


# ---------------------------------------------------------------- recipes

def mixed_small(n_bitmaps: int = 100, seed: int = SEED_BASE + 0, n_min: int = 1000, n_max: int = 50000,
                ulog2: int = 26, n_hot: int = 32) -> BitmapSet:
    """100 bitmaps over [0, 2^26), sizes U{1000..50000}, 40/30/30 sparse/dense/run mix."""
    hot = hot_keys(seed, n_hot, 1 << (ulog2 - 16))
    lists = []
    for i in range(n_bitmaps):
        n = n_min + rand(seed, 1_000_000 + i, 0) % (n_max - n_min + 1)
        lists.append(mixed_bitmap(seed, i, n, ulog2, hot))
    return BitmapSet.from_list(lists)


def consecutive_pairs(n_bitmaps: int):
    ia = np.arange(n_bitmaps - 1, dtype=np.uint32)
    return ia, ia + 1


def array_stress(n_pairs: int = 100_000, seed: int = SEED_BASE + 1, s: float = 1.2, kmax: int = 4096,
                 rmax: int = 1000) -> tuple[BitmapSet, np.ndarray, np.ndarray]:
    """Pairs of one-container bitmaps (key 0); bitmap 2p is A_p, bitmap 2p+1 is B_p."""
    L = _load()
    ca = np.zeros(n_pairs, dtype=np.uint32)
    cb = np.zeros(n_pairs, dtype=np.uint32)
    L.synth_zipf_pair_sizes(seed, 0, n_pairs, s, kmax, rmax, _p32(ca), _p32(cb))
    sizes = np.empty(2 * n_pairs, dtype=np.uint64)
    sizes[0::2] = ca
    sizes[1::2] = cb
    offs = np.zeros(2 * n_pairs + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    vals = np.zeros(int(offs[-1]), dtype=np.uint32)
    base = vals.ctypes.data
    for i in range(2 * n_pairs):
        o = int(offs[i])
        L.synth_distinct_u16(seed, (1 << 32) + i, int(sizes[i]), 0,
                             ctypes.cast(base + 4 * o, _u32p))
    ia = np.arange(0, 2 * n_pairs, 2, dtype=np.uint32)
    return BitmapSet(vals, offs), ia, ia + 1


def uniform_size_pairs(n_pairs: int, seed: int, a_range, b_range) -> tuple[BitmapSet, np.ndarray, np.ndarray]:
    """Pairs of one-container bitmaps (key 0) with sizes uniform on the given
    inclusive ranges (sizes above 4096 give bitset containers); bitmap 2p is
    A_p, bitmap 2p+1 is B_p; values distinct uniform uint16, sorted."""
    L = _load()
    sizes = np.empty(2 * n_pairs, dtype=np.uint64)
    for i in range(2 * n_pairs):
        lo, hi = a_range if i % 2 == 0 else b_range
        sizes[i] = lo + rand(seed, 1 << 44, i) % (hi - lo + 1)
    offs = np.zeros(2 * n_pairs + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    vals = np.zeros(int(offs[-1]), dtype=np.uint32)
    base = vals.ctypes.data
    for i in range(2 * n_pairs):
        L.synth_distinct_u16(seed, (1 << 45) + i, int(sizes[i]), 0, ctypes.cast(base + 4 * int(offs[i]), _u32p))
    ia = np.arange(0, 2 * n_pairs, 2, dtype=np.uint32)
    return BitmapSet(vals, offs), ia, ia + 1


def random_pairs(n: int, n_pairs: int, seed: int, stream: int = 1 << 41):
    ia = np.zeros(n_pairs, dtype=np.uint32)
    ib = np.zeros(n_pairs, dtype=np.uint32)
    _load().synth_random_pairs(seed, stream, n, n_pairs, _p32(ia), _p32(ib))
    return ia, ib


DENSE_SEED = SEED_BASE + 2


def dense_container(b: int, k: int, seed: int = DENSE_SEED) -> np.ndarray:
    w = np.zeros(1024, dtype=np.uint64)
    _load().synth_dense_container(seed, b, k, _p64(w))
    return w


def dense_bitmap_values(b: int, n_keys: int = 256, seed: int = DENSE_SEED) -> np.ndarray:
    out = np.zeros(n_keys * 65536, dtype=np.uint32)
    n = _load().synth_dense_bitmap_values(seed, b, n_keys, _p32(out))
    return out[:n].copy()


def dense_bitsets_device(words_ptr: int, b0: int, n_bitmaps: int, n_keys: int, stream_ptr: int = 0,
                         seed: int = DENSE_SEED) -> None:
    """Fill device memory at words_ptr with bitmaps b0..b0+n_bitmaps-1, laid out [bitmap][key][1024] u64."""
    global _lib_gpu
    if _lib_gpu is None:
        if not os.path.exists(_LIB_GPU):
            raise RuntimeError("synth/libsynth_gpu.so is not built (run __graft_entry__.build())")
        _lib_gpu = ctypes.CDLL(_LIB_GPU)
        _lib_gpu.synth_dense_bitsets_device.restype = ctypes.c_int
        _lib_gpu.synth_dense_bitsets_device.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                                        ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    rc = _lib_gpu.synth_dense_bitsets_device(seed, b0, n_bitmaps, n_keys, ctypes.c_void_p(words_ptr),
                                             ctypes.c_void_p(stream_ptr))
    if rc != 0:
        raise RuntimeError(f"synth_dense_bitsets_device failed: {rc}")


def lognormal_card(idx: int, median: float, sigma: float, lo: int, hi: int, seed: int, stream: int = 1 << 43):
    return int(_load().synth_lognormal_card(seed, stream, idx, median, sigma, lo, hi))
