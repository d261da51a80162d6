"""The seeded input generators: published SplitMix64 outputs, determinism and
the shape of each workload recipe."""
import numpy as np

import synth


def test_splitmix64_reference_outputs():
    # SplitMix64 with state 0: first three outputs of the published generator
    g = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1
    assert synth.mix64(g) == 0xE220A8397B1DCDAF
    assert synth.mix64((2 * g) & M) == 0x6E789E6AA1B965F4
    assert synth.mix64((3 * g) & M) == 0x06C45D188009454F


def test_counter_based_definition():
    g = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1
    seed, stream, ctr = 12345, 7, 99
    key = synth.mix64((seed + (stream + 1) * g) & M)
    assert synth.rand(seed, stream, ctr) == synth.mix64((key + (ctr + 1) * g) & M)


def test_mixed_small_shape_and_determinism():
    s = synth.mixed_small(n_bitmaps=12)
    s2 = synth.mixed_small(n_bitmaps=12)
    assert np.array_equal(s.values, s2.values) and np.array_equal(s.offsets, s2.offsets)
    for i in range(len(s)):
        v = s[i]
        assert v.size > 0 and np.all(np.diff(v.astype(np.int64)) > 0)
        assert int(v[-1]) < (1 << 26)
        assert 500 <= v.size <= 50000


def test_array_stress_shape():
    bs, ia, ib = synth.array_stress(n_pairs=2000)
    sizes = np.diff(bs.offsets)
    assert len(bs) == 4000 and sizes.min() >= 1 and sizes.max() <= 4096
    a, b = sizes[0::2], sizes[1::2]
    assert np.all(np.maximum(a, b) <= 1000 * np.minimum(a, b))
    for i in range(0, 4000, 97):
        v = bs[i]
        assert np.all(np.diff(v.astype(np.int64)) > 0) and int(v[-1]) < 65536
    assert np.array_equal(ia + 1, ib)


def test_dense_container_density():
    for b, k in [(0, 0), (5, 17), (19999, 255)]:
        w = synth.dense_container(b, k)
        c = sum(bin(int(x)).count("1") for x in w)
        assert 0.18 * 65536 < c < 0.82 * 65536
    v = synth.dense_bitmap_values(3, n_keys=4)
    assert np.all(np.diff(v.astype(np.int64)) > 0) and int(v[-1]) < 4 * 65536


def test_random_pairs():
    ia, ib = synth.random_pairs(20000, 5000, seed=synth.DENSE_SEED)
    assert ia.max() < 20000 and ib.max() < 20000 and np.all(ia != ib)
    ia2, ib2 = synth.random_pairs(20000, 5000, seed=synth.DENSE_SEED)
    assert np.array_equal(ia, ia2) and np.array_equal(ib, ib2)
