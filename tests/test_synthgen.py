"""The seeded input generator: published SplitMix64 values, determinism, and
agreement of the C filler with the numpy definition."""
import numpy as np

import synthgen


def test_splitmix64_published_first_output():
    # SplitMix64 started from state 0: first output 0xE220A8397B1DCDAF.
    assert int(synthgen.stream(0, 0, 1)[0]) == 0xE220A8397B1DCDAF


def test_counter_based_offsets():
    full = synthgen.stream(1234, 0, 100)
    assert np.array_equal(full[40:60], synthgen.stream(1234, 40, 20))


def test_uniform_grid_and_range():
    a = synthgen.uniform_pm1_np(1001, 200, 300)
    assert a.dtype == np.float32
    assert a.min() >= -1.0 and a.max() < 1.0
    k = a.astype(np.float64) * 2**23
    assert np.array_equal(k, np.round(k))
    assert abs(float(a.mean())) < 0.01 and abs(float(a.std()) - 1 / np.sqrt(3)) < 0.01


def test_c_filler_matches_numpy():
    synthgen.build()
    for seed in (1, 1001, 2**63 + 5):
        assert np.array_equal(synthgen.uniform_pm1(seed, 300, 301), synthgen.uniform_pm1_np(seed, 300, 301))
        assert np.array_equal(synthgen.int_range(seed, 300, 257, -2, 2),
                              synthgen.int_range_np(seed, 300, 257, -2, 2))
        assert np.array_equal(synthgen.loguniform(seed, 256, 300), synthgen.loguniform_np(seed, 256, 300))


def test_loguniform_octaves():
    a = synthgen.loguniform_np(9, 100, 1000)
    e = np.floor(np.log2(np.abs(a.astype(np.float64))))
    assert e.min() == -8 and e.max() == 7
    counts = np.bincount((e + 8).astype(int).ravel())
    assert counts.min() > 0.9 * counts.mean()
    assert 0.45 < np.mean(a < 0) < 0.55


def test_shapes_multiples_of_64():
    s = synthgen.shapes_loguniform(3001, 256)
    assert s.shape == (256, 3)
    assert np.all(s % 64 == 0) and s.min() >= 256 and s.max() <= 6144
