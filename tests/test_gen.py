"""The seeded input generator (shared by the oracle tests and the GPU path)."""
import numpy as np

from paper_1208_3933_amd import gen


def test_splitmix64_reference_vector():
    # First outputs of SplitMix64 seeded with 1234567, as published with the
    # generator's reference implementation.
    assert [int(x) for x in gen.splitmix64(1234567, 5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_stream_offsets_are_consistent():
    a = gen.splitmix64(42, 100)
    b = gen.splitmix64(42, 60, start=40)
    assert (a[40:] == b).all()


def test_processing_times_range_and_determinism():
    p = gen.processing_times(200, 20, gen.make_seed(2, 0, 0))
    assert p.dtype == np.int32 and p.shape == (200, 20)
    assert p.min() >= 1 and p.max() <= 99
    assert (p == gen.processing_times(200, 20, gen.make_seed(2, 0, 0))).all()
    assert abs(p.mean() - 50) < 2


def test_pool_rows_are_permutations():
    pre, dep = gen.random_pool(50, 1000, gen.make_seed(1, 0, 1))
    assert pre.shape == (1000, 50) and dep.shape == (1000,)
    assert (np.sort(pre, axis=1) == np.arange(50)).all()
    assert dep.min() == 0 and dep.max() == 49
    pre2, dep2 = gen.random_pool(50, 1000, gen.make_seed(1, 0, 1))
    assert (pre == pre2).all() and (dep == dep2).all()


def test_pool_sizes_lognormal():
    s = gen.lognormal_pool_sizes(64, gen.make_seed(3, 0, 3))
    assert s.min() >= 256 and s.max() <= 131072
    assert 1000 < np.median(s) < 16000
