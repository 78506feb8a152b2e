"""Pins for the oracle's probe generator (SplitMix64, Rademacher entries)."""
import numpy as np

from oracle import rng


def test_splitmix64_published_vector():
    # First five outputs of SplitMix64 seeded with 1234567, the test vector of
    # the generator's reference implementation (S. Vigna, splitmix64.c).
    got = [int(v) for v in rng.splitmix64_outputs(1234567, 5)]
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_rademacher_values_and_balance():
    S = rng.rademacher(7, 0, 4096, 16)
    assert set(np.unique(S)) == {-1.0, 1.0}
    # mean of 65536 fair signs: |mean| < 5/sqrt(N)
    assert abs(S.mean()) < 5.0 / np.sqrt(S.size)
    # columns nearly uncorrelated
    C = S.T @ S / S.shape[0]
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 5.0 / np.sqrt(S.shape[0])


def test_rademacher_layout_independent_of_width():
    a = rng.rademacher(3, 1, 1000, 4)
    b = rng.rademacher(3, 1, 1000, 9)
    np.testing.assert_array_equal(a, b[:, :4])
    # streams and seeds differ
    assert not np.array_equal(rng.rademacher(3, 0, 1000, 4), a)
    assert not np.array_equal(rng.rademacher(4, 1, 1000, 4), a)


def test_rademacher_entry_definition():
    # entry(row, col) = sign of output (col*n + row + 1) of SplitMix64(key)
    n = 37
    key = rng.stream_key(11, 1)
    x = int(rng.splitmix64_outputs(key, 1, start=2 * n + 5 + 1)[0])
    S = rng.rademacher(11, 1, n, 3)
    assert S[5, 2] == (-1.0 if x >> 63 else 1.0)


def test_gaussian_entries_are_standard_normal():
    # Kolmogorov-Smirnov against N(0, 1), moments, and no correlation between
    # columns or streams; entries depend on (seed, stream, row, col) only.
    from scipy import stats

    n, c = 40000, 3
    G = rng.gaussian(11, 1, n, c)
    for j in range(c):
        assert stats.kstest(G[:, j], "norm").pvalue > 1e-3
    x = G.ravel()
    se = 1.0 / np.sqrt(x.size)
    assert abs(x.mean()) < 5 * se
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0) * se
    assert abs(stats.kurtosis(x, fisher=False) - 3.0) < 5 * np.sqrt(24.0) * se
    C = np.corrcoef(np.hstack([G, rng.gaussian(11, 0, n, 1)]).T)
    assert np.abs(C - np.eye(c + 1)).max() < 5.0 / np.sqrt(n)
    assert np.array_equal(rng.gaussian(11, 1, 500, 2)[:, 1], rng.gaussian(11, 1, 500, 3)[:, 1])
    assert not np.array_equal(rng.gaussian(11, 1, 500, 1), rng.gaussian(12, 1, 500, 1))
