"""Pins for the oracle's Gaussian test matrix (the randn step of Algorithm 1).

The oracle's Philox4x64-10 is checked word for word against numpy's own,
independently written Philox bit generator; the normal variates against
their distribution; the layout against the prefix property.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import philox as ph


@pytest.mark.parametrize("key", [(0, 0), (1, 2), (2 ** 64 - 1, 12345), (0xDEADBEEF, 7)])
def test_words_match_numpy_philox(key):
    n = 64
    ours = ph.gaussian_words(n, key[0], key[1], first_block=5)
    # numpy's generator advances the counter before producing a block, so a
    # generator started at counter c yields the block for c + 1 first.
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array([4, 0, 0, 0], dtype=np.uint64))
    ref = g.random_raw(4 * n).astype(np.uint64).reshape(n, 4)
    assert np.array_equal(ours, ref)


def test_words_high_counter_words_and_carry():
    ctr = np.array([[2 ** 64 - 1, 3, 2 ** 63, 9]], dtype=np.uint64)
    ours = ph.philox4x64_10(ctr, (11, 22))
    g = np.random.Philox(key=np.array([11, 22], dtype=np.uint64),
                          counter=np.array([2 ** 64 - 2, 3, 2 ** 63, 9], dtype=np.uint64))
    assert np.array_equal(ours, g.random_raw(4).astype(np.uint64).reshape(1, 4))


def test_mulhilo_against_python_integers():
    r = np.random.default_rng(3)
    a = r.integers(0, 2 ** 63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = r.integers(0, 2 ** 63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    hi, lo = ph._mulhilo(a, b)
    for x, y, h, lw in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(lw) == p & (2 ** 64 - 1)


def test_uniform_mapping_extremes():
    w = np.array([0, 2 ** 64 - 1, 2 ** 63], dtype=np.uint64)
    u = ph.uniforms_from_words(w)
    assert u[0] == 0.5 * 2.0 ** -52
    assert u[1] == 1.0 - 0.5 * 2.0 ** -52
    assert u[2] == 0.5 + 0.5 * 2.0 ** -52
    assert np.all((u > 0) & (u < 1))


def test_box_muller_on_chosen_words():
    # u_a = 0.5*2^-52*(2k+1); pick words giving u_a = 0.5 +- tiny, u_b = 0.25
    wa = np.uint64(2 ** 63)            # u = 0.5 + 2^-53
    wb = np.uint64(2 ** 62)            # u = 0.25 + 2^-53
    z = ph.normals_from_block_words(np.array([[wa, wb, wa, wb]], dtype=np.uint64))[0]
    ua = 0.5 + 2.0 ** -53
    ub = 0.25 + 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(ua))
    assert z[0] == pytest.approx(r * np.cos(2 * np.pi * ub), abs=1e-15)
    assert z[1] == pytest.approx(r * np.sin(2 * np.pi * ub), abs=1e-15)
    assert z[1] == pytest.approx(np.sqrt(2 * np.log(2.0)), rel=1e-12)


def test_gaussian_moments_and_ks():
    z = ph.gaussian_matrix(1000, 500, seed=42).ravel()
    assert abs(z.mean()) < 5e-3
    assert abs(z.std() - 1.0) < 5e-3
    assert abs(stats.skew(z)) < 1e-2
    assert abs(stats.kurtosis(z)) < 2e-2
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_prefix_property_and_column_major_index():
    a = ph.gaussian_matrix(37, 11, seed=9)
    b = ph.gaussian_matrix(37, 4, seed=9)
    assert np.array_equal(a[:, :4], b)
    flat = ph.normals_from_block_words(ph.gaussian_words((37 * 11 + 3) // 4, 9)).ravel()
    i, j = 13, 7
    assert a[i, j] == flat[i + j * 37]


def test_streams_and_seeds_differ():
    a = ph.gaussian_matrix(16, 4, seed=1, stream=0)
    b = ph.gaussian_matrix(16, 4, seed=1, stream=1)
    c = ph.gaussian_matrix(16, 4, seed=2, stream=0)
    assert not np.allclose(a, b) and not np.allclose(a, c)
