"""Pins of the oracle's counter-based noise: raw Philox4x64-10 words against
numpy's independent implementation, and the statistics of the normals."""
import numpy as np
import pytest

from oracle import rng


@pytest.mark.parametrize("seed", [0, 1, 7, 1000 + 599, 2 ** 63 + 12345, 2 ** 64 + 3])
def test_raw_words_match_numpy_philox(seed):
    ref = np.random.Philox(key=seed).random_raw(1003)
    got = rng.raw_words(seed, 1003)
    assert got.dtype == np.uint64
    assert np.array_equal(got, ref)


def test_mulhilo_against_python_integers():
    g = np.random.default_rng(5)
    a = g.integers(0, 2 ** 63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    with np.errstate(over="ignore"):
        hi, lo = rng._mulhilo(a, rng.M0)
    for x, h, l in zip(a, hi, lo):
        p = int(x) * int(rng.M0)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


def test_normals_statistics():
    z = rng.white_noise(64, 42).ravel()
    n = z.size
    assert abs(z.mean()) < 4 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 4 * np.sqrt(2.0 / n)
    # fourth moment of a unit normal is 3
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    # white: the binned power spectrum is flat (= 1 per mode)
    pk = np.abs(np.fft.rfftn(z.reshape(64, 64, 64))) ** 2 / n
    shells = [pk[1:8].mean(), pk[8:16].mean(), pk[16:32].mean()]
    assert all(abs(s - 1.0) < 0.05 for s in shells)


def test_box_muller_pairs_follow_the_recipe():
    """Element 4c+1 and 4c uses words (4c, 4c+1): r sin / r cos of the same
    angle, so z0^2 + z1^2 = -2 ln(1 - u0)."""
    w = rng.raw_words(9, 8)
    u = (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    z = rng.white_noise(2, 9).ravel()
    assert np.isclose(z[0] ** 2 + z[1] ** 2, -2 * np.log1p(-u[0]), rtol=1e-14)
    assert np.isclose(np.arctan2(z[1], z[0]) % (2 * np.pi), 2 * np.pi * u[1], rtol=1e-12)
    assert np.isclose(z[2] ** 2 + z[3] ** 2, -2 * np.log1p(-u[2]), rtol=1e-14)
