"""Pins for the oracle's Philox4x32-10 / Box-Muller stream (sketch matrix of
Alg. 1, step 1).  No published known-answer values are available offline, so
the stream is pinned by two independent formulations (vectorised uint64 vs
Python big integers), by structural properties of the definition, and by the
distribution the paper asks for (i.i.d. standard normal)."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


def test_vectorised_matches_bigint_formulation():
    rng = np.random.default_rng(0)
    ctrs = rng.integers(0, 2 ** 32, size=(64, 4), dtype=np.uint64)
    ctrs[0] = 0
    ctrs[1] = 2 ** 32 - 1
    keys = rng.integers(0, 2 ** 32, size=(64, 2), dtype=np.uint64)
    keys[0] = 0
    keys[1] = 2 ** 32 - 1
    for (c0, c1, c2, c3), (k0, k1) in zip(ctrs, keys):
        v = philox.philox4x32(np.array([c0]), np.array([c1]), np.array([c2]), np.array([c3]), k0, k1)
        s = philox.philox4x32_scalar((c0, c1, c2, c3), (k0, k1))
        assert tuple(int(w[0]) for w in v) == s


def test_round_count_matters_and_key_matters():
    a = philox.philox4x32_scalar((1, 2, 3, 4), (5, 6), rounds=10)
    b = philox.philox4x32_scalar((1, 2, 3, 4), (5, 6), rounds=9)
    c = philox.philox4x32_scalar((1, 2, 3, 4), (5, 7), rounds=10)
    assert a != b and a != c


def test_one_round_is_the_published_bijection():
    # one round from a zero key: outputs follow the multiply/xor/swap rule
    c = (0x12345678, 0x9ABCDEF0, 0x0FEDCBA9, 0x87654321)
    out = philox.philox4x32_scalar(c, (0, 0), rounds=1)
    p0 = 0xD2511F53 * c[0]
    p1 = 0xCD9E8D57 * c[2]
    assert out == ((p1 >> 32) ^ c[1], p1 & 0xFFFFFFFF, (p0 >> 32) ^ c[3], p0 & 0xFFFFFFFF)


def test_uniform_words_are_uniform():
    n = 1 << 18
    L = np.arange(n, dtype=np.uint64)
    w = philox.philox4x32(L, np.zeros_like(L), np.zeros_like(L), np.zeros_like(L), 42, 0)
    for word in w:
        counts = np.bincount((word >> np.uint64(24)).astype(np.int64), minlength=256)
        chi2 = float(np.sum((counts - n / 256) ** 2 / (n / 256)))
        assert stats.chi2.sf(chi2, 255) > 1e-4


def test_unit_interval_is_open():
    zero = np.array([0], dtype=np.uint64)
    top = np.array([2 ** 32 - 1], dtype=np.uint64)
    assert philox.words_to_unit(zero, zero)[0] == 0.5 * 2.0 ** -52
    assert philox.words_to_unit(top, top)[0] < 1.0


def test_gaussian_moments_and_ks():
    z = philox.gaussian_at(2024, 1, np.arange(1 << 20, dtype=np.uint64))
    assert abs(z.mean()) < 5e-3
    assert abs(z.var() - 1.0) < 5e-3
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # even and odd indices (cos and sin halves) are each standard normal and
    # uncorrelated with each other
    assert stats.kstest(z[0::2], "norm").pvalue > 1e-4
    assert stats.kstest(z[1::2], "norm").pvalue > 1e-4
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 5e-3


def test_omega_layout_and_nesting():
    J, S = 37, 5
    Om = philox.omega(9, 2, J, S)
    flat = philox.gaussian_at(9, 2, np.arange(J * S, dtype=np.uint64))
    assert np.array_equal(Om[:, 3], flat[3 * J:4 * J])          # column-major index
    assert np.array_equal(philox.omega(9, 2, J, 8)[:, :S], Om)  # nested in S
    assert not np.array_equal(philox.omega(9, 1, J, S), Om)     # mode enters the counter
    assert not np.array_equal(philox.omega(10, 2, J, S), Om)    # seed enters the key


def test_seed_key_split():
    assert philox.seed_key(0x1122334455667788) == (0x55667788, 0x11223344)
