"""Pins of the oracle's CDF table and sampler (the error distribution of Alg. 1-2).

The sampler is pinned exhaustively: over all 2^16 keystream words, value 0 must occur
2 (T[0] + 1) times and each of +-k exactly T[k] - T[k-1] times.  The table is pinned by
properties of the distribution it encodes (symmetry, full support, variance close to
sigma^2 for the truncated discrete Gaussian)."""
import math

import numpy as np
import pytest

REGISTRY = [640, 976, 1344, 4096, 8192, 16384, 32768]


@pytest.mark.parametrize("n", REGISTRY)
def test_table_shape(orc, n):
    p = orc.params_for(n)
    T = orc.cdf_table(p.K, p.sigma).astype(np.int64)
    assert len(T) == p.K + 1
    assert T[-1] == 2**15 - 1
    assert np.all(np.diff(T) > 0), "every |e| <= K must have nonzero mass"
    assert T[0] >= 0


@pytest.mark.parametrize("n", [640, 976, 1344])
def test_exhaustive_histogram(orc, n):
    p = orc.params_for(n)
    T = orc.cdf_table(p.K, p.sigma)
    vals = np.array([orc.sample_word(u, T, p.K) for u in range(1 << 16)])
    Ti = T.astype(np.int64)
    assert (vals == 0).sum() == 2 * (Ti[0] + 1)
    for k in range(1, p.K + 1):
        assert (vals == k).sum() == Ti[k] - Ti[k - 1]
        assert (vals == -k).sum() == Ti[k] - Ti[k - 1]
    assert np.abs(vals).max() == p.K
    assert vals.sum() == 0  # symmetric
    # bit 0 of the word is the sign, bits 1..15 the magnitude rank
    assert orc.sample_word(0x0001, T, p.K) == 0
    assert orc.sample_word(0xFFFE, T, p.K) == p.K
    assert orc.sample_word(0xFFFF, T, p.K) == -p.K


@pytest.mark.parametrize("n", REGISTRY)
def test_variance_close_to_sigma(orc, n):
    p = orc.params_for(n)
    T = orc.cdf_table(p.K, p.sigma).astype(np.int64)
    prob = np.diff(np.concatenate([[-1], T])) / 32768.0  # P(|e| = k)
    var = float(sum(prob[k] * k * k for k in range(p.K + 1)))
    # discrete Gaussians of width >= 1 have variance within a few percent of sigma^2
    assert abs(var - p.sigma ** 2) < 0.05 * p.sigma ** 2


@pytest.mark.parametrize("n", [640, 976])
def test_table_against_erf_approximation(orc, n):
    """For wide tables the discrete mass follows from the continuous one: the sum over
    |x| <= k equals the integral over |x| <= k + 1/2 minus f'(k + 1/2) / 12 (midpoint
    Euler-Maclaurin), an independent route to the same numbers up to rounding."""
    p = orc.params_for(n)
    T = orc.cdf_table(p.K, p.sigma).astype(np.int64)
    s = p.sigma
    for k in range(p.K):
        x = k + 0.5
        fprime = -(x / s ** 2) * math.exp(-x * x / (2 * s * s))
        approx = 32768 * (math.erf(x / (s * math.sqrt(2))) - fprime / (12 * s * math.sqrt(2 * math.pi)))
        assert abs((T[k] + 1) - approx) < 2.5


def test_stream_is_sampler_of_keystream(orc):
    p = orc.params_for(1344)
    key = bytes(range(16, 32))
    T = orc.cdf_table(p.K, p.sigma)
    words = orc.ctr_words(key, 2, 11, 300)
    got = orc.sample_stream(p, key, 2, 11, 300)
    assert np.array_equal(got, [orc.sample_word(int(u), T, p.K) for u in words])


@pytest.mark.parametrize("n", REGISTRY)
def test_table_is_nearest_15_bit_cdf(orc, n):
    """Each entry is pinned exactly, not just near its target: the sampler gives |e| <= k with
    probability (T[k] + 1) / 2^15 (the exhaustive histogram above), and that probability must
    be the 15-bit value nearest to the truncated discrete Gaussian's P(|x| <= k).  Here the
    Gaussian sums are evaluated in 50-digit decimal arithmetic, a separate route from the
    oracle's IEEE double sums; a dropped -1, a floor in place of rounding, or a normalisation
    over the wrong support moves some entry by at least one and fails."""
    from decimal import Decimal, getcontext

    getcontext().prec = 50
    p = orc.params_for(n)
    T = orc.cdf_table(p.K, p.sigma).astype(np.int64)
    s2 = 2 * Decimal(repr(p.sigma)) ** 2
    w = [(-Decimal(x * x) / s2).exp() for x in range(p.K + 1)]
    total = w[0] + 2 * sum(w[1:])
    acc = Decimal(0)
    for k in range(p.K):
        acc += w[k] if k == 0 else 2 * w[k]
        target = Decimal(32768) * acc / total
        # not a near-tie, so that double and decimal rounding cannot disagree
        frac = target - int(target)
        assert abs(frac - Decimal("0.5")) > Decimal("1e-9"), (k, target)
        assert abs(Decimal(int(T[k]) + 1) - target) <= Decimal("0.5"), (k, int(T[k]), target)
    assert T[p.K] == 32767
