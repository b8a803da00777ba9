"""Pins of the sensor-noise oracle (paper section III.A: Gaussian sensor noise at a
drawn SNR; the deviates come from a counter-based generator that the GPU library and
the oracle each implement from its published definition).

* Philox4x32-10 against the known-answer vectors published with the generator
  (tests/golden/philox4x32_10_kat.json): a wrong multiplier, word order, key schedule
  or round count fails them.
* The Box-Muller deviates against the standard normal law (Kolmogorov-Smirnov test
  with scipy's normal CDF, moments), and independence across microphones, rooms and
  the four words of one counter.
* The counter layout: a prefix of a longer draw is the shorter draw.
"""
import json
import os

import numpy as np
import pytest
from scipy import stats

from oracle import noise

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")


def test_philox_known_answer_vectors():
    kat = json.load(open(GOLDEN))
    for v in kat["vectors"]:
        ctr = [int(w, 16) for w in v["counter"]]
        key = [int(w, 16) for w in v["key"]]
        got = noise.philox4x32_10([ctr], key)[0]
        assert ["%08x" % int(w) for w in got] == v["out"]


def test_philox_words_are_uniform():
    # 2^18 counters: the top byte of every word is flat (chi-square), and consecutive counters
    # give uncorrelated words
    j = np.arange(1 << 18)
    w = noise.philox4x32_10(np.stack([j, 0 * j + 3, 0 * j + 5, 0 * j], axis=1), (12345, 678))
    top = (w >> np.uint64(24)).astype(np.int64)
    for k in range(4):
        h = np.bincount(top[:, k], minlength=256)
        assert stats.chisquare(h).pvalue > 1e-4
    u = noise.uniforms(w)
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(np.corrcoef(u[:-1, 0], u[1:, 0])[0, 1]) < 5.0 / np.sqrt(len(u))


def test_deviates_are_standard_normal_and_independent():
    n = 200000
    z = noise.deviates(2108, 7, 4, n)
    assert z.shape == (4, n)
    for m in range(4):
        assert stats.kstest(z[m], "norm").pvalue > 1e-4
        assert abs(z[m].mean()) < 5.0 / np.sqrt(n)
        assert abs(z[m].var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
        assert abs(stats.kurtosis(z[m], fisher=False) - 3.0) < 0.1
    c = np.corrcoef(z)
    assert np.all(np.abs(c[np.triu_indices(4, 1)]) < 5.0 / np.sqrt(n))
    # the four samples drawn from one counter (cos/sin pairs) are uncorrelated
    q = z[0].reshape(-1, 4).T
    cq = np.corrcoef(q)
    assert np.all(np.abs(cq[np.triu_indices(4, 1)]) < 5.0 / np.sqrt(n / 4))
    # another room and another seed give unrelated streams
    o = noise.deviates(2108, 8, 1, n)[0]
    s = noise.deviates(2109, 7, 1, n)[0]
    assert abs(np.corrcoef(z[0], o)[0, 1]) < 5.0 / np.sqrt(n)
    assert abs(np.corrcoef(z[0], s)[0, 1]) < 5.0 / np.sqrt(n)
    assert np.abs(z).max() <= np.sqrt(48.0 * np.log(2.0)) + 1e-12


def test_deviates_prefix_and_tail_probability():
    a = noise.deviates(5, 2, 3, 1001)
    b = noise.deviates(5, 2, 3, 37)
    assert np.array_equal(a[:, :37], b)
    # P(|z| < 1) of the standard normal, 0.682689...
    z = noise.deviates(99, 0, 2, 100000).ravel()
    p = np.mean(np.abs(z) < 1.0)
    assert abs(p - (stats.norm.cdf(1.0) - stats.norm.cdf(-1.0))) < 5.0 * np.sqrt(0.25 / z.size)
