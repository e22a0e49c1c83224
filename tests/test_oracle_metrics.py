"""Pins of oracle/metrics.py against hand-worked values.

Every GPU parity gate goes through ``metrics.compare``; each case below is
computed by hand (in the comments) so that a wrong normaliser, a dropped
conjugate, a swapped reference/tested pair or a wrong 2^N factor fails.
"""

import math

import numpy as np
import pytest

from oracle import metrics


def test_rel_l2_and_max_scaled_by_hand():
    # a = (1, i, -1, 0): ||a|| = sqrt(3), rms(a) = sqrt(3) / sqrt(4) = sqrt(3) / 2
    # b - a = (0.1, 0, 0, 0.2i): ||b - a|| = sqrt(0.01 + 0.04) = sqrt(0.05)
    # rel_l2 = sqrt(0.05 / 3); max_scaled = 0.2 / (sqrt(3) / 2) = 0.4 / sqrt(3)
    a = np.array([1, 1j, -1, 0])
    b = a + np.array([0.1, 0, 0, 0.2j])
    r = metrics.compare(a, b, 2)
    assert r["rel_l2"] == pytest.approx(math.sqrt(0.05 / 3), rel=1e-14)
    assert r["max_scaled"] == pytest.approx(0.4 / math.sqrt(3), rel=1e-14)
    # the reference is the first argument: normalising by ||b|| = sqrt(3.25)
    # instead would give sqrt(0.05 / 3.25)
    s = metrics.compare(b, a, 2)
    assert s["rel_l2"] == pytest.approx(math.sqrt(0.05 / 3.25), rel=1e-14)
    assert s["rel_l2"] != pytest.approx(r["rel_l2"], rel=1e-3)


def test_rel_l2_zero_for_equal_sets():
    a = np.exp(1j * np.arange(7.0)) * np.arange(1, 8)
    r = metrics.compare(a, a.copy(), 3)
    assert r["rel_l2"] == 0.0 and r["max_scaled"] == 0.0
    assert r["f_ovl"] == pytest.approx(1.0, abs=1e-15)


def test_per_amplitude_relative_error_by_hand():
    # |b_i - a_i| / |a_i| = (0.1, 0, 0, 0); sorted (0, 0, 0, 0.1): median 0,
    # the 0.99 quantile interpolates at position 0.99 * 3 = 2.97 -> 0.097
    a = np.array([1.0, 2.0, 4.0, 8.0])
    b = np.array([1.1, 2.0, 4.0, 8.0])
    r = metrics.compare(a, b, 2)
    assert r["rel_median"] == 0.0
    assert r["rel_p99"] == pytest.approx(0.097, rel=1e-12)


def test_f_ovl_global_phase_and_rotation():
    a = np.array([0.6, 0.8j, 0.0])
    for theta in (0.3, 1.7, -2.9):
        assert metrics.compare(a, np.exp(1j * theta) * a, 2)["f_ovl"] == pytest.approx(1.0, abs=1e-14)
    # real rotation by phi in a plane: |<a, b>|^2 = cos^2(phi)
    for phi in (0.2, 0.7, 1.3):
        a2 = np.array([1.0, 0.0])
        b2 = np.array([math.cos(phi), math.sin(phi)])
        assert metrics.compare(a2, b2, 1)["f_ovl"] == pytest.approx(math.cos(phi) ** 2, rel=1e-14)
    # the conjugate matters: a = b = (1, i) gives sum conj(a) b = 2 -> 1;
    # without the conjugate the sum would be 1 + i*i = 0
    c = np.array([1.0, 1j])
    assert metrics.compare(c, c, 1)["f_ovl"] == pytest.approx(1.0, abs=1e-15)
    # scale invariance: |<a, 3b>|^2 / (|a|^2 |3b|^2) is unchanged
    assert metrics.compare(a, 3 * np.exp(0.4j) * a, 2)["f_ovl"] == pytest.approx(1.0, abs=1e-14)


def test_f_xeb_by_hand():
    # N = 2 (2^N = 4).  Reference probabilities p = (1/2, 1/4, 1/4, 0):
    # P = 2^N p = (2, 1, 1, 0), mean(P^2) = 6/4 = 1.5, denominator 0.5.
    a = np.sqrt([0.5, 0.25, 0.25, 0.0]) * np.exp(1j * np.array([0.1, 2.0, -1.0, 0.5]))
    # tested = reference: F = (1.5 - 1) / 0.5 = 1
    assert metrics.compare(a, a, 2)["f_xeb"] == pytest.approx(1.0, rel=1e-14)
    # uniform tested q: Q = (1, 1, 1, 1), mean(PQ) = 1 -> F = 0
    u = np.full(4, 0.5 + 0j)
    assert metrics.compare(a, u, 2)["f_xeb"] == pytest.approx(0.0, abs=1e-14)
    # q = (3/8, 1/4, 1/4, 1/8): Q = (1.5, 1, 1, 0.5), mean(PQ) = (3 + 1 + 1 + 0) / 4
    # = 1.25 -> F = 0.25 / 0.5 = 0.5.  (Normalising by mean(Q^2) = 1.125
    # instead would give 2; a 2^(N-1) factor would give a negative value.)
    q = np.sqrt([3 / 8, 1 / 4, 1 / 4, 1 / 8]) * np.exp(1j * np.array([1.0, 0.0, 3.0, -2.0]))
    assert metrics.compare(a, q, 2)["f_xeb"] == pytest.approx(0.5, rel=1e-13)
    # phases do not enter F_xeb
    assert metrics.compare(a, q * np.exp(0.9j), 2)["f_xeb"] == pytest.approx(0.5, rel=1e-13)


def test_f_xeb_undefined_for_flat_reference():
    # mean(P^2) = 1 exactly: F_xeb has no defined value and is reported as NaN
    u = np.full(4, 0.5 + 0j)
    assert math.isnan(metrics.compare(u, u, 2)["f_xeb"])
