"""Pins of the frugal-sampling reference (oracle/sampling.py) against its
closed forms and against exact distributions from the state vector."""

import numpy as np
import pytest

from circuits import grid, random_circuit
from oracle import sampling, sv


def test_batch_enumeration_order():
    # N = 3, open qubits [2, 0] (qubit 2 is the most significant bit of x)
    c = sampling.batch_bitstrings([[1, 1, 0]], [2, 0])
    assert c.shape == (1, 4, 3)
    assert c[0].tolist() == [[0, 1, 0], [1, 1, 0], [0, 1, 1], [1, 1, 1]]


def test_acceptance_probability_closed_form():
    # a candidate with 2^N p / M = a is accepted with probability min(1, a)
    rng = np.random.default_rng(3)
    n, m = 4, 5.0
    for a in (0.0, 0.1, 0.37, 0.9, 1.0, 2.5):
        p = np.full(200000, a * m / 2 ** n)
        rate = sampling.frugal_accept(p, rng.random(p.size), n, m).mean()
        expect = min(1.0, a)
        assert abs(rate - expect) < 5 * np.sqrt(max(expect * (1 - expect), 1e-12) / p.size) + 1e-12


def test_accepted_distribution_is_p():
    # every candidate of a 10-qubit random circuit drawn R times; with M
    # bounding 2^N p the accepted counts follow p and the rate is 1/M
    c = random_circuit(grid(2, 5), 8, 21)
    n = c.n
    allbits = ((np.arange(2 ** n)[:, None] >> np.arange(n - 1, -1, -1)) & 1).astype(np.uint8)
    p = np.abs(sv.amplitudes(c, allbits)) ** 2
    m = 1.01 * 2 ** n * p.max()
    rng = np.random.default_rng(5)
    reps = 400
    counts = np.zeros(2 ** n)
    for _ in range(reps):
        counts += sampling.frugal_accept(p, rng.random(2 ** n), n, m)
    total = counts.sum()
    assert abs(total / (reps * 2 ** n) - 1 / m) < 5 * np.sqrt((1 / m) / (reps * 2 ** n))
    # total variation between the accepted histogram and p
    tv = 0.5 * np.abs(counts / total - p).sum()
    assert tv < 0.05, tv
    # a wrong rule (accepting with probability p, not 2^N p / M) is far from p
    wrong = np.zeros(2 ** n)
    for _ in range(reps):
        wrong += p * 2 ** n / m > 0.5
    assert 0.5 * np.abs(wrong / wrong.sum() - p).sum() > 2 * tv
