"""Frugal rejection sampling, plain reference (test infrastructure).

Published method (frugal rejection sampling of the random-circuit sampling
literature): a uniformly drawn candidate bitstring s with probability
p(s) = |<s|U|0>|^2 is accepted when 2^N p(s) / M > u for a uniform u in
[0, 1), i.e. with probability min(1, 2^N p(s) / M).  If M bounds 2^N p on
every candidate, accepted bitstrings are distributed as p, and the overall
acceptance rate is 1 / M.  The paper names the simulation of measurements
(sampling) as an advantage of the tensor-network-state representation
(introduction); correlated batches give the 2^k amplitudes of the
candidates that share N - k fixed bits in one contraction.

Only tests, smoke() and the bench's CPU leg use this module.
"""

import numpy as np


def frugal_accept(probs, uniforms, n_qubits: int, m_bound: float) -> np.ndarray:
    """Accept flags, in FP64: 2^N p / M > u."""
    p = np.asarray(probs, np.float64)
    u = np.asarray(uniforms, np.float64)
    return p * (2.0 ** n_qubits / m_bound) > u


def batch_bitstrings(fixed_bits, open_qubits) -> np.ndarray:
    """The 2^k candidates of each batch, [n][2^k][N]: the fixed bits with the
    open qubits set from x, the first open qubit the most significant bit."""
    fixed = np.asarray(fixed_bits, np.uint8)
    fixed = fixed.reshape(-1, fixed.shape[-1])
    k = len(open_qubits)
    out = np.repeat(fixed[:, None, :], 1 << k, axis=1).copy()
    for x in range(1 << k):
        for i, q in enumerate(open_qubits):
            out[:, x, q] = (x >> (k - 1 - i)) & 1
    return out
