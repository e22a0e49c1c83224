"""Full-unitary brute force (oracle, test infrastructure), N <= 10.

Builds every gate as a 2^N x 2^N matrix from Kronecker products of 2x2
operators (|a'><a| on the gate's qubits, identity elsewhere), multiplies them in
time order and reads amp(s) = U[idx(s), 0].  This is an independent check of
the state-vector oracle: it uses no index arithmetic at all.
"""

from functools import reduce

import numpy as np

_I = np.eye(2, dtype=np.complex128)


def _unit(a_out: int, a_in: int) -> np.ndarray:
    m = np.zeros((2, 2), np.complex128)
    m[a_out, a_in] = 1.0
    return m


def gate_unitary(n: int, q0: int, q1: int, m: np.ndarray) -> np.ndarray:
    """2^N x 2^N matrix of one gate.  Qubit 0 is the most significant factor."""
    total = np.zeros((1 << n, 1 << n), np.complex128)
    if q1 < 0:
        for ao in range(2):
            for ai in range(2):
                if m[ao, ai] == 0:
                    continue
                ops = [_I] * n
                ops[q0] = _unit(ao, ai)
                total += m[ao, ai] * reduce(np.kron, ops)
        return total
    for r in range(4):
        for c in range(4):
            if m[r, c] == 0:
                continue
            ops = [_I] * n
            ops[q0] = _unit(r >> 1, c >> 1)
            ops[q1] = _unit(r & 1, c & 1)
            total += m[r, c] * reduce(np.kron, ops)
    return total


def circuit_unitary(circ) -> np.ndarray:
    n = circ.n
    if n > 10:
        raise ValueError("dense brute force is limited to N <= 10")
    u = np.eye(1 << n, dtype=np.complex128)
    for g in circ.gates:
        u = gate_unitary(n, g.q0, g.q1, np.asarray(g.matrix)) @ u
    return u


def state(circ) -> np.ndarray:
    return circuit_unitary(circ)[:, 0].copy()
