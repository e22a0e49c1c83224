"""Explicit gate matrices of the random-circuit gate set.

The paper takes its gate set from the Sycamore experiment without writing the
matrices down; these are the usual definitions.  Matrices are row-major with
rows indexing the output basis state.  Two-qubit gates use basis index
2*b(q0) + b(q1).
"""

import numpy as np

_S = 1.0 / np.sqrt(2.0)

SQRT_X = _S * np.array([[1, -1j], [-1j, 1]], dtype=np.complex128)
SQRT_Y = _S * np.array([[1, -1], [1, 1]], dtype=np.complex128)
SQRT_W = _S * np.array([[1, -np.exp(1j * np.pi / 4)],
                        [np.exp(-1j * np.pi / 4), 1]], dtype=np.complex128)

SINGLE_QUBIT = {"sqrtX": SQRT_X, "sqrtY": SQRT_Y, "sqrtW": SQRT_W}

CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)


def fsim(theta: float, phi: float) -> np.ndarray:
    """fSim(theta, phi): partial iSWAP by theta plus a controlled phase phi."""
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[1, 0, 0, 0],
                     [0, c, -1j * s, 0],
                     [0, -1j * s, c, 0],
                     [0, 0, 0, np.exp(-1j * phi)]], dtype=np.complex128)
