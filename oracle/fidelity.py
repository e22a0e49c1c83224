"""Circuit-fidelity model and required bitstring count (oracle).

"Verification of RQCs" section, Eq. (9): F = prod over gates (1 - e_g) times
prod over qubits (1 - e_q), with the Sycamore error rates the paper quotes
(single-qubit gate 0.16 %, two-qubit gate 0.62 %, readout 3.8 %).  Resolving
F > 0 at three standard deviations with sigma = 1/sqrt(N_s) needs
N_s >= (3 / F)^2.
"""

E1, E2, EQ = 0.0016, 0.0062, 0.038


def fidelity(n1: int, n2: int, n_qubits: int, e1: float = E1, e2: float = E2,
             eq: float = EQ) -> float:
    f = 1.0
    for _ in range(n1):
        f *= 1.0 - e1
    for _ in range(n2):
        f *= 1.0 - e2
    for _ in range(n_qubits):
        f *= 1.0 - eq
    return f


def n_samples(f: float) -> float:
    return (3.0 / f) ** 2
