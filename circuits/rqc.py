"""Seeded random quantum circuits (RQCs), mirror circuits and bitstrings.

A cycle is one layer of single-qubit gates on every qubit followed by fSim on
every coupler of that cycle's pattern.  Depth d is the number of cycles, as in
the paper.  By default a final single-qubit layer closes the circuit (the usual
RQC shape; without it the last fSim layer meets a computational-basis bra
directly and the bra side of the network is artificially easy).

Single-qubit choice: cycle 0 draws uniformly from {sqrtX, sqrtY, sqrtW}; every
later layer draws uniformly from the two gates that differ from the qubit's
previous one.  Draws use numpy's PCG64 ``default_rng(seed)`` in qubit order
within a layer.
"""

from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .gates import SQRT_X, SQRT_Y, SQRT_W, fsim
from .lattice import Lattice, grid, diagonal53

_ORDER = [("sqrtX", SQRT_X), ("sqrtY", SQRT_Y), ("sqrtW", SQRT_W)]


@dataclass
class Gate:
    q0: int
    q1: int          # -1 for a single-qubit gate
    cycle: int
    matrix: np.ndarray
    name: str = ""


@dataclass
class Circuit:
    n: int
    edges: List[tuple]
    gates: List[Gate]
    depth: int
    name: str = ""

    # flat views for the C ABI and the oracle ------------------------------
    def edge_array(self) -> np.ndarray:
        return np.ascontiguousarray(np.array(self.edges, dtype=np.int32).reshape(-1, 2))

    def gate_arrays(self):
        """(q0, q1, cycle, mats): mats[g] holds the row-major complex matrix as
        interleaved (re, im) doubles, 2x2 in the first 8 entries or 4x4 in 32."""
        g = len(self.gates)
        q0 = np.empty(g, np.int32)
        q1 = np.empty(g, np.int32)
        cy = np.empty(g, np.int32)
        mats = np.zeros((g, 32), np.float64)
        for i, gt in enumerate(self.gates):
            q0[i], q1[i], cy[i] = gt.q0, gt.q1, gt.cycle
            flat = np.asarray(gt.matrix, np.complex128).reshape(-1)
            mats[i, 0:2 * flat.size:2] = flat.real
            mats[i, 1:2 * flat.size:2] = flat.imag
        return q0, q1, cy, mats

    def count(self):
        n1 = sum(1 for g in self.gates if g.q1 < 0)
        return n1, len(self.gates) - n1


def random_circuit(lat: Lattice, depth: int, seed: int, theta: float = np.pi / 2,
                   phi: float = np.pi / 6, final_layer: bool = True,
                   clifford: bool = False) -> Circuit:
    """Random circuit on ``lat``.  ``clifford=True`` draws single-qubit gates
    from {sqrtX, sqrtY} (repeats allowed) and uses fSim(pi/2, 0), which keeps
    the whole circuit Clifford."""
    rng = np.random.default_rng(seed)
    two_q = fsim(np.pi / 2, 0.0) if clifford else fsim(theta, phi)
    prev = [-1] * lat.n
    gates: List[Gate] = []

    def one_qubit_layer(cycle):
        for q in range(lat.n):
            if clifford:
                k = int(rng.integers(2))
            elif prev[q] < 0:
                k = int(rng.integers(3))
            else:
                others = [i for i in range(3) if i != prev[q]]
                k = others[int(rng.integers(2))]
            prev[q] = k
            name, m = _ORDER[k]
            gates.append(Gate(q, -1, cycle, m.copy(), name))

    for c in range(depth):
        one_qubit_layer(c)
        for eid in lat.pattern_for_cycle(c):
            u, v = lat.edges[eid]
            gates.append(Gate(u, v, c, two_q.copy(), "fsim"))
    if final_layer:
        one_qubit_layer(depth)
    return Circuit(lat.n, list(lat.edges), gates, depth + (1 if final_layer else 0),
                   f"{lat.name}_d{depth}_s{seed}{'_clifford' if clifford else ''}")


def mirror_circuit(lat: Lattice, half_depth: int, seed: int, clifford: bool = False) -> Circuit:
    """W = U^-1 U with U a random circuit of ``half_depth`` cycles (no final
    layer).  Cycles of the inverse half are numbered half_depth..2*half_depth-1,
    so splitting the two-sided evolution at ``half_depth`` puts U on the ket
    side and U^-1 on the bra side.  <0|W|0> = 1 and every other amplitude is 0.
    """
    u = random_circuit(lat, half_depth, seed, final_layer=False, clifford=clifford)
    inv = []
    for g in reversed(u.gates):
        inv.append(Gate(g.q0, g.q1, 2 * half_depth - 1 - g.cycle,
                        np.conj(g.matrix.T).copy(), g.name + "_dag"))
    return Circuit(lat.n, list(lat.edges), u.gates + inv, 2 * half_depth,
                   f"{lat.name}_mirror{half_depth}_s{seed}")


def bitstrings(n_qubits: int, count: int, seed: int) -> np.ndarray:
    """``count`` i.i.d. uniform bitstrings, uint8 [count, n_qubits]."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.integers(0, 2, size=(count, n_qubits), dtype=np.uint8))


_CONFIGS = {
    # name: (lattice factory, cycles, circuit seed, bitstring seed, bitstrings)
    "grid3x4_d8": (lambda: grid(3, 4), 8, 1, 101, 64),
    "grid5x5_d10": (lambda: grid(5, 5), 10, 2, 102, 1024),
    "diag53_d12": (diagonal53, 12, 3, 103, 4096),
    "grid8x13_d8": (lambda: grid(8, 13), 8, 5, 105, 256),
}


def config(name: str, final_layer: bool = True, n_bits: Optional[int] = None):
    """Named workload: returns (circuit, bitstrings)."""
    make, depth, cseed, bseed, nb = _CONFIGS[name]
    lat = make()
    circ = random_circuit(lat, depth, cseed, final_layer=final_layer)
    bits = bitstrings(lat.n, nb if n_bits is None else n_bits, bseed)
    return circ, bits
