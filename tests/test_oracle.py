"""Pins of the CPU oracle against facts outside the oracle itself.

Each check is chosen so that a plausible mistake in the oracle (a wrong bit
order, a transposed gate, a dropped phase, a wrong pairing of indices) fails:
closed-form gate identities, an independent Kronecker-product brute force,
textbook states (Bell, GHZ), norm conservation, mirror circuits, and the
stabilizer formalism on Clifford circuits.
"""

import itertools

import numpy as np
import pytest

from circuits import (SQRT_X, SQRT_Y, SQRT_W, CZ, fsim, grid, diagonal53, random_circuit,
                      mirror_circuit, bitstrings)
from circuits.rqc import Circuit, Gate
from oracle import dense, sv, stabilizer

X = np.array([[0, 1], [1, 0]], complex)
Y = np.array([[0, -1j], [1j, 0]], complex)
H = np.array([[1, 1], [1, -1]], complex) / np.sqrt(2)
CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], complex)


def all_bits(n):
    return np.array(list(itertools.product((0, 1), repeat=n)), np.uint8)


# --- gate set -------------------------------------------------------------

@pytest.mark.parametrize("g", [SQRT_X, SQRT_Y, SQRT_W, fsim(np.pi / 2, np.pi / 6),
                               fsim(np.pi / 2, 0.0), CZ])
def test_gates_unitary(g):
    assert np.abs(g.conj().T @ g - np.eye(g.shape[0])).max() < 1e-15


def test_sqrt_gates_square_to_paulis():
    w = (X + Y) / np.sqrt(2)
    assert np.allclose(SQRT_X @ SQRT_X, -1j * X, atol=1e-15)
    assert np.allclose(SQRT_Y @ SQRT_Y, -1j * Y, atol=1e-15)
    assert np.allclose(SQRT_W @ SQRT_W, -1j * w, atol=1e-15)


def test_fsim_limits():
    # fSim(0, 0) is the identity; fSim(pi/2, 0) swaps |01> and |10> with -i.
    assert np.allclose(fsim(0, 0), np.eye(4))
    f = fsim(np.pi / 2, 0)
    e01 = np.array([0, 1, 0, 0], complex)
    assert np.allclose(f @ e01, [0, 0, -1j, 0])


# --- state vector: textbook states ----------------------------------------

def _circ(n, gates):
    edges = sorted({(min(a, b), max(a, b)) for a, b, _ in gates if b >= 0})
    return Circuit(n, edges, [Gate(a, b, 0, np.asarray(m, complex)) for a, b, m in gates], 1)


def test_bell_state_bit_order():
    # H on qubit 0 then CNOT(control 0, target 1): (|00> + |11>)/sqrt(2)
    c = _circ(2, [(0, -1, H), (0, 1, CNOT)])
    psi = sv.state(c)
    assert np.allclose(psi, [1 / np.sqrt(2), 0, 0, 1 / np.sqrt(2)], atol=1e-15)


def test_single_flip_sets_leading_bit():
    # X on qubit 0 of 3: amplitude 1 at bitstring 100, dense index 4 = 2^(N-1-0)
    c = _circ(3, [(0, -1, X)])
    psi = sv.state(c)
    assert psi[4] == 1 and np.count_nonzero(psi) == 1
    assert sv.amplitudes(c, np.array([[1, 0, 0]], np.uint8))[0] == 1


def test_controlled_gate_orientation():
    # CNOT with q0 = 2 (control) and q1 = 0 (target), after X on qubit 2:
    # |001> -> |101>
    c = _circ(3, [(2, -1, X), (2, 0, CNOT)])
    amp = sv.amplitudes(c, np.array([[1, 0, 1]], np.uint8))[0]
    assert abs(amp - 1) < 1e-15


@pytest.mark.parametrize("n", [3, 6, 12])
def test_ghz(n):
    gates = [(0, -1, H)] + [(q, q + 1, CNOT) for q in range(n - 1)]
    c = _circ(n, gates)
    a = sv.amplitudes(c, np.array([[0] * n, [1] * n, [1] + [0] * (n - 1)], np.uint8))
    assert np.allclose(a, [2 ** -0.5, 2 ** -0.5, 0], atol=1e-15)


# --- state vector vs Kronecker brute force ---------------------------------

@pytest.mark.parametrize("rows,cols,depth,seed", [(2, 2, 4, 11), (2, 3, 5, 12), (3, 3, 4, 13),
                                                   (2, 4, 6, 14)])
def test_sv_matches_dense(rows, cols, depth, seed):
    c = random_circuit(grid(rows, cols), depth, seed)
    a = sv.state(c)
    b = dense.state(c)
    assert np.abs(a - b).max() < 1e-13


def test_sv_matches_dense_arbitrary_pairs():
    # random pairs in both orientations, non-adjacent, random unitaries
    rng = np.random.default_rng(7)
    n = 6
    gates = []
    for _ in range(25):
        if rng.random() < 0.4:
            q = int(rng.integers(n))
            m = np.linalg.qr(rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2)))[0]
            gates.append((q, -1, m))
        else:
            a, b = rng.choice(n, 2, replace=False)
            m = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))[0]
            gates.append((int(a), int(b), m))
    c = _circ(n, gates)
    assert np.abs(sv.state(c) - dense.state(c)).max() < 1e-13


@pytest.mark.parametrize("n_rows,n_cols,depth", [(3, 4, 8), (4, 4, 10)])
def test_norm_conserved(n_rows, n_cols, depth):
    c = random_circuit(grid(n_rows, n_cols), depth, 3)
    psi = sv.state(c)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-12


def test_gather_matches_index():
    c = random_circuit(grid(3, 4), 8, 1)
    psi = sv.state(c)
    bits = bitstrings(12, 20, 101)
    a = sv.amplitudes_from_state(12, psi, bits)
    for b, amp in zip(bits, a):
        assert amp == psi[sv.index_of(b)]


@pytest.mark.parametrize("half", [2, 4])
def test_mirror_circuit(half):
    c = mirror_circuit(grid(3, 4), half, 21)
    psi = sv.state(c)
    assert abs(psi[0] - 1) < 1e-13
    assert np.abs(psi[1:]).max() < 1e-13


# --- stabilizer tableau ---------------------------------------------------

def test_tableau_ghz():
    n = 5
    c = _circ(n, [(0, -1, H)] + [(q, q + 1, CNOT) for q in range(n - 1)])
    p = stabilizer.probabilities(c, all_bits(n))
    expect = np.zeros(2 ** n)
    expect[0] = expect[-1] = 0.5
    assert np.array_equal(p, expect)


def test_tableau_rejects_non_clifford():
    c = _circ(2, [(0, -1, SQRT_W)])
    with pytest.raises(ValueError):
        stabilizer.probabilities(c, all_bits(2))


@pytest.mark.parametrize("rows,cols,depth,seed", [(2, 3, 6, 31), (3, 4, 8, 32), (3, 4, 5, 33)])
def test_tableau_matches_state_vector(rows, cols, depth, seed):
    c = random_circuit(grid(rows, cols), depth, seed, clifford=True)
    n = c.n
    bits = all_bits(n)
    p_tab = stabilizer.probabilities(c, bits)
    p_sv = np.abs(sv.amplitudes(c, bits)) ** 2
    assert np.abs(p_tab - p_sv).max() < 1e-12
    nz = p_tab[p_tab > 0]
    assert np.allclose(nz, nz[0]) and abs(p_tab.sum() - 1) < 1e-12


def test_tableau_scales_to_53_qubits():
    c = random_circuit(diagonal53(), 8, 5, clifford=True)
    bits = bitstrings(53, 16, 9)
    p = stabilizer.probabilities(c, bits)
    nz = p[p > 0]
    # every nonzero probability is the same power of two
    if nz.size:
        assert np.allclose(nz, nz[0])
        assert float(np.log2(nz[0])).is_integer()


@pytest.mark.parametrize("rows,cols,depth,seed", [(3, 4, 8, 32), (3, 4, 5, 33), (2, 4, 6, 34)])
def test_support_sample_against_state_vector(rows, cols, depth, seed):
    # the sampler draws from the set the dense state vector says is nonzero,
    # that set has 2^rank elements, and the samples cover it uniformly
    c = random_circuit(grid(rows, cols), depth, seed, clifford=True)
    n = c.n
    tab = stabilizer.run(c)
    rank, _ = tab.z_subgroup()
    p_sv = np.abs(sv.amplitudes(c, all_bits(n))) ** 2
    support = np.nonzero(p_sv > 1e-12)[0]
    assert len(support) == 2 ** rank
    s = stabilizer.support_sample(tab, 4000, 7)
    idx = s.astype(np.int64) @ (1 << np.arange(n - 1, -1, -1))
    assert np.all(p_sv[idx] > 1e-12)
    counts = np.bincount(idx, minlength=2 ** n)[support]
    if len(support) <= 64:
        # every element drawn, none wildly over-represented
        assert counts.min() > 0 and counts.max() < 6 * 4000 / len(support)


def test_support_sample_scales_to_104_qubits():
    c = random_circuit(grid(8, 13), 8, 15, clifford=True)
    tab = stabilizer.run(c)
    s = stabilizer.support_sample(tab, 8, 3)
    p = tab.probabilities(s)
    rank, _ = tab.z_subgroup()
    assert np.all(p == 2.0 ** -rank)
