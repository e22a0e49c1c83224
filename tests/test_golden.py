"""Pins against numbers the paper prints (tests/golden/paper_values.txt).

The fixture holds only printed values, each with its passage; the checks
below compare the oracle's fidelity model and the library's host planner with
them, so that a mistyped rate or a wrong bond rule fails here and not only by
comparison of one implementation with the other."""

import os

import numpy as np
import pytest

import paper_2011_02621_amd as T
from circuits import CZ, fsim, config
from circuits.rqc import Circuit, Gate
from oracle import fidelity

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_values.txt")


def _paper_values():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, value = line.split()[:2]
            vals[name] = float(value)
    return vals


PV = _paper_values()


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(-1)
    yield c
    c.close()


def test_fixture_has_every_value():
    assert set(PV) == {"e1", "e2", "eq", "sigma_count", "chi_controlled", "chi_iswap",
                       "chi_fsim", "first_bond_chi4"}


def test_oracle_error_rates_are_the_papers():
    # each rate alone: one gate of one kind, or one qubit read out
    assert fidelity.fidelity(1, 0, 0) == pytest.approx(1 - PV["e1"], abs=0)
    assert fidelity.fidelity(0, 1, 0) == pytest.approx(1 - PV["e2"], abs=0)
    assert fidelity.fidelity(0, 0, 1) == pytest.approx(1 - PV["eq"], abs=0)
    # the three-sigma count
    for f in (0.5, 1e-2, 2e-3):
        assert fidelity.n_samples(f) == pytest.approx((PV["sigma_count"] / f) ** 2, rel=1e-15)


def test_library_fidelity_uses_the_papers_rates(ctx):
    # the planner's Eq. (9) figure with the printed rates, gate counts taken
    # from the circuit itself
    for name, final in (("diag53_d12", False), ("diag53_d12", True), ("grid3x4_d8", True)):
        c, _ = config(name, final_layer=final)
        n1, n2 = c.count()
        want = (1 - PV["e1"]) ** n1 * (1 - PV["e2"]) ** n2 * (1 - PV["eq"]) ** c.n
        i = ctx.plan(c, split_cycle=1, path_mode="greedy", max_intermediate_elems=1 << 60).info()
        assert i.fidelity == pytest.approx(want, rel=1e-12)
        assert i.n_samples == pytest.approx((PV["sigma_count"] / want) ** 2, rel=1e-12)


def _cphase(phi):
    return np.diag([1, 1, 1, np.exp(1j * phi)])


CNOT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], complex)
ISWAP = np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]], complex)


@pytest.mark.parametrize("gate,key", [
    (CZ, "chi_controlled"), (CNOT, "chi_controlled"), (_cphase(0.7), "chi_controlled"),
    (ISWAP, "chi_iswap"), (fsim(np.pi / 2, np.pi / 6), "chi_fsim"), (fsim(0.3, 1.1), "chi_fsim"),
])
def test_gate_bond_is_the_printed_rank(ctx, gate, key):
    # chain 0-1-2-3: CZ on (0,1) and (2,3) first gives qubits 1 and 2 one
    # outer bond of 2 each, so the compression bound 2 * 2 = 4 on the middle
    # bond no longer hides the gate's own rank: the middle bond is chi_o.
    edges = [(0, 1), (1, 2), (2, 3)]
    gates = [Gate(0, 1, 0, CZ), Gate(2, 3, 0, CZ), Gate(1, 2, 0, np.asarray(gate, complex))]
    i = ctx.plan(Circuit(4, edges, gates, 1), split_cycle=1).info()
    assert list(i.bond_ket) == [2, int(PV[key]), 2]


def test_first_chi4_gate_leaves_the_printed_bond(ctx):
    for g in (ISWAP, fsim(np.pi / 2, np.pi / 6)):
        c = Circuit(2, [(0, 1)], [Gate(0, 1, 0, g)], 1)
        assert list(ctx.plan(c, split_cycle=1).info().bond_ket) == [int(PV["first_bond_chi4"])]


def _operator_schmidt(g):
    # O[(a b), (a' b')] regrouped as M[(a a'), (b b')]; its singular values
    # are the operator Schmidt coefficients of the split O = sum_s P_s (x) Q_s
    o = np.asarray(g, complex).reshape(2, 2, 2, 2)      # a, b, a', b'
    m = o.transpose(0, 2, 1, 3).reshape(4, 4)
    return np.linalg.svd(m, compute_uv=False)


@pytest.mark.parametrize("gate,key,sigma", [
    (CZ, "chi_controlled", [np.sqrt(2), np.sqrt(2), 0, 0]),
    (CNOT, "chi_controlled", [np.sqrt(2), np.sqrt(2), 0, 0]),
    (ISWAP, "chi_iswap", [1, 1, 1, 1]),
    (fsim(np.pi / 2, np.pi / 6), "chi_fsim", [1, 1, 1, 1]),
])
def test_generator_gates_have_the_printed_split_rank(gate, key, sigma):
    # the circuit generator's matrices split with the rank the paper prints;
    # the coefficients' squares add up to the Frobenius norm squared, 4
    s = _operator_schmidt(gate)
    assert int((s > 1e-12).sum()) == int(PV[key])
    assert np.allclose(s, sigma, atol=1e-12)
    assert np.isclose((s ** 2).sum(), 4.0, atol=1e-12)
