"""Pins of the path-score brute force and the fidelity closed form."""

import math

import numpy as np
import pytest

from oracle import fidelity, paths
from circuits import diagonal53, grid, random_circuit


def test_chain_by_hand():
    # 3-site chain 0 -(a=2)- 1 -(b=3)- 2.
    # order 0,1,2: Cost({0},1) = a*b = 6, then Cost({0,1},2) = b = 3 -> 9
    # order 1,0,2: Cost({1},0) = a*b = 6, Cost({0,1},2) = 3 -> 9
    # order 0,2,1: Cost({0},2) = a*b = 6 (no shared leg), Cost({0,2},1) = 6 -> 12
    # order 2,1,0: Cost({2},1) = a*b = 6, Cost({1,2},0) = a = 2 -> 8 (optimal)
    edges, dims = [(0, 1), (1, 2)], [2, 3]
    assert paths.score([0, 1, 2], 3, edges, dims)[0] == 9
    assert paths.score([0, 2, 1], 3, edges, dims)[0] == 12
    assert paths.score([2, 1, 0], 3, edges, dims)[0] == 8
    assert paths.brute_force(3, edges, dims)[0] == 8  # also reached by 1,2,0


def test_triangle_by_hand():
    # triangle with dims 2 (0-1), 4 (1-2), 8 (0-2): every order costs
    # Cost(first pair) = product of all three dims = 64, then the remaining two
    # open legs meet the last site: their product.
    edges, dims = [(0, 1), (1, 2), (0, 2)], [2, 4, 8]
    s, _ = paths.score([0, 1, 2], 3, edges, dims)
    assert s == 64 + 4 * 8
    assert paths.brute_force(3, edges, dims)[0] == 64 + 2 * 4


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_equals_subset_dp(seed):
    rng = np.random.default_rng(seed)
    n = 7
    edges = set()
    for q in range(1, n):  # spanning tree + extra edges
        edges.add((int(rng.integers(q)), q))
    while len(edges) < n + 3:
        a, b = sorted(rng.choice(n, 2, replace=False))
        edges.add((int(a), int(b)))
    edges = sorted(edges)
    dims = [int(2 ** rng.integers(1, 4)) for _ in edges]
    assert paths.brute_force(n, edges, dims)[0] == paths.subset_dp(n, edges, dims)


def test_bridge_by_hand():
    # two heavy pairs joined by a thin bond: A -(8)- B -(2)- C -(8)- D.
    # Linear A,B,C,D: Cost(A,B) = 8*2 = 16, Cost({A,B},C) = 2*8 = 16,
    # Cost({A,B,C},D) = 8 -> 40, and no linear order does better.  With C,D
    # as a side branch (window of positions 2..3): the branch costs
    # Cost(C,D) = 2*8 = 16, the main path Cost(A,B) = 16, and absorbing the
    # branch's tensor (only the thin bond left) costs 2 -> 34, which is also
    # the best of every contraction tree.
    edges, dims = [(0, 1), (1, 2), (2, 3)], [8, 2, 8]
    assert paths.score([0, 1, 2, 3], 4, edges, dims)[0] == 40
    assert paths.subset_dp(4, edges, dims) == 40
    s, peak, bpeak = paths.tree_score([0, 1, 2, 3], [(2, 4)], 4, edges, dims)
    assert (s, peak, bpeak) == (34, 8, 16)
    assert paths.tree_optimum(4, edges, dims) == 34


def test_tree_optimum_by_hand():
    # the 3-site chain above: pairing (1,2) first costs a*b = 6, then the
    # remaining leg a = 2 -> 8, the same as the best linear order
    assert paths.tree_optimum(3, [(0, 1), (1, 2)], [2, 3]) == 8
    # triangle: every tree pairs two sites first (64) and then meets the
    # third site through its two legs; the cheapest pair leaves 2 * 4
    assert paths.tree_optimum(3, [(0, 1), (1, 2), (0, 2)], [2, 4, 8]) == 64 + 8


@pytest.mark.parametrize("seed", range(4))
def test_tree_score_without_windows_is_linear(seed):
    rng = np.random.default_rng(seed)
    g = grid(3, 3)
    dims = [int(2 ** rng.integers(1, 4)) for _ in g.edges]
    order = [int(x) for x in rng.permutation(g.n)]
    s, peak = paths.score(order, g.n, g.edges, dims)
    assert paths.tree_score(order, [], g.n, g.edges, dims)[:2] == (s, peak)
    # a tree contraction can only do as well as or better than linear paths
    assert paths.tree_optimum(g.n, g.edges, dims) <= paths.subset_dp(g.n, g.edges, dims)


def test_bounded_brute_force_by_hand():
    # the 3-site chain 0 -(a=2)- 1 -(b=3)- 2: orders, (score, largest tensor):
    # 2,1,0 -> (8, 3): tensors {b}=3, {a}=2, scalar;  1,2,0 -> (8, 6);
    # 0,1,2 -> (9, 3); 1,0,2 -> (9, 6); 0,2,1 -> (12, 6); 2,0,1 -> (12, 6).
    # A bound of 3 elements keeps 2,1,0 and 0,1,2; a bound of 2 keeps none
    # (only site 0 starts within it, and its next tensor has 3 or 6 elements).
    edges, dims = [(0, 1), (1, 2)], [2, 3]
    assert paths.brute_force_bounded(3, edges, dims, 6)[0] == 8
    assert paths.brute_force_bounded(3, edges, dims, 3) == (8, [2, 1, 0])
    assert paths.brute_force_bounded(3, edges, dims, 2) == (None, None)


def test_intermediate_size_tracks_open_legs():
    g = grid(2, 3)
    dims = [2] * len(g.edges)
    _, big = paths.score([0, 1, 2, 3, 4, 5], g.n, g.edges, dims)
    # after {0,1,2} the open legs are the three verticals: 2^3
    assert big == 8


def test_fidelity_closed_form_53q():
    # 53-qubit diagonal lattice, 12 cycles ABCDCDAB, no final layer:
    # 636 single-qubit gates, 258 fSim gates.
    c = random_circuit(diagonal53(), 12, 3, final_layer=False)
    n1, n2 = c.count()
    assert (n1, n2) == (636, 258)
    f = fidelity.fidelity(n1, n2, 53)
    assert abs(f - 9.314e-3) < 5e-6
    assert abs(fidelity.n_samples(f) / 1.0375e5 - 1) < 2e-3


def test_fidelity_closed_form_with_final_layer():
    c = random_circuit(diagonal53(), 12, 3)
    n1, n2 = c.count()
    assert (n1, n2) == (689, 258)
    f = fidelity.fidelity(n1, n2, 53)
    assert abs(f - 8.556e-3) < 5e-6


def test_fidelity_small_grid():
    c = random_circuit(grid(3, 4), 8, 1, final_layer=False)
    n1, n2 = c.count()
    assert (n1, n2) == (96, 34)
    assert abs(fidelity.fidelity(n1, n2, 12) - 0.436) < 5e-4


def test_fidelity_limits():
    assert fidelity.fidelity(0, 0, 0) == 1.0
    assert fidelity.n_samples(1.0) == 9.0
    # one two-qubit gate only
    assert fidelity.fidelity(0, 1, 0) == pytest.approx(1 - 0.0062)
    assert fidelity.fidelity(0, 0, 1) == pytest.approx(1 - 0.038)
