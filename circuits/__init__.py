"""Seeded synthetic random-quantum-circuit inputs.

This package only *describes* circuits: lattices, coupler patterns, explicit
gate matrices, seeded gate choices and bitstrings.  It contains none of the
amplitude method's arithmetic, so both the CPU oracle (``oracle/``) and the GPU
library (``paper_2011_02621_amd``) can consume the same inputs without sharing
any computation.

The paper evaluates on Sycamore-like random circuits whose device layout and
gate files come from the cited Sycamore work and are not reproduced here.  The
lattices and patterns below are synthetic stand-ins of the same shape:
interleaved layers of single-qubit gates drawn from {sqrt(X), sqrt(Y),
sqrt(W)} and fSim(pi/2, pi/6) two-qubit gates on nearest-neighbour couplers,
applied pattern by pattern (the paper's "Verification of RQCs" section and the
gate set it takes from the Sycamore experiment).
"""

from .lattice import Lattice, grid, diagonal53, diagonal_sites
from .gates import SQRT_X, SQRT_Y, SQRT_W, fsim, CZ
from .rqc import Circuit, random_circuit, mirror_circuit, bitstrings, config

__all__ = [
    "Lattice", "grid", "diagonal53", "diagonal_sites",
    "SQRT_X", "SQRT_Y", "SQRT_W", "fsim", "CZ",
    "Circuit", "random_circuit", "mirror_circuit", "bitstrings", "config",
]
