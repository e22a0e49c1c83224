"""Qubit lattices (graphs G = {V, E}) and their coupler patterns.

A lattice is the connected graph of the paper's "State initialization" section:
one node per qubit and one edge per coupled pair.  Each coupler pattern is a
matching (no qubit appears twice), so all gates of one pattern commute and form
one layer.
"""

from dataclasses import dataclass, field
from typing import Dict, List, Tuple


@dataclass
class Lattice:
    name: str
    n: int
    edges: List[Tuple[int, int]]            # (u, v), u < v, sorted
    patterns: Dict[str, List[int]]          # pattern name -> edge ids
    sequence: str                           # pattern order per cycle, e.g. "ABCD"
    coords: List[Tuple[int, int]] = field(default_factory=list)

    def degree(self) -> List[int]:
        deg = [0] * self.n
        for u, v in self.edges:
            deg[u] += 1
            deg[v] += 1
        return deg

    def pattern_for_cycle(self, c: int) -> List[int]:
        return self.patterns[self.sequence[c % len(self.sequence)]]

    def sub(self, keep: int, name: str = None) -> "Lattice":
        """The induced sub-lattice on the first ``keep`` qubits."""
        remap = {q: q for q in range(keep)}
        edges, old_to_new = [], {}
        for eid, (u, v) in enumerate(self.edges):
            if u < keep and v < keep:
                old_to_new[eid] = len(edges)
                edges.append((u, v))
        pats = {k: [old_to_new[e] for e in es if e in old_to_new]
                for k, es in self.patterns.items()}
        del remap
        return Lattice(name or f"{self.name}[:{keep}]", keep, edges, pats,
                       self.sequence, self.coords[:keep])


def grid(rows: int, cols: int) -> Lattice:
    """rows x cols square grid; qubit (r, c) has index r*cols + c.

    Patterns: A = horizontal couplers (r,c)-(r,c+1) with c even, B = the same
    with c odd, C = vertical couplers (r,c)-(r+1,c) with r even, D = the same
    with r odd.  Cycle order ABCD.
    """
    idx = lambda r, c: r * cols + c
    raw = []  # (u, v, pattern)
    for r in range(rows):
        for c in range(cols - 1):
            raw.append((idx(r, c), idx(r, c + 1), "A" if c % 2 == 0 else "B"))
    for r in range(rows - 1):
        for c in range(cols):
            raw.append((idx(r, c), idx(r + 1, c), "C" if r % 2 == 0 else "D"))
    raw.sort()
    edges = [(u, v) for u, v, _ in raw]
    pats = {k: [i for i, e in enumerate(raw) if e[2] == k] for k in "ABCD"}
    coords = [(r, c) for r in range(rows) for c in range(cols)]
    return Lattice(f"grid{rows}x{cols}", rows * cols, edges, pats, "ABCD", coords)


def diagonal_sites():
    """The 54 sites (x, y) of a diagonal (rotated square) lattice with 9 rows.

    Row y holds x in {y mod 2 + 2j : j = 0..5}; sites are coupled along the two
    diagonals (x, y)-(x +- 1, y + 1).
    """
    return [(y % 2 + 2 * j, y) for y in range(9) for j in range(6)]


def diagonal53() -> Lattice:
    """53-qubit diagonal lattice: the 54-site lattice with site (10, 0) removed.

    Couplers (x, y)-(x+1, y+1) form pattern A when y is even and B when y is
    odd; couplers (x, y)-(x-1, y+1) form C (y even) and D (y odd).  Cycle order
    ABCDCDAB.  Qubits are numbered by row, then by x.
    """
    sites = [s for s in diagonal_sites() if s != (10, 0)]
    sites.sort(key=lambda s: (s[1], s[0]))
    index = {s: i for i, s in enumerate(sites)}
    raw = []
    for (x, y) in sites:
        for dx, even, odd in ((+1, "A", "B"), (-1, "C", "D")):
            t = (x + dx, y + 1)
            if t in index:
                u, v = index[(x, y)], index[t]
                raw.append((min(u, v), max(u, v), even if y % 2 == 0 else odd))
    raw.sort()
    edges = [(u, v) for u, v, _ in raw]
    pats = {k: [i for i, e in enumerate(raw) if e[2] == k] for k in "ABCD"}
    return Lattice("diag53", len(sites), edges, pats, "ABCDCDAB", sites)
