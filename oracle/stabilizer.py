"""Stabilizer-tableau oracle for Clifford circuits (test infrastructure).

Published method (Aaronson & Gottesman, "Improved simulation of stabilizer
circuits", 2004), written here from its definition rather than from any code:
the state U|0^N> is represented by N commuting Pauli generators, each
i^e * prod_q X^{x_q} Z^{z_q}.  Every Clifford gate conjugates the generators.
Its action on the local Paulis is read off the gate's explicit matrix, so the
oracle consumes exactly the gate list that the GPU library consumes.

Amplitude magnitudes follow from the Z-type subgroup of the stabilizer group:
if the generators reduce (by GF(2) elimination on their X parts) to rank r in
X and k = N - r pure Z-type elements +-Z^z, then |<s|psi>|^2 = 2^-r when every
Z-type element satisfies sign * (-1)^(z.s) = +1, and 0 otherwise.  This pins
the tensor-network amplitudes of Clifford variants of the random circuits at
sizes (53, 104 qubits) that no dense state vector reaches.
"""

import itertools

import numpy as np

_X = np.array([[0, 1], [1, 0]], np.complex128)
_Z = np.array([[1, 0], [0, -1]], np.complex128)
_I = np.eye(2, dtype=np.complex128)


def _local_pauli(bits):
    """bits = (x_a, z_a[, x_b, z_b]) -> matrix of X^x Z^z (x) ..."""
    mats = []
    for i in range(0, len(bits), 2):
        x, z = bits[i], bits[i + 1]
        mats.append((_X if x else _I) @ (_Z if z else _I))
    m = mats[0]
    for t in mats[1:]:
        m = np.kron(m, t)
    return m


def conjugation_table(u: np.ndarray):
    """For each local Pauli P (bit tuple) return (e, P') with U P U^dag = i^e P'.
    Raises ValueError when U is not Clifford."""
    nq = 1 if u.shape[0] == 2 else 2
    cands = list(itertools.product((0, 1), repeat=2 * nq))
    paulis = {c: _local_pauli(c) for c in cands}
    table = {}
    for c in cands:
        m = u @ paulis[c] @ u.conj().T
        found = None
        for q in cands:
            coef = np.trace(paulis[q].conj().T @ m) / (2 ** nq)
            if abs(coef) > 1e-6:
                if abs(abs(coef) - 1) > 1e-6 or found is not None:
                    raise ValueError("gate is not Clifford")
                k = int(np.round(np.angle(coef) / (np.pi / 2))) % 4
                if abs(coef - 1j ** k) > 1e-6:
                    raise ValueError("gate is not Clifford")
                found = (k, q)
        if found is None:
            raise ValueError("gate is not Clifford")
        table[c] = found
    return table


class Tableau:
    def __init__(self, n: int):
        self.n = n
        self.e = np.zeros(n, np.int64)           # phase exponent of i
        self.x = np.zeros((n, n), np.uint8)
        self.z = np.eye(n, dtype=np.uint8)       # |0^N> is stabilised by Z_q

    def apply(self, q0: int, q1: int, u: np.ndarray, table=None):
        table = table or conjugation_table(u)
        qs = [q0] if q1 < 0 else [q0, q1]
        for g in range(self.n):
            key = []
            for q in qs:
                key += [int(self.x[g, q]), int(self.z[g, q])]
            k, new = table[tuple(key)]
            self.e[g] = (self.e[g] + k) % 4
            for i, q in enumerate(qs):
                self.x[g, q], self.z[g, q] = new[2 * i], new[2 * i + 1]

    @staticmethod
    def _mul(e1, x1, z1, e2, x2, z2):
        # X^a Z^b X^c Z^d = (-1)^(b c) X^(a+c) Z^(b+d), qubit by qubit
        sign = int(np.dot(z1.astype(np.int64), x2.astype(np.int64)) % 2)
        return (e1 + e2 + 2 * sign) % 4, x1 ^ x2, z1 ^ z2

    def z_subgroup(self):
        """Row-reduce on the X parts; return (rank_x, list of (e, z) Z-type rows)."""
        e, x, z = self.e.copy(), self.x.copy(), self.z.copy()
        n, rank = self.n, 0
        for col in range(n):
            piv = None
            for r in range(rank, n):
                if x[r, col]:
                    piv = r
                    break
            if piv is None:
                continue
            if piv != rank:
                e[[piv, rank]] = e[[rank, piv]]
                x[[piv, rank]] = x[[rank, piv]]
                z[[piv, rank]] = z[[rank, piv]]
            for r in range(n):
                if r != rank and x[r, col]:
                    e[r], x[r], z[r] = self._mul(e[r], x[r], z[r], e[rank], x[rank], z[rank])
            rank += 1
        ztype = []
        for r in range(rank, n):
            assert not x[r].any()
            if e[r] % 2:
                raise AssertionError("Z-type stabilizer with imaginary phase")
            ztype.append((int(e[r]), z[r].copy()))
        return rank, ztype

    def probabilities(self, bits: np.ndarray) -> np.ndarray:
        """|<s|psi>|^2 for each row s of bits."""
        rank, ztype = self.z_subgroup()
        bits = np.asarray(bits, np.int64).reshape(-1, self.n)
        out = np.full(bits.shape[0], 2.0 ** (-rank))
        for e, zz in ztype:
            sign = 1 if e == 0 else -1
            par = (bits @ zz.astype(np.int64)) % 2
            ok = (sign * (1 - 2 * par)) == 1
            out = np.where(ok, out, 0.0)
        return out


def support_sample(tab: Tableau, count: int, seed: int) -> np.ndarray:
    """Uniform bitstrings from the support of the state: the s with nonzero
    amplitude solve z . s = (e / 2) mod 2 for every Z-type stabilizer
    (e, z), an affine subspace of GF(2)^N.  Gauss-Jordan elimination gives
    a particular solution and a null-space basis; each sample adds a random
    combination of the basis (numpy default_rng(seed))."""
    _, ztype = tab.z_subgroup()
    n = tab.n
    rows = [(zz.astype(np.uint8).copy(), (e // 2) % 2) for e, zz in ztype]
    a = np.array([r[0] for r in rows], np.uint8).reshape(-1, n)
    b = np.array([r[1] for r in rows], np.uint8)
    pivots, r = [], 0
    for col in range(n):
        hit = [i for i in range(r, a.shape[0]) if a[i, col]]
        if not hit:
            continue
        i = hit[0]
        a[[r, i]] = a[[i, r]]
        b[[r, i]] = b[[i, r]]
        for j in range(a.shape[0]):
            if j != r and a[j, col]:
                a[j] ^= a[r]
                b[j] ^= b[r]
        pivots.append(col)
        r += 1
    if np.any(b[r:]):
        raise AssertionError("inconsistent Z-type stabilizers")
    free = [c for c in range(n) if c not in pivots]
    rng = np.random.default_rng(seed)
    out = np.zeros((count, n), np.uint8)
    for t in range(count):
        s = np.zeros(n, np.uint8)
        s[free] = rng.integers(0, 2, len(free))
        for i, col in enumerate(pivots):
            s[col] = (b[i] + int(np.dot(a[i, free].astype(np.int64), s[free]))) % 2
        out[t] = s
    return out


def run(circ) -> Tableau:
    """Evolve |0^N> through a Clifford circuit."""
    tab = Tableau(circ.n)
    cache = {}
    for g in circ.gates:
        key = (g.q1 < 0, np.asarray(g.matrix).tobytes())
        if key not in cache:
            cache[key] = conjugation_table(np.asarray(g.matrix))
        tab.apply(g.q0, g.q1, np.asarray(g.matrix), cache[key])
    return tab


def probabilities(circ, bits: np.ndarray) -> np.ndarray:
    return run(circ).probabilities(bits)
