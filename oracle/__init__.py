"""CPU oracle for the amplitude method -- test infrastructure, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import or run anything here.  The oracle shares no code with
the GPU library (``paper_2011_02621_amd``): no kernels, headers, helpers or
tables.  Both sides read the same seeded inputs from ``circuits``.

Contents, each tied to the passage of the paper it follows:

* ``sv``          -- dense complex128 state vector (plain C + OpenMP): the plain
                     definition amp(s) = <s|U|0^N> that the method reaches
                     exactly (Eq. (1) initial state, the two-sided evolution and
                     overlap of Eq. (8) evaluate exactly this number).
* ``dense``       -- full-unitary brute force from Kronecker products (N <= 10),
                     an independent check of ``sv``.
* ``stabilizer``  -- Aaronson-Gottesman stabilizer tableau for Clifford
                     circuits at any N: |amp|^2 in {0, 2^-r} exactly.
* ``paths``       -- brute-force optimum over all linear contraction orders of
                     the score of the supplement's path section (the minimum
                     over perm(N) that Algorithm 1 searches for).
* ``fidelity``    -- the closed form of Eq. (9) and the bitstring count
                     N_s >= (3/F)^2.
* ``metrics``     -- error and fidelity statistics between two amplitude sets.
"""
