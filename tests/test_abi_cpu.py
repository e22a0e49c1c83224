"""Host-side tests of the C ABI (no GPU): symbol exports, planning-only
contexts, error codes, bond-dimension pins of the paper and the path search
against the oracle's brute force."""

import re
import os

import numpy as np
import pytest

import paper_2011_02621_amd as T
from circuits import CZ, fsim, grid, diagonal53, random_circuit, config
from circuits.rqc import Circuit, Gate
from oracle import paths

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(-1)
    yield c
    c.close()


def test_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "tns.h")).read()
    declared = set(re.findall(r"^(?:tns_status|void|const char \*)\s*\n?\s*(tns_\w+)\(", header, re.M))
    declared |= set(re.findall(r"\b(tns_\w+)\(", header)) - {"tns_gate", "tns_plan_info"}
    lib = T.load_library()
    assert declared, "no declarations parsed"
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(T.EXPORTED) <= declared


def test_version():
    assert "gfx950" in T.version()


def test_planning_only_context_rejects_compute(ctx):
    c, bits = config("grid3x4_d8")
    p = ctx.plan(c, precision="c128")
    with pytest.raises(T.TnsError) as e:
        ctx.amplitudes(p, bits[:2])
    assert e.value.name == "TNS_E_NO_DEVICE"


def _two_qubit_circuit(n, edges, ops):
    gates = [Gate(a, b, cyc, np.asarray(m, complex)) for a, b, cyc, m in ops]
    return Circuit(n, edges, gates, 1)


def test_sample_frugal_argument_errors(ctx):
    c, bits = config("grid3x4_d8")
    p = ctx.plan(c, open_qubits=[0, 1])
    u = np.zeros((2, 4))
    with pytest.raises(T.TnsError) as e:
        ctx.sample_frugal(p, bits[:2], u, m_bound=0.0)
    assert e.value.name == "TNS_E_INVALID_ARG"
    with pytest.raises(T.TnsError) as e:
        ctx.sample_frugal(p, bits[:2], u, m_bound=10.0)
    assert e.value.name == "TNS_E_NO_DEVICE"


def test_serving_argument_errors():
    # host-side checks of the serving calls: knob ranges, a planning-only
    # context, and NULL request handles
    import ctypes
    lib = T.load_library()
    c = T.Context(-1)
    try:
        for kw in ({"n_workers": 17}, {"n_workers": -1}, {"item_flops": -1.0},
                   {"item_flops": float("nan")}):
            with pytest.raises(T.TnsError) as e:
                c.configure_serving(**kw)
            assert e.value.name == "TNS_E_INVALID_ARG", kw
        c.configure_serving(n_workers=2, item_flops=1e12)   # accepted before any submit
        circ, bits = config("grid3x4_d8")
        p = c.plan(circ, precision="c64")
        with pytest.raises(T.TnsError) as e:
            c.submit(p, bits[:2])
        assert e.value.name == "TNS_E_NO_DEVICE"
        p.close()
    finally:
        c.close()
    d = ctypes.c_int(7)
    t, r = ctypes.c_double(), ctypes.c_double()
    assert T.STATUS[lib.tns_poll(None, ctypes.byref(d))] == "TNS_E_INVALID_ARG"
    assert T.STATUS[lib.tns_wait(None)] == "TNS_E_INVALID_ARG"
    assert T.STATUS[lib.tns_cancel(None)] == "TNS_E_INVALID_ARG"
    assert T.STATUS[lib.tns_request_latency(None, ctypes.byref(t), ctypes.byref(r))] == "TNS_E_INVALID_ARG"
    assert lib.tns_request_free(None) == 0
    assert lib.tns_plan_destroy(None) == 0
    assert lib.tns_finalize(None) == 0


def test_bad_circuits(ctx):
    good = _two_qubit_circuit(2, [(0, 1)], [(0, 1, 0, fsim(np.pi / 2, np.pi / 6))])
    ctx.plan(good)
    cases = {
        "non-edge": _two_qubit_circuit(3, [(0, 1), (1, 2)], [(0, 2, 0, CZ)]),
        "qubit range": _two_qubit_circuit(2, [(0, 1)], [(0, 5, 0, CZ)]),
        "not unitary": _two_qubit_circuit(2, [(0, 1)], [(0, 1, 0, 2 * CZ)]),
        "duplicate edge": _two_qubit_circuit(2, [(0, 1), (1, 0)], [(0, 1, 0, CZ)]),
    }
    for name, circ in cases.items():
        with pytest.raises(T.TnsError) as e:
            ctx.plan(circ)
        assert e.value.name == "TNS_E_BAD_CIRCUIT", name


def test_bad_path_and_cuts(ctx):
    c, _ = config("grid3x4_d8")
    with pytest.raises(T.TnsError) as e:
        ctx.plan(c, path=[0] * 12)
    assert e.value.name == "TNS_E_BAD_PATH"
    with pytest.raises(T.TnsError) as e:
        ctx.plan(c, cuts=[999])
    assert e.value.name == "TNS_E_BAD_PATH"
    with pytest.raises(T.TnsError) as e:
        ctx.plan(c, split_cycle=99)
    assert e.value.name == "TNS_E_INVALID_ARG"


def test_first_gate_compression_bond_is_two(ctx):
    # Eq. (7): a qubit's first chi=4 gate leaves a bond of at most 2.
    c = _two_qubit_circuit(4, [(0, 1), (1, 2), (2, 3)],
                           [(0, 1, 0, fsim(np.pi / 2, np.pi / 6)), (2, 3, 0, fsim(np.pi / 2, np.pi / 6))])
    p = ctx.plan(c, split_cycle=1)
    i = p.info()
    assert list(i.bond_ket) == [2, 1, 2]
    assert list(i.bond_bra) == [1, 1, 1]


def test_controlled_gate_has_rank_two(ctx):
    # Eq. (2): chi_o = 2 for a controlled gate.  Two CZs on the same pair
    # of fresh qubits: 2 then min(2*2, 2 * rest = 2) = 2.
    c = _two_qubit_circuit(2, [(0, 1)], [(0, 1, 0, CZ), (0, 1, 0, CZ)])
    assert list(ctx.plan(c, split_cycle=1).info().bond_ket) == [2]
    # a chain: the middle qubit's bonds are not capped by a single leg
    c = _two_qubit_circuit(3, [(0, 1), (1, 2)], [(0, 1, 0, CZ), (1, 2, 0, CZ), (0, 1, 0, CZ)])
    assert list(ctx.plan(c, split_cycle=1).info().bond_ket) == [2, 2]


def test_dcd_pattern_is_capped(ctx):
    # gates on (k,l), (l,r), (k,l): the k-l bond would reach chi^2 = 16 but
    # is capped at 2 * (rest of k) = 2 when k has no other bond.
    f = fsim(np.pi / 2, np.pi / 6)
    c = _two_qubit_circuit(3, [(0, 1), (1, 2)], [(0, 1, 0, f), (1, 2, 0, f), (0, 1, 0, f)])
    i = ctx.plan(c, split_cycle=1).info()
    assert i.bond_ket[0] == 2


def test_overlap_bonds_multiply(ctx):
    c, _ = config("grid3x4_d8")
    i = ctx.plan(c, split_cycle=4).info()
    assert np.array_equal(i.bond_overlap, i.bond_ket * i.bond_bra)


def test_plan_info_consistency(ctx):
    c, _ = config("grid5x5_d10")
    i = ctx.plan(c, precision="c64").info()
    assert sorted(i.path.tolist()) == list(range(25))
    assert len(i.step_m) == 24
    flops = 8 * np.sum(i.step_m.astype(float) * i.step_k * i.step_n) * i.n_slices
    assert flops == pytest.approx(i.flops_per_amp)
    assert i.step_m[-1] == 1 and i.step_n[-1] == 1 and i.step_kernel[-1] == 2
    # the reported scores are the oracle's: the order as one linear path, and
    # the plan with its side branches
    dims = [float(d) for d in i.bond_overlap]
    s, _ = paths.score(i.path.tolist(), c.n, c.edges, dims)
    assert s == pytest.approx(i.linear_score)
    windows = [tuple(w) for w in i.branch_windows.tolist()]
    ts, peak, bpeak = paths.tree_score(i.path.tolist(), windows, c.n, c.edges, dims)
    assert ts == pytest.approx(i.path_score) and peak == i.peak_elems
    assert len(windows) > 0 and i.path_score < i.linear_score
    assert set(i.step_chain.tolist()) == set(range(len(windows) + 1))


def test_branches_off_is_the_linear_path(ctx):
    c, _ = config("grid5x5_d10")
    i = ctx.plan(c, precision="c64", branches=False).info()
    assert len(i.branch_windows) == 0 and i.path_score == pytest.approx(i.linear_score)
    assert set(i.step_chain.tolist()) == {0}


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_branch_plans_within_the_tree_optimum(ctx, seed):
    # 3x3 grids: the plan's summed cost, with whatever branches it chose, is
    # the oracle's cost of that plan, no worse than its own linear path, and
    # no better than the best contraction tree (exhaustive, oracle)
    c = random_circuit(grid(3, 3), 5, seed)
    i = ctx.plan(c, precision="c64").info()
    dims = [float(d) for d in i.bond_overlap]
    windows = [tuple(w) for w in i.branch_windows.tolist()]
    ts, peak, _ = paths.tree_score(i.path.tolist(), windows, c.n, c.edges, dims)
    assert ts == pytest.approx(i.path_score) and peak == i.peak_elems
    assert i.path_score <= i.linear_score * (1 + 1e-12)
    assert paths.tree_optimum(c.n, c.edges, dims) <= i.path_score * (1 + 1e-12)


def _small_rows_fits(m, k, n, csize):
    # the row-tiled small-step kernel: at least 64 rows, 8 padded rows of A in
    # 32 KiB and the padded B^T in 32 KiB of LDS
    rb = min(256, 32768 // ((k + 1) * csize))
    return m >= 64 and rb >= 8 and n * (k + 1) * csize <= 32768


@pytest.mark.parametrize("workload", ["grid5x5_d10", "diag53_d12"])
def test_permutes_fused_into_stores(ctx, workload):
    # a boundary permute after an MFMA GEMM step (either form), or after a
    # small step that the row-tiled kernel takes, is done by that step's store
    c, _ = config(workload, n_bits=1)
    for prec in ("c64", "c128"):
        i = ctx.plan(c, precision=prec).info()
        elem = 16 if prec == "c128" else 8
        # the step arrays start at the first contraction (entry t is step t+1
        # after the starting tensor)
        sp, k = np.asarray(i.step_permute), np.asarray(i.step_kernel)
        m, kk, n = (np.asarray(a) for a in (i.step_m, i.step_k, i.step_n))
        fusable = [k[t] in (0, 3) or (k[t] == 1 and _small_rows_fits(m[t], kk[t], n[t], elem))
                   for t in range(len(k))]
        # complex64 wide steps take the three-multiplication GEMM (class 3)
        wide = [t for t in range(len(k))
                if k[t] in (0, 3) and kk[t] % 2 == 0 and kk[t] >= 128 and n[t] >= 64 and m[t] >= 64]
        assert all(k[t] == (3 if prec == "c64" else 0) for t in wide)
        assert (sp == 2).sum() > 0
        # the producer of step t's boundary tensor: the previous step of the
        # same chain (main path or branch), none for a chain's first step
        ch = np.asarray(i.step_chain)
        prod = [max([u for u in range(t) if ch[u] == ch[t]], default=-1) for t in range(len(k))]
        for t in np.nonzero(sp == 2)[0]:
            assert prod[t] >= 0 and fusable[prod[t]]
        for t in np.nonzero(sp == 1)[0]:
            assert prod[t] < 0 or not fusable[prod[t]]
        if workload == "diag53_d12":
            # the large permutes there follow small steps
            assert any(sp[t] == 2 and k[t - 1] == 1 for t in range(1, len(k)))
        # permute launches only (the permuted tensor holds M * K elements):
        # the fused ones are not counted
        launched = sum(2.0 * elem * m[t] * kk[t] for t in np.nonzero(sp == 1)[0])
        assert i.permute_bytes_per_amp == pytest.approx(launched * i.n_slices)


def test_fidelity_reported(ctx):
    c, _ = config("diag53_d12", final_layer=False)
    i = ctx.plan(c, split_cycle=6, path_mode="greedy", max_intermediate_elems=1 << 60).info()
    assert i.fidelity == pytest.approx(9.314e-3, abs=5e-6)


def test_explicit_cuts_multiply_slices(ctx):
    c, _ = config("grid3x4_d8")
    i0 = ctx.plan(c, split_cycle=4).info()
    i1 = ctx.plan(c, split_cycle=4, cuts=[3, 10]).info()
    assert i1.n_slices == i0.bond_overlap[3] * i0.bond_overlap[10]
    assert list(i1.cut_edges) == [3, 10]


def test_slice_prefix_accounting(ctx):
    # cutting leaves the sub-networks different only in the cut indices, so
    # the steps before the first site that carries a cut bond are the same in
    # every slice: the plan reports them as a prefix counted once per
    # bitstring.  On a linear path the start site is order[0] and step j
    # absorbs order[j + 1], so the prefix holds the t - 1 steps before the
    # first cut site at position t (none when t < 2: the start alone is not
    # shared).
    c, _ = config("grid5x5_d10")
    order = [int(x) for x in ctx.plan(c, precision="c64").info().path]
    edges = [tuple(map(int, e)) for e in c.edges]
    seen = set()
    for e, (a, b) in enumerate(edges):
        t = min(order.index(a), order.index(b))
        if t in seen and t not in (0, 1):
            continue
        seen.add(t)
        i = ctx.plan(c, precision="c64", cuts=[e], path=order, branches=False).info()
        want = t - 1 if t >= 2 else 0
        assert i.n_prefix_steps == want, (a, b, t)
        mkn = 8 * i.step_m.astype(float) * i.step_k * i.step_n
        assert i.prefix_flops_per_amp == pytest.approx(np.sum(mkn[:want]))
        ns = i.n_slices
        assert ns == i.bond_overlap[e] and ns > 1
        assert i.flops_per_amp == pytest.approx(ns * np.sum(mkn) - (ns - 1) * np.sum(mkn[:want]))


def test_automatic_cuts_respect_limit(ctx):
    c, _ = config("grid5x5_d10")
    i = ctx.plan(c, precision="c64", max_intermediate_elems=1 << 18).info()
    assert i.peak_elems <= 1 << 18 and i.n_slices > 1


def test_open_qubits_plan(ctx):
    c, _ = config("grid3x4_d8")
    i0 = ctx.plan(c, split_cycle=4).info()
    i1 = ctx.plan(c, split_cycle=4, open_qubits=[11, 0]).info()
    assert list(i1.open_qubits) == [11, 0]
    assert len(i1.bond_overlap) == len(i0.bond_overlap) + 2
    # the open legs have dimension 2 on the bra side and 1 on the ket side
    assert list(i1.bond_bra[-2:]) == [2, 2] and list(i1.bond_ket[-2:]) == [1, 1]
    assert i1.flops_per_amp >= i0.flops_per_amp
    for bad in ([12], [1, 1]):
        with pytest.raises(T.TnsError) as e:
            ctx.plan(c, open_qubits=bad)
        assert e.value.name == "TNS_E_INVALID_ARG"


# --- path search vs brute force (supplement, Algorithm 1 and Eq. (optscore))

def _random_graph(seed, n):
    rng = np.random.default_rng(seed)
    edges = set()
    for q in range(1, n):
        edges.add((int(rng.integers(q)), q))
    while len(edges) < n + 2:
        a, b = sorted(rng.choice(n, 2, replace=False))
        edges.add((int(a), int(b)))
    edges = sorted(edges)
    dims = [float(2 ** rng.integers(1, 5)) for _ in edges]
    return edges, dims


@pytest.mark.parametrize("seed", range(8))
def test_algorithm1_without_assumptions_is_optimal(seed):
    n = 7
    edges, dims = _random_graph(seed, n)
    best, _ = paths.brute_force(n, edges, dims)
    order, score = T.path_search(n, edges, dims, mode="algorithm1", assumptions=False)
    assert sorted(order) == list(range(n))
    assert paths.score(order, n, edges, dims)[0] == score
    assert score == best


@pytest.mark.parametrize("seed", range(6))
def test_size_bounded_algorithm1_is_optimal_among_bounded_orders(seed):
    # with the assumptions off Algorithm 1 is exact; with a size bound it is
    # exact over the orders whose every intermediate fits (oracle brute force)
    n = 7
    edges, dims = _random_graph(200 + seed, n)
    _, free_peak = paths.score(paths.brute_force(n, edges, dims)[1], n, edges, dims)
    sizes = sorted({paths.score(list(o), n, edges, dims)[1]
                    for o in [np.random.default_rng(seed + k).permutation(n).tolist() for k in range(40)]})
    for bound in sizes[: len(sizes) // 2 + 1]:
        best, _ = paths.brute_force_bounded(n, edges, dims, bound)
        if best is None:
            with pytest.raises(T.TnsError):
                T.path_search(n, edges, dims, mode="algorithm1", assumptions=False, max_intermediate=bound)
            continue
        order, score = T.path_search(n, edges, dims, mode="algorithm1", assumptions=False,
                                     max_intermediate=bound)
        s, peak = paths.score(order, n, edges, dims)
        assert s == score == best and peak <= bound
    assert free_peak > 0


@pytest.mark.parametrize("seed", range(4))
def test_restricted_searches_are_admissible(seed):
    n = 8
    edges, dims = _random_graph(100 + seed, n)
    best, _ = paths.brute_force(n, edges, dims)
    for mode in ("algorithm1", "greedy"):
        order, score = T.path_search(n, edges, dims, mode=mode, assumptions=True)
        assert sorted(order) == list(range(n))
        assert paths.score(order, n, edges, dims)[0] == score >= best


def test_algorithm1_grid_beats_or_ties_greedy():
    g = grid(4, 4)
    rng = np.random.default_rng(3)
    dims = [float(2 ** rng.integers(2, 5)) for _ in g.edges]
    _, s1 = T.path_search(g.n, g.edges, dims, mode="algorithm1")
    _, sg = T.path_search(g.n, g.edges, dims, mode="greedy")
    assert s1 <= sg


def test_exhausted_exact_search_falls_back_to_greedy(ctx):
    # Algorithm 1 without its assumptions and a tiny state budget: the plan
    # keeps the greedy path and reports the search as incomplete
    c, _ = config("grid3x4_d8")
    i = ctx.plan(c, path_mode="algorithm1", path_assumptions=False, max_search_states=3).info()
    g = ctx.plan(c, path_mode="greedy").info()
    assert not i.search_complete
    assert list(i.path) == list(g.path)
    assert i.flops_per_amp == g.flops_per_amp
