"""GPU parity: amplitudes through the C ABI against the CPU oracle.

Tolerances (the paper states none; the requirement is relative error <= 1e-10
for complex128 and <= 1e-4 for complex64): rel_l2 = ||b - a|| / ||a|| over the
batch, plus max |b_i - a_i| / rms(a) <= 10 x the tolerance.
"""

import sys

import numpy as np
import pytest

import paper_2011_02621_amd as T
from circuits import config, grid, diagonal53, random_circuit, mirror_circuit, bitstrings
from oracle import sv, stabilizer, sampling
from oracle.metrics import compare

pytestmark = pytest.mark.gpu

# split-BF16: the 6-product (hi/mid/lo) form is gated at the complex64
# tolerance; the 3-product form (hi/lo, ~2^-16 per product) is reported and
# gated loosely.
TOL = {"c128": 1e-10, "c64": 1e-4, "c64_bf16x6": 1e-4, "c64_bf16x3": 1e-3}


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(0)
    yield c
    c.close()


def check(ref, got, n, prec):
    m = compare(ref, got, n)
    tol = TOL[prec]
    assert m["rel_l2"] <= tol, m
    assert m["max_scaled"] <= 10 * tol, m
    return m


@pytest.fixture(scope="module")
def small():
    c, bits = config("grid3x4_d8")
    return c, bits, sv.amplitudes(c, bits)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_grid3x4_all_bitstrings(ctx, small, prec):
    c, bits, ref = small
    say("grid3x4_d8", prec, bits.shape)
    p = ctx.plan(c, precision=prec)
    got = ctx.amplitudes(p, bits)
    check(ref, got, c.n, prec)


def test_grid3x4_every_split_is_exact(ctx, small):
    c, bits, ref = small
    for k in range(0, c.depth + 1):
        say("grid3x4_d8 split", k)
        p = ctx.plan(c, split_cycle=k, precision="c128")
        got = ctx.amplitudes(p, bits[:16])
        assert compare(ref[:16], got, c.n)["rel_l2"] <= 1e-12


def random_connected_order(n, edges, seed):
    rng = np.random.default_rng(seed)
    nbr = {q: set() for q in range(n)}
    for a, b in edges:
        nbr[a].add(b)
        nbr[b].add(a)
    order = [int(rng.integers(n))]
    while len(order) < n:
        front = sorted({x for q in order for x in nbr[q]} - set(order))
        order.append(int(front[int(rng.integers(len(front)))]))
    return order


def test_grid3x4_paths_and_cuts_agree(ctx, small):
    c, bits, ref = small
    variants = [dict(path_mode="greedy"), dict(path_mode="algorithm1"),
                dict(path=random_connected_order(c.n, c.edges, 0)),
                dict(path=random_connected_order(c.n, c.edges, 1)),
                dict(cuts=[2, 9]), dict(cuts=[0, 5, 11]), dict(max_intermediate_elems=1 << 8)]
    for v in variants:
        say("grid3x4_d8 variant", v)
        p = ctx.plan(c, split_cycle=4, precision="c128", **v)
        got = ctx.amplitudes(p, bits)
        assert compare(ref, got, c.n)["rel_l2"] <= 1e-12, v


def test_slice_ranges_add_up(ctx, small):
    c, bits, ref = small
    p = ctx.plan(c, split_cycle=4, precision="c128", cuts=[2, 9])
    ns = p.info().n_slices
    say("grid3x4_d8 slice ranges of", ns)
    full = ctx.amplitudes(p, bits)
    parts = [ctx.amplitudes(p, bits, slices=r) for r in ((0, 1), (1, 100), (100, ns))]
    assert compare(full, sum(parts), c.n)["rel_l2"] <= 1e-13
    check(ref, full, c.n, "c128")
    with pytest.raises(T.TnsError):
        ctx.amplitudes(p, bits, slices=(5, 5))


def late_cuts(c, order, k):
    """Up to k bonds whose sites both sit in the last four places of order."""
    edges = [tuple(map(int, e)) for e in c.edges]
    late = [e for e, (a, b) in enumerate(edges) if min(order.index(a), order.index(b)) >= c.n - 4]
    return late[:k]


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_slice_prefix_shared(ctx, small, prec):
    # cut bonds between the last sites of the order: every slice shares the
    # steps before them, which run once per bitstring and are copied to each
    # (bitstring, slice) unit.  Amplitudes against the oracle; a range of one
    # slice (computed without sharing) plus the others (shared) is the whole.
    c, bits, ref = small
    order = [int(x) for x in ctx.plan(c, split_cycle=4, precision=prec).info().path]
    cuts = late_cuts(c, order, 2)
    p = ctx.plan(c, split_cycle=4, precision=prec, cuts=cuts, path=order, branches=False)
    i = p.info()
    say("grid3x4_d8 prefix", prec, "cuts", cuts, "prefix steps", i.n_prefix_steps, "of", len(i.step_m),
        "slices", i.n_slices)
    assert i.n_prefix_steps >= c.n - 5 and i.n_slices > 1
    got = ctx.amplitudes(p, bits)
    check(ref, got, c.n, prec)
    parts = [ctx.amplitudes(p, bits, slices=r) for r in ((0, 1), (1, 7), (7, i.n_slices))]
    assert compare(got, sum(parts), c.n)["rel_l2"] <= (1e-13 if prec == "c128" else 1e-6)


def fill_open(bits, open_qubits):
    """All bitstrings of each row with its open bits set to x = 0..2^k-1
    (first open qubit most significant)."""
    k = len(open_qubits)
    out = np.repeat(bits[:, None, :], 1 << k, axis=1).copy()
    for x in range(1 << k):
        for i, q in enumerate(open_qubits):
            out[:, x, q] = (x >> (k - 1 - i)) & 1
    return out


@pytest.mark.parametrize("prec,opts", [("c128", {}), ("c64", {}), ("c128", {"cuts": [2, 9]}),
                                       ("c128", {"split_cycle": 0}), ("c128", {"split_cycle": 9})])
def test_open_qubits_batch(ctx, prec, opts):
    c, bits = config("grid3x4_d8", n_bits=8)
    oq = [11, 0, 6]
    full = fill_open(bits, oq)
    ref = sv.amplitudes(c, full.reshape(-1, c.n)).reshape(len(bits), 8)
    say("grid3x4_d8 open", oq, prec, opts)
    p = ctx.plan(c, precision=prec, open_qubits=oq, **opts)
    got = ctx.amplitudes(p, bits)
    assert got.shape == (8, 8)
    check(ref.reshape(-1), got.reshape(-1), c.n, prec)


def test_open_qubits_53(ctx):
    # 53 qubits, depth 8: 2^6 amplitudes per contraction against single ones
    c = random_circuit(diagonal53(), 8, 31)
    oq = [47, 48, 49, 50, 51, 52]
    bits = bitstrings(53, 2, 32)
    say("diag53 d8 open", oq)
    p1 = ctx.plan(c, precision="c128")
    po = ctx.plan(c, precision="c128", open_qubits=oq)
    got = ctx.amplitudes(po, bits)
    full = fill_open(bits, oq).reshape(-1, 53)
    one = ctx.amplitudes(p1, full)
    assert compare(one, got.reshape(-1), 53)["rel_l2"] <= 1e-10


def test_no_final_layer(ctx):
    c, bits = config("grid3x4_d8", final_layer=False)
    ref = sv.amplitudes(c, bits)
    for k in (0, 5, 8):
        say("grid3x4_d8 no final layer split", k)
        got = ctx.amplitudes(ctx.plan(c, split_cycle=k), bits)
        check(ref, got, c.n, "c128")


def test_norm_by_enumeration(ctx):
    c = random_circuit(grid(3, 4), 6, 77)
    allbits = np.array([[(i >> (11 - q)) & 1 for q in range(12)] for i in range(4096)], np.uint8)
    say("grid3x4 d6 all 4096 bitstrings")
    got = ctx.amplitudes(ctx.plan(c, precision="c128"), allbits)
    assert abs(np.sum(np.abs(got) ** 2) - 1) < 1e-11


def test_mirror_small(ctx):
    c = mirror_circuit(grid(3, 4), 4, 5)
    bits = np.vstack([np.zeros((1, 12), np.uint8), bitstrings(12, 15, 3)])
    say("mirror 3x4")
    got = ctx.amplitudes(ctx.plan(c, split_cycle=4), bits)
    assert abs(got[0] - 1) < 1e-12
    assert np.abs(got[1:][bits[1:].any(axis=1)]).max() < 1e-12


@pytest.fixture(scope="module")
def grid5x5_d10_ref():
    c, bits = config("grid5x5_d10")
    say("grid5x5_d10 oracle, 1024 bitstrings")
    return c, bits, sv.amplitudes(c, bits)


@pytest.mark.parametrize("prec", ["c128", "c64", "c64_bf16x6", "c64_bf16x3"])
def test_grid5x5_d10(ctx, grid5x5_d10_ref, prec):
    # every one of the workload's 1024 bitstrings, in every precision
    c, bits, ref = grid5x5_d10_ref
    say("grid5x5_d10", prec, "plan + contract", len(bits))
    p = ctx.plan(c, precision=prec)
    got = ctx.amplitudes(p, bits)
    m = check(ref, got, c.n, prec)
    say("grid5x5_d10", prec, "rel_l2 %.3e max_scaled %.3e f_xeb %.6f" % (m["rel_l2"], m["max_scaled"], m["f_xeb"]))


def _row_kernel_steps(info, csize):
    # small steps that the row-tiled kernel takes (at least 64 rows, 8 padded
    # rows of A in 32 KiB, padded B^T in 32 KiB), and those whose store does
    # the next step's permute
    k, sp = np.asarray(info.step_kernel), np.asarray(info.step_permute)
    rows = []
    for t in range(len(k)):
        m, kk, n = int(info.step_m[t]), int(info.step_k[t]), int(info.step_n[t])
        rb = min(256, 32768 // ((kk + 1) * csize))
        if k[t] == 1 and m >= 64 and rb >= 8 and n * (kk + 1) * csize <= 32768:
            rows.append(t)
    fused = [t for t in rows if t + 1 < len(k) and sp[t + 1] == 2]
    return rows, fused


def test_slice_prefix_grid5x5_d10(ctx, grid5x5_d10_ref):
    # the 25-qubit batch with one cut bond absorbed half-way along the path
    # (sites 13 and 18): the first twelve steps are shared by the slices
    c, bits, ref = grid5x5_d10_ref
    order = [int(x) for x in ctx.plan(c, precision="c64").info().path]
    edges = [tuple(map(int, e)) for e in c.edges]
    p = ctx.plan(c, precision="c64", cuts=[edges.index((13, 18))], path=order, branches=False)
    i = p.info()
    say("grid5x5_d10 prefix steps", i.n_prefix_steps, "slices", i.n_slices)
    assert i.n_prefix_steps > 0
    got = ctx.amplitudes(p, bits)
    check(ref, got, c.n, "c64")


@pytest.fixture(scope="module")
def grid5x5_d8():
    c = random_circuit(grid(5, 5), 8, 7)
    bits = bitstrings(25, 64, 77)
    return c, bits, sv.amplitudes(c, bits)


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("split", [1, 2])
def test_small_row_steps_grid5x5_d8(ctx, grid5x5_d8, prec, split):
    # random 25-qubit circuit whose plan has small-bond steps of 64 .. 262144
    # rows, several storing in the next step's order, against the oracle
    c, bits, ref = grid5x5_d8
    p = ctx.plan(c, precision=prec, split_cycle=split)
    rows, fused = _row_kernel_steps(p.info(), 16 if prec == "c128" else 8)
    say("grid5x5_d8 small steps", prec, split, "row steps", len(rows), "fused", len(fused))
    assert len(rows) >= 4 and len(fused) >= 1
    got = ctx.amplitudes(p, bits)
    check(ref, got, c.n, prec)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_more_units_than_a_grid_dimension(ctx, small, prec):
    # 70000 bitstrings of a 12-qubit plan: a launch carries up to 65536
    # (bitstring x slice) units, beyond the 65535 blocks of a grid's y
    # dimension, so every launcher has to split its units
    c, _, _ = small
    bits = bitstrings(c.n, 70000, 7)
    say("grid3x4_d8 many units", prec, bits.shape)
    ref = sv.amplitudes(c, bits)
    got = ctx.amplitudes(ctx.plan(c, precision=prec), bits)
    check(ref, got, c.n, prec)


@pytest.mark.parametrize("prec", ["c64_bf16x6", "c64_bf16x3"])
def test_grid3x4_split_bf16(ctx, small, prec):
    c, bits, ref = small
    say("grid3x4_d8", prec)
    got = ctx.amplitudes(ctx.plan(c, precision=prec), bits)
    check(ref, got, c.n, prec)


def test_mirror_53(ctx):
    c = mirror_circuit(diagonal53(), 3, 8)
    bits = np.vstack([np.zeros((1, 53), np.uint8), bitstrings(53, 3, 4)])
    say("mirror diag53 3+3")
    got = ctx.amplitudes(ctx.plan(c, split_cycle=3, precision="c128"), bits)
    assert abs(got[0] - 1) < 1e-10
    assert np.abs(got[1:]).max() < 1e-10


@pytest.mark.parametrize("rows,cols,seed", [(2, 3, 8), (2, 3, 9), (3, 3, 9), (5, 5, 7)])
def test_mirror_every_split(ctx, rows, cols, seed):
    # Exactly cancelling gates (U then U^-1) leave rows of the compressed
    # site matrices at ~1e-150 of their scale; the Jacobi rotations must stay
    # unitary there.  Every split point, zero bitstring and random ones.
    c = mirror_circuit(grid(rows, cols), 4, seed)
    n = rows * cols
    bits = np.vstack([np.zeros((1, n), np.uint8), bitstrings(n, 7, 5)])
    say("mirror grid%dx%d seed %d, every split" % (rows, cols, seed))
    for k in range(0, 9):
        p = ctx.plan(c, precision="c128", split_cycle=k)
        got = ctx.amplitudes(p, bits)
        assert abs(got[0] - 1) < 1e-10, (k, got[0])
        assert np.abs(got[1:]).max() < 1e-10, k
        p.close()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_mirror_104(ctx, prec):
    # 104 qubits, 4 + 4 cycles: 103 contraction steps, most of their boundary
    # permutes done by the producing GEMM's store; <0|W|0> = 1 exactly and
    # every other amplitude is 0
    c = mirror_circuit(grid(8, 13), 4, 7)
    bits = np.vstack([np.zeros((1, 104), np.uint8), bitstrings(104, 3, 9)])
    say("mirror grid8x13 4+4", prec)
    p = ctx.plan(c, precision=prec)
    assert (np.asarray(p.info().step_permute) == 2).sum() > 50
    got = ctx.amplitudes(p, bits)
    tol = TOL[prec]
    assert abs(got[0] - 1) < tol
    assert np.abs(got[1:]).max() < tol


def test_clifford_53_against_tableau(ctx):
    c = random_circuit(diagonal53(), 6, 13, clifford=True)
    bits = bitstrings(53, 8, 14)
    say("clifford diag53 d6")
    p_ref = stabilizer.probabilities(c, bits)
    got = ctx.amplitudes(ctx.plan(c, precision="c128"), bits)
    assert np.abs(np.abs(got) ** 2 - p_ref).max() <= 1e-10 * max(p_ref.max(), 2.0 ** -53)


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_clifford_104_against_tableau(ctx, prec):
    # 104 qubits, 8 cycles: the same bond dimensions, path shape and 2^32-
    # element intermediates as the random 8x13 workload, with exact
    # probabilities from the tableau; two bitstrings from the state's support
    # (|amp|^2 = 2^-rank) and one uniform one (almost surely outside it)
    c = random_circuit(grid(8, 13), 8, 15, clifford=True)
    tab = stabilizer.run(c)
    bits = np.vstack([stabilizer.support_sample(tab, 2, 3), bitstrings(104, 1, 17)])
    p_ref = tab.probabilities(bits)
    assert p_ref[0] > 0 and p_ref[1] > 0
    say("clifford grid8x13 d8", prec, "plan")
    p = ctx.plan(c, precision=prec, split_cycle=1)
    say("clifford grid8x13 d8", prec, "contract, %.2e flop/amp" % p.info().flops_per_amp)
    got = ctx.amplitudes(p, bits)
    tol = TOL[prec]
    assert np.abs(np.abs(got) ** 2 - p_ref).max() <= 2 * tol * max(p_ref.max(), 2.0 ** -104)


# slices whose cut indices are (0, 0), (0, 1), (8, 0) and (15, 15): the slice
# maps then offset both cut bonds of the 2^32-element network
D12_SLICES = (0, 1, 128, 255)


@pytest.fixture(scope="module")
def diag53_d12_slices(ctx):
    # complex128 partial sums over single slices of the 53-qubit depth-12
    # contraction, with the path and cuts the other precisions reuse
    c, bits = config("diag53_d12", n_bits=1)
    say("diag53_d12 c128 plan")
    p = ctx.plan(c, precision="c128")
    i = p.info()
    same = dict(split_cycle=int(i.split_cycle), path=i.path.tolist(), cuts=i.cut_edges.tolist())
    ref = {}
    for sl in D12_SLICES:
        say("diag53_d12 c128 slice", sl)
        ref[sl] = ctx.amplitudes(p, bits, slices=(sl, sl + 1))[0]
    p.close()
    return c, bits, same, ref, int(i.n_slices), int(i.peak_elems), len(i.cut_edges)


@pytest.mark.parametrize("prec", ["c64", "c64_bf16x6"])
def test_diag53_d12_slices_against_c128(ctx, diag53_d12_slices, prec):
    # the launch configuration the bench times at 53 qubits, depth 12 (256
    # slices, 2^32-element intermediates); no oracle reaches this size, so
    # the property checked is that each slice's partial sum agrees with the
    # complex128 path on the same network to the complex64 tolerance
    c, bits, same, ref, n_slices, peak, n_cuts = diag53_d12_slices
    assert n_slices == 256 and peak == 1 << 32 and n_cuts == 2
    p = ctx.plan(c, precision=prec, **same)
    slices = D12_SLICES if prec == "c64" else (0, 255)
    for sl in slices:
        got = ctx.amplitudes(p, bits, slices=(sl, sl + 1))[0]
        rel = float(abs(got - ref[sl]) / abs(ref[sl]))
        say("diag53_d12", prec, "slice", sl, "rel %.3e" % rel)
        assert rel <= TOL[prec]
    p.close()
    # distinct slices carry distinct scalars (the offsets are applied)
    vals = [ref[sl] for sl in D12_SLICES]
    assert len({complex(v) for v in vals}) == len(vals)


def test_diag53_d12_correlated_batch_slice(ctx):
    # the 4096-amplitude correlated batch (12 open qubits, the last ones the
    # path absorbs) at 53 qubits, depth 12: one slice, complex64 against
    # complex128 on the same network, over all 4096 partial sums
    c, bits = config("diag53_d12", n_bits=1)
    p0 = T.Context(-1).plan(c, precision="c64")
    oq = [int(q) for q in p0.info().path[-12:]]
    p0.close()
    say("diag53_d12 correlated batch c128 plan")
    p = ctx.plan(c, precision="c128", open_qubits=oq)
    i = p.info()
    same = dict(split_cycle=int(i.split_cycle), path=i.path.tolist(), cuts=i.cut_edges.tolist(),
                open_qubits=oq)
    sl = int(i.n_slices) - 3
    ref = ctx.amplitudes(p, bits, slices=(sl, sl + 1)).reshape(-1)
    p.close()
    say("diag53_d12 correlated batch c64, slice", sl)
    p = ctx.plan(c, precision="c64", **same)
    got = ctx.amplitudes(p, bits, slices=(sl, sl + 1)).reshape(-1)
    p.close()
    assert ref.shape == (4096,)
    m = compare(ref, got, c.n)
    say("diag53_d12 correlated batch rel_l2 %.3e max_scaled %.3e" % (m["rel_l2"], m["max_scaled"]))
    assert m["rel_l2"] <= TOL["c64"] and m["max_scaled"] <= 10 * TOL["c64"]


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_frugal_sampling(ctx, prec):
    # correlated batches of 2^3 candidates; decisions against the oracle's
    # FP64 probabilities with the same uniform numbers (a decision may differ
    # only where 2^N p / M lies within the amplitude error of u)
    c, _ = config("grid3x4_d8")
    oq = [11, 0, 5]
    fixed = bitstrings(12, 16, 41)
    u = np.random.default_rng(42).random((16, 8))
    m = 2.0
    say("frugal sampling", prec)
    p = ctx.plan(c, precision=prec, open_qubits=oq)
    acc, amps = ctx.sample_frugal(p, fixed, u, m)
    cand = sampling.batch_bitstrings(fixed, oq)
    ref = sv.amplitudes(c, cand.reshape(-1, 12)).reshape(16, 8)
    check(ref.reshape(-1), amps.reshape(-1), c.n, prec)
    acc_ref = sampling.frugal_accept(np.abs(ref) ** 2, u, c.n, m)
    margin = np.abs(np.abs(ref) ** 2 * 2.0 ** c.n / m - u)
    differ = acc != acc_ref
    thr = 1e-6 if prec == "c64" else 1e-12
    assert not np.any(differ & (margin > thr))
    assert 0 < acc.sum() < acc.size


def test_empty_single_and_duplicate_batches(ctx, small):
    c, bits, ref = small
    p = ctx.plan(c, precision="c128")
    say("empty / single / duplicate batches")
    assert ctx.amplitudes(p, bits[:0]).shape == (0,)
    got1 = ctx.amplitudes(p, bits[3:4])
    assert abs(got1[0] - ref[3]) <= 1e-10 * np.linalg.norm(ref) / np.sqrt(len(ref))
    dup = np.repeat(bits[5:6], 9, axis=0)
    got = ctx.amplitudes(p, dup)
    assert np.all(got == got[0]) and abs(got[0] - ref[5]) < 1e-10 * np.abs(ref).max()


def test_small_budget_ragged_batches():
    # a 48 MiB budget forces small bitstring batches and few units per
    # launch, with ragged tails in both; 4100 bitstrings also exceed the
    # per-batch cap of 4096
    c, _ = config("grid3x4_d8")
    bits = bitstrings(12, 4100, 77)
    ref = sv.amplitudes(c, bits)
    say("small budget, 4100 bitstrings")
    small_ctx = T.Context(0, 48 << 20)
    try:
        for prec in ("c128", "c64"):
            got = small_ctx.amplitudes(small_ctx.plan(c, precision=prec), bits)
            check(ref, got, c.n, prec)
    finally:
        small_ctx.close()


def test_stream_argument(ctx, small):
    import torch
    c, bits, ref = small
    s = torch.cuda.Stream()
    say("explicit torch stream")
    got = ctx.amplitudes(ctx.plan(c), bits, stream=s.cuda_stream)
    check(ref, got, c.n, "c128")


def test_serving_equivalence(ctx, small):
    c, bits, ref = small
    c2, bits2 = config("grid5x5_d10", n_bits=24)
    p1 = ctx.plan(c, precision="c64")
    p2 = ctx.plan(c2, precision="c64")
    alone1 = ctx.amplitudes(p1, bits)
    alone2 = ctx.amplitudes(p2, bits2)
    say("serving mix")
    reqs = []
    for i in range(6):
        reqs.append(ctx.submit(p2, bits2))
        reqs.append(ctx.submit(p1, bits))
    outs = [r.wait() for r in reqs]
    for i, o in enumerate(outs):
        want = alone2 if i % 2 == 0 else alone1
        assert np.array_equal(o, want)
    check(ref, outs[1], c.n, "c64")
