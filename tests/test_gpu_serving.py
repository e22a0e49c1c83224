"""Serving (continuous batching) through the C ABI: results alone and in the
mix, sliced requests cut into (bitstring, slice) work items, overlap of
concurrent requests, memory admission, cancellation, and the host-forcible
failure paths (admission, out of memory, an external allocator)."""

import sys
import time

import numpy as np
import pytest

import paper_2011_02621_amd as T
from circuits import config, grid, random_circuit, bitstrings
from oracle import sv
from oracle.metrics import compare

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g12():
    c, bits = config("grid3x4_d8")
    return c, bits, sv.amplitudes(c, bits)


def _cut_plan(ctx, c, prec="c64"):
    # explicit cuts on two couplers of the 3x4 grid: several slices per amplitude
    return ctx.plan(c, precision=prec, cuts=[0, 5])


def test_sliced_requests_in_single_units(g12):
    # every work item is one (bitstring, slice) unit; the request's partial
    # sums are added in slice order, so the served result is the same alone
    # and beside other requests, and matches the oracle
    c, bits, ref = g12
    ctx = T.Context(0)
    try:
        ctx.configure_serving(n_workers=3, item_flops=1.0)
        p = _cut_plan(ctx, c)
        assert p.info().n_slices > 1
        say("serving: sliced plan with", p.info().n_slices, "slices, single-unit items")
        alone = ctx.submit(p, bits).wait().copy()
        m = compare(ref, alone, c.n)
        assert m["rel_l2"] <= 1e-4 and m["max_scaled"] <= 1e-3, m
        c2, bits2 = config("grid5x5_d10", n_bits=8)
        p2 = ctx.plan(c2, precision="c64")
        reqs = []
        for i in range(4):
            reqs.append(ctx.submit(p2, bits2))
            reqs.append(ctx.submit(p, bits))
        outs = [r.wait() for r in reqs]
        for i in range(1, len(outs), 2):
            assert np.array_equal(outs[i], alone)
        sync = ctx.amplitudes(p, bits)
        assert np.abs(sync - alone).max() <= 1e-6 * np.abs(ref).max()
    finally:
        ctx.close()


def test_many_short_requests_freed_at_once(g12):
    # each request is freed the moment its wait returns, while the workers
    # still complete and notify the others: the request must not be touched
    # after the waiter has seen it done
    c, bits, ref = g12
    ctx = T.Context(0)
    try:
        p = ctx.plan(c, precision="c64")
        alone = ctx.amplitudes(p, bits[:4])
        say("64 short requests, freed as they finish")
        reqs = [ctx.submit(p, bits[:4]) for _ in range(64)]
        for r in reqs:
            got = r.wait().copy()
            r.close()
            assert np.array_equal(got, alone)
        p.close()
    finally:
        ctx.close()


def test_sliced_requests_share_the_prefix(g12):
    # cut bonds among the last sites of the path: each work item covering
    # several slices computes the prefix once per bitstring; the served result
    # matches the synchronous call and the oracle
    c, bits, ref = g12
    ctx = T.Context(0)
    try:
        order = [int(x) for x in ctx.plan(c, split_cycle=4, precision="c64").info().path]
        edges = [tuple(map(int, e)) for e in c.edges]
        cuts = [e for e, (a, b) in enumerate(edges) if min(order.index(a), order.index(b)) >= c.n - 4][:2]
        p = ctx.plan(c, split_cycle=4, precision="c64", cuts=cuts, path=order, branches=False)
        i = p.info()
        assert i.n_prefix_steps > 0 and i.n_slices > 1
        say("serving: prefix of", i.n_prefix_steps, "steps,", i.n_slices, "slices")
        served = [ctx.submit(p, bits) for _ in range(3)]
        outs = [r.wait().copy() for r in served]
        sync = ctx.amplitudes(p, bits)
        for o in outs:
            assert np.abs(o - sync).max() <= 1e-6 * np.abs(ref).max()
        m = compare(ref, outs[0], c.n)
        assert m["rel_l2"] <= 1e-4 and m["max_scaled"] <= 1e-3, m
    finally:
        ctx.close()


def test_two_requests_run_together():
    # two requests submitted together run concurrently: each one's run
    # interval (admission to completion) overlaps the other's
    c, bits = config("grid5x5_d10", n_bits=192)
    ctx = T.Context(0)
    try:
        p = ctx.plan(c, precision="c64")
        ctx.amplitudes(p, bits[:4])
        say("serving: two requests of 192 bitstrings")
        t0 = time.perf_counter()
        r1 = ctx.submit(p, bits)
        t1 = time.perf_counter()
        r2 = ctx.submit(p, bits[::-1].copy())
        t2 = time.perf_counter()
        a1, a2 = r1.wait().copy(), r2.wait().copy()
        (tot1, run1), (tot2, run2) = r1.latency_ms(), r2.latency_ms()
        # run interval of a request, ms after t0: [submit + total - run, submit + total]
        sub1, sub2 = 0.0, (t1 - t0) * 1e3
        s1, e1 = sub1 + tot1 - run1, sub1 + tot1
        s2, e2 = sub2 + tot2 - run2, sub2 + tot2
        say("runs [%.0f, %.0f] and [%.0f, %.0f] ms" % (s1, e1, s2, e2))
        assert s2 < e1 - 1.0 and s1 < e2 - 1.0
        assert np.array_equal(a1, a2[::-1])
        assert t2 - t0 < 0.5 * min(run1, run2) * 1e-3
    finally:
        ctx.close()


def test_memory_pool_admits_items_as_memory_frees():
    # a budget whose worker pool holds one item of the 25-qubit plan at a
    # time: requests of two plans wait for memory, idle workers return their
    # workspace, and every result is right
    c5, b5 = config("grid5x5_d10", n_bits=6)
    c3, b3 = config("grid3x4_d8")
    ref3 = sv.amplitudes(c3, b3)
    probe = T.Context(0)
    p5 = probe.plan(c5, precision="c64")
    unit = p5.info().device_bytes_per_unit
    want5 = probe.amplitudes(p5, b5)
    probe.close()
    budget = int(unit * 2.2)   # pool = 3/4 of it: one unit of the 25-qubit plan
    ctx = T.Context(0, budget)
    try:
        ctx.configure_serving(n_workers=3, item_flops=1.0)
        p5 = ctx.plan(c5, precision="c64")
        p3 = ctx.plan(c3, precision="c64")
        say("serving: pool of %.0f MiB, 25-qubit units of %.0f MiB" % (0.75 * budget / 2 ** 20, unit / 2 ** 20))
        reqs = [ctx.submit(p5, b5), ctx.submit(p3, b3), ctx.submit(p5, b5[::-1].copy()), ctx.submit(p3, b3)]
        outs = [r.wait() for r in reqs]
        assert np.array_equal(outs[0], want5) and np.array_equal(outs[2], want5[::-1])
        for o in (outs[1], outs[3]):
            m = compare(ref3, o, c3.n)
            assert m["rel_l2"] <= 1e-4, m
    finally:
        ctx.close()


def test_cancel_mid_flight():
    c, bits = config("grid5x5_d10")
    c3, b3 = config("grid3x4_d8")
    ctx = T.Context(0)
    try:
        ctx.configure_serving(n_workers=2, item_flops=1.0)
        p = ctx.plan(c, precision="c64")
        p3 = ctx.plan(c3, precision="c128")
        say("serving: cancel a 1024-bitstring request")
        long_req = ctx.submit(p, bits)
        other = ctx.submit(p3, b3)
        time.sleep(0.05)
        long_req.cancel()
        with pytest.raises(T.TnsError) as e:
            long_req.wait()
        assert e.value.name == "TNS_E_CANCELLED"
        got = other.wait()
        m = compare(sv.amplitudes(c3, b3), got, c3.n)
        assert m["rel_l2"] <= 1e-10, m
        # the context keeps serving after a cancellation
        again = ctx.submit(p3, b3[:4]).wait()
        assert np.array_equal(again, got[:4])
    finally:
        ctx.close()


def test_admission_and_out_of_memory_are_reported():
    c, _ = config("grid5x5_d10", n_bits=1)
    probe = T.Context(-1)
    unit = probe.plan(c, precision="c64").info().device_bytes_per_unit
    probe.close()
    # budget above one unit (the plan is created) but a pool below it
    ctx = T.Context(0, int(unit * 1.2))
    try:
        p = ctx.plan(c, precision="c64")
        say("serving: admission refused")
        with pytest.raises(T.TnsError) as e:
            ctx.submit(p, bitstrings(25, 2, 1))
        assert e.value.name == "TNS_E_ADMISSION"
    finally:
        ctx.close()
    # a budget below one unit: the plan itself is refused
    ctx = T.Context(0, 48 << 20)
    try:
        with pytest.raises(T.TnsError) as e:
            ctx.plan(c, precision="c64")
        assert e.value.name == "TNS_E_OUT_OF_MEMORY"
    finally:
        ctx.close()


def test_torch_allocator(g12):
    import torch
    c, bits, ref = g12
    ctx = T.Context(0)
    try:
        ctx.use_torch_allocator()
        before = torch.cuda.memory_allocated()
        p = ctx.plan(c, precision="c128")
        assert torch.cuda.memory_allocated() > before
        say("torch allocator: sync and served")
        got = ctx.amplitudes(p, bits)
        m = compare(ref, got, c.n)
        assert m["rel_l2"] <= 1e-10, m
        served = ctx.submit(p, bits).wait()
        assert np.array_equal(served, got)
        p.close()
    finally:
        ctx.close()
