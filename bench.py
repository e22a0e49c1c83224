#!/usr/bin/env python3
"""Benchmark: amplitudes/s of the tensor-network-states amplitude path on one
MI355X, with the dominant kernel's roofline and the CPU oracle beside it.

Headline (default): one whole amplitude of the 53-qubit diagonal lattice at
depth 12 (12 random cycles and a closing single-qubit layer, circuit seed 3,
the first bitstring of seed 103), complex64 on FP32 MFMA.  The plan cuts the
merged network into independent slices (sub-networks whose scalars add up to
the amplitude); the K timed steps split the slices into K consecutive ranges,
each step runs the whole path -- bra evolution with SVD compression, overlap
merge, slice gathers, every permute + complex GEMM of the contraction path and
the FP64 slice sum -- over its range, and the host adds the K partial sums in
FP64.  So the timed region computes the amplitude whole, and value = 1 /
(timed seconds).  Warm-up steps run single slices.  Tensors stay in HBM; the
bitstring (53 bytes) is uploaded and the partial sums come back inside each
step.

Other legs (25-qubit batches, depth 10, correlated batches, 104 qubits,
serving) run only when named in --legs.  --slice-range A:B computes one
partial sum over slices [A, B) and prints it alone (reference runs in
complex128, which take longer than one call allows).

Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# dense MFMA peaks of MI355X (TFLOP/s): FP32 for complex64, FP64 for
# complex128, BF16 for the split-BF16 forms, whose BF16 products are the
# executed flops (the complex product's 8 M K N count is reported beside it
# as credited_tflops)
PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6, "c64_bf16x3": 2500.0, "c64_bf16x6": 2500.0}
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant kernel (k_gemm_3m), from rocprofv3
# FETCH_SIZE and WRITE_SIZE runs scaled by a plain-copy calibration.  The
# figure is read from the summary in profiles/ that records it, keyed by the
# sha256 prefix of the kernel source the counters were taken on, the workload
# and the algorithmic bytes per launch; any change makes the entry stale and
# the line reports null.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm3m_diag53_d12_traffic.md")


def measured_traffic(src_hash, workload, alg_mib):
    """HBM bytes per k_gemm_3m launch recorded for this kernel source, or None."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    for ln in lines:
        if ln.startswith("traffic_entry:"):
            f = dict(kv.split("=", 1) for kv in ln.split(":", 1)[1].split())
            if (f.get("kernel_sha") == src_hash and f.get("workload") == workload
                    and abs(float(f.get("alg_mib_per_launch", -1)) - alg_mib) < 0.5):
                return float(f["bytes_per_launch"])
    return None


def kernel_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_2011_02621_amd", "csrc", "kernels_contract.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_l2(a, b):
    return float(np.linalg.norm(b - a) / np.linalg.norm(a))


def xeb(a, b, n):
    p = np.abs(a) ** 2 * 2.0 ** n
    q = np.abs(b) ** 2 * 2.0 ** n
    return float((np.mean(p * q) - 1) / (np.mean(p * p) - 1))


def serving_pool(T, size, seed):
    """Seeded circuits of the serving mix: 20-53 qubits, half on the first N
    sites of a floor(sqrt(N))-row grid, half on the first N sites of the
    53-qubit diagonal lattice, depths 6-12."""
    import math
    from circuits import grid, diagonal53, random_circuit
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(size):
        kind = "grid" if rng.random() < 0.5 else "diag"
        n = int(rng.integers(20, 54))
        d = int(rng.integers(6, 13))
        r = math.isqrt(n)
        lat = grid(r, -(-n // r)).sub(n) if kind == "grid" else diagonal53().sub(n)
        pool.append((f"{kind}{n}_d{d}", random_circuit(lat, d, 4000 + i)))
    return pool, rng


def serving_run(T, ctx, torch, n_req=200, pool_size=24, cap_gpu_s=5.0, nominal_tflops=100.0,
                load=0.7, seed=4, max_elems=1 << 28):
    """Continuous batching on the serving mix (complex64).  The pool's plans
    are compiled ahead and stay resident; they are compiled with a
    2^28-element intermediate limit (2 GiB per (bitstring, slice) unit in
    complex64), so the circuits beyond it are sliced and served as blocks of
    (bitstring, slice) units.  Admission: a request whose planned work (flops
    per amplitude x bitstrings) exceeds cap_gpu_s at nominal_tflops is
    rejected and counted; the library admits the rest by memory.  Bitstrings
    per request are log-uniform in 1..1024.  Arrivals are Poisson at the rate
    that gives the stated offered load, from service times measured on the
    device before the run."""
    import math
    from circuits import bitstrings
    pool, rng = serving_pool(T, pool_size, seed)
    pctx = T.Context(-1)
    plans = []
    for name, circ in pool:
        # screen with the unsliced cost (no cut search) on the host planner
        q = pctx.plan(circ, precision="c64", max_intermediate_elems=1 << 62, path_mode="greedy")
        fl = q.info().flops_per_amp
        q.close()
        if fl / (nominal_tflops * 1e12) > cap_gpu_s:
            plans.append((name, circ, None, fl, None))
            continue
        p = ctx.plan(circ, precision="c64", max_intermediate_elems=max_elems)
        fl = p.info().flops_per_amp
        if fl / (nominal_tflops * 1e12) > cap_gpu_s:
            p.close()
            plans.append((name, circ, None, fl, None))
            continue
        # service-time model: a call costs o + a * n (one and sixteen
        # bitstrings, synchronous); a served request is cut into work items
        # as the library does (about 4e13 flops, at most 1024 bitstrings,
        # slice ranges for single heavy bitstrings) and pays o per item
        b = bitstrings(circ.n, 16, 9000)
        ctx.amplitudes(p, b[:1])
        torch.cuda.synchronize()
        t = time.perf_counter(); ctx.amplitudes(p, b[:1]); t1 = time.perf_counter() - t
        t = time.perf_counter(); ctx.amplitudes(p, b); t16 = time.perf_counter() - t
        a = max((t16 - t1) / 15, 0.0)
        n_sl = int(p.info().n_slices)
        nb_item = int(min(1024, max(1, 4e13 // max(fl, 1.0))))
        ns_item = n_sl if nb_item > 1 else int(min(n_sl, max(1, 4e13 // max(fl / n_sl, 1.0))))
        plans.append((name, circ, p, fl, (max(t1 - a, 0.0), a, nb_item, -(-n_sl // ns_item))))
        print(f"[bench] serving pool: {name} planned, {p.info().n_slices} slices", file=sys.stderr, flush=True)
    pctx.close()
    reqs, rejected_work = [], 0
    for i in range(n_req):
        k = int(rng.integers(len(plans)))
        nb = int(min(1024, max(1, round(math.exp(rng.uniform(0, math.log(1024)))))))
        name, circ, p, fl, model = plans[k]
        if p is None or fl * nb / (nominal_tflops * 1e12) > cap_gpu_s:
            rejected_work += 1
            continue
        o, a, nb_item, chunks = model
        items = -(-nb // nb_item) * chunks
        reqs.append((k, bitstrings(circ.n, nb, 20000 + i), o * items + a * nb))
    mean_service = float(np.mean([r[2] for r in reqs]))
    rate = load / mean_service
    gaps = rng.exponential(1.0 / rate, size=len(reqs))
    torch.cuda.synchronize()
    handles, rejected_mem = [], 0
    t0 = time.perf_counter()
    t_next = t0
    for (k, bits, _), gap in zip(reqs, gaps):
        t_next += gap
        delay = t_next - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        try:
            handles.append((k, ctx.submit(plans[k][2], bits)))
        except T.TnsError as e:
            if e.name != "TNS_E_ADMISSION":
                raise
            rejected_mem += 1
    print(f"[bench] serving: {len(handles)} requests submitted", file=sys.stderr, flush=True)
    total_amps, lat, lat_sliced = 0, [], []
    for k, h in handles:
        h.wait()
        total_amps += h.bits.shape[0]
        lat.append(h.latency_ms()[0])
        if plans[k][2].info().n_slices > 1:
            lat_sliced.append(lat[-1])
    wall = time.perf_counter() - t0
    sliced_pool = [n for n, _, p, _, _ in plans if p is not None and p.info().n_slices > 1]
    for _, _, p, _, _ in plans:
        if p is not None:
            p.close()
    lat = np.array(lat)
    return {"mix": "20-53 qubits (grid / diagonal lattice), depths 6-12, 1-1024 bitstrings, c64",
            "arrivals": n_req, "served": len(handles), "served_sliced": len(lat_sliced),
            "rejected_work_cap": rejected_work, "rejected_memory": rejected_mem,
            "work_cap_gpu_s": cap_gpu_s, "max_intermediate_elems": max_elems,
            "pool": [n for n, _, _, _, _ in plans],
            "pool_sliced": sliced_pool,
            "pool_rejected": [n for n, _, p, _, _ in plans if p is None],
            "offered_load": load, "mean_service_ms": round(mean_service * 1e3, 2),
            "wall_s": round(wall, 2), "amps_per_s": round(total_amps / wall, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "p50_ms_sliced": round(float(np.percentile(lat_sliced, 50)), 3) if lat_sliced else None}


def bench_104(T, ctx, args, torch):
    """104 qubits on the 8x13 grid, 8 cycles: a few bitstrings of the
    256-bitstring batch timed in complex64, split-BF16 and complex128, with
    the complex64 and split-BF16 amplitudes compared to complex128."""
    from circuits import config
    out = {}
    circ, bits = config("grid8x13_d8")
    t = time.perf_counter()
    base = ctx.plan(circ, precision="c64")
    out["plan_s"] = round(time.perf_counter() - t, 2)
    ib = base.info()
    same = dict(split_cycle=int(ib.split_cycle), path=ib.path.tolist(), cuts=ib.cut_edges.tolist())
    out.update({"flops_per_amp": ib.flops_per_amp, "n_slices": int(ib.n_slices),
                "split": int(ib.split_cycle), "peak_elems": int(ib.peak_elems),
                "batch": int(len(bits))})
    nb = args.b104_bits
    amps = {}
    for prec in ("c64", "c64_bf16x3", "c128"):
        plan = base if prec == "c64" else ctx.plan(circ, precision=prec, **same)
        sub = bits[:nb if prec != "c128" else max(1, nb // 2)]
        ctx.amplitudes(plan, sub[:1])
        torch.cuda.synchronize()
        t = time.perf_counter()
        a, st = ctx.amplitudes(plan, sub, stats=True)
        dt = time.perf_counter() - t
        amps[prec] = a
        out[prec] = {"bitstrings_timed": int(len(sub)), "amps_per_s": round(len(sub) / dt, 4),
                     "est_s_per_batch": round(dt / len(sub) * len(bits), 1),
                     "tflops": round(ib.flops_per_amp * len(sub) / dt / 1e12, 2),
                     "gemm_tflops": round(st["gemm_flops"] / (st["ms_gemm"] * 1e-3) / 1e12, 2)
                     if st["ms_gemm"] else None,
                     "gemm_mfma_tflops": round(st["gemm_mfma_flops"] / (st["ms_gemm"] * 1e-3) / 1e12, 2)
                     if st["ms_gemm"] else None,
                     "ms_per_amp": {k: round(st[k] / len(sub), 1) for k in
                                    ("ms_total", "ms_gemm", "ms_permute", "ms_small", "ms_bra", "ms_merge")},
                     "permute_GBps": round(st["permute_bytes"] / (st["ms_permute"] * 1e-3) / 1e9, 1)
                     if st["ms_permute"] else None}
        if plan is not base:
            plan.close()
        print(f"[bench] grid8x13_d8 {prec}: {len(sub) / dt:.3f} amps/s", file=sys.stderr, flush=True)
    k = len(amps["c128"])
    for prec in ("c64", "c64_bf16x3"):
        out[prec]["rel_l2_vs_c128"] = rel_l2(amps["c128"], amps[prec][:k])
    base.close()
    return {"grid8x13_d8": out}


class _Skip(Exception):
    pass


def bench_53(T, ctx, args, torch):
    """53-qubit diagonal lattice.  Depth 10: full amplitudes of random
    bitstrings and a correlated batch (the 12 qubits the path absorbs last are
    left open, one contraction gives 4096 amplitudes).  Depth 12: one amplitude
    is ~1e17 flops, so a few slices of a contraction are timed (partial sums
    over a slice range) and the full contraction is extrapolated; complex64,
    split-BF16 and complex128 partial sums are compared."""
    from circuits import config, random_circuit, diagonal53, bitstrings
    out = {}
    k_open = 12

    def timed(plan, bits, slices=None):
        ctx.amplitudes(plan, bits[:1], slices=(0, 1) if slices else None)
        torch.cuda.synchronize()
        t = time.perf_counter()
        a, st = ctx.amplitudes(plan, bits, stats=True, slices=slices)
        return a, time.perf_counter() - t, st

    # ---- depth 10
    try:
        if args.d12_only:
            raise _Skip()
        c10 = random_circuit(diagonal53(), 10, 3)
        b10 = bitstrings(53, 64, 103)
        res = {}
        amps = {}
        single = {}
        for prec in ("c64", "c128"):
            p10 = ctx.plan(c10, precision=prec)
            amps[prec], dt, _ = timed(p10, b10)
            i10 = p10.info()
            single = i10
            res[prec] = {"amps_per_s": round(len(b10) / dt, 2),
                         "tflops": round(i10.flops_per_amp * len(b10) / dt / 1e12, 2)}
            p10.close()
        res["flops_per_amp"] = single.flops_per_amp
        res["c64_rel_l2_vs_c128"] = rel_l2(amps["c128"], amps["c64"])
        oq = [int(q) for q in single.path[-k_open:]]
        corr = {"open_qubits": oq, "amplitudes_per_contraction": 1 << k_open}
        ca = {}
        for prec in ("c64", "c128"):
            po = ctx.plan(c10, precision=prec, open_qubits=oq)
            ca[prec], dt, _ = timed(po, b10[:4])
            io = po.info()
            corr[prec] = {"amps_per_s": round(4 * (1 << k_open) / dt, 1),
                          "tflops": round(io.flops_per_amp * 4 / dt / 1e12, 2)}
            corr["flops_per_contraction"] = io.flops_per_amp
            po.close()
        corr["c64_rel_l2_vs_c128"] = rel_l2(ca["c128"].reshape(-1), ca["c64"].reshape(-1))
        res["correlated_batch"] = corr
        # frugal rejection sampling over correlated batches (M = 10)
        ps = ctx.plan(c10, precision="c64", open_qubits=oq)
        fixed = bitstrings(53, 8, 104)
        u = np.random.default_rng(105).random((len(fixed), 1 << k_open))
        ctx.sample_frugal(ps, fixed[:1], u[:1], 10.0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        acc, _ = ctx.sample_frugal(ps, fixed, u, 10.0)
        dt = time.perf_counter() - t
        res["frugal_sampling"] = {"m_bound": 10.0, "batches": int(len(fixed)),
                                  "candidates": int(acc.size), "accepted": int(acc.sum()),
                                  "accept_rate": round(float(acc.mean()), 5),
                                  "samples_per_s": round(float(acc.sum()) / dt, 1)}
        ps.close()
        out["diag53_d10"] = res
        print("[bench] diag53_d10 done", file=sys.stderr, flush=True)
    except _Skip:
        pass
    except Exception as e:
        out["diag53_d10"] = {"error": str(e)}

    # ---- depth 12
    try:
        if getattr(args, "no_d12", False):
            raise _Skip()
        c53, b53 = config("diag53_d12", n_bits=1)
        res = {}
        t = time.perf_counter()
        p64 = ctx.plan(c53, precision="c64")
        res["plan_s"] = round(time.perf_counter() - t, 2)
        i53 = p64.info()
        oq = [int(q) for q in i53.path[-k_open:]]
        legs = [(label, opts) for label, opts in (("single", {}), ("correlated_batch", {"open_qubits": oq}))
                if label in args.d12_legs.split(",")]
        precs = args.d12_precisions.split(",")
        for label, opts in legs:
            base = p64 if not opts else ctx.plan(c53, precision="c64", **opts)
            ib = base.info()
            same = dict(split_cycle=int(ib.split_cycle), path=ib.path.tolist(),
                        cuts=ib.cut_edges.tolist(), **opts)
            ns = int(ib.n_slices)
            nt = min(ns, args.d12_slices)
            per = 1 << len(opts.get("open_qubits", []))
            r = {"flops_per_contraction": ib.flops_per_amp, "amplitudes_per_contraction": per,
                 "n_slices": ns, "split": int(ib.split_cycle), "peak_elems": int(ib.peak_elems),
                 "slices_timed": nt}
            parts = {}
            for prec in precs:
                plan = base if prec == "c64" else ctx.plan(c53, precision=prec, **same)
                a, dt, st = timed(plan, b53, slices=(0, nt))
                parts[prec] = a.reshape(-1)
                est = dt / nt * ns
                r[prec] = {"s_per_slice": round(dt / nt, 3), "est_s_per_contraction": round(est, 1),
                           "est_amps_per_s": round(per / est, 5),
                           "tflops": round(ib.flops_per_amp * nt / ns / dt / 1e12, 2),
                           "gemm_tflops": round(st["gemm_flops"] / (st["ms_gemm"] * 1e-3) / 1e12, 2)
                           if st["ms_gemm"] else None,
                           "gemm_mfma_tflops": round(st["gemm_mfma_flops"] / (st["ms_gemm"] * 1e-3) / 1e12, 2)
                           if st["ms_gemm"] else None}
                if plan is not base:
                    plan.close()
                print(f"[bench] diag53_d12 {label} {prec}: {dt / nt:.2f} s/slice", file=sys.stderr, flush=True)
            for prec in parts:
                if prec != "c128" and "c128" in parts:
                    r[prec]["partial_rel_l2_vs_c128"] = rel_l2(parts["c128"], parts[prec])
            if opts:
                r["open_qubits"] = oq
                base.close()
            res[label] = r
        p64.close()
        out["diag53_d12"] = res
    except _Skip:
        pass
    except Exception as e:
        out["diag53_d12"] = {"error": str(e)}
    return out


def gemm_roofline(agg, precision, workload):
    """Roofline of the dominant kernel from the per-launch HIP events of the
    timed steps.  complex64: the three-multiplication GEMM k_gemm_3m, whose
    MFMA instructions execute 6 M K N real flops per complex product; its
    achieved rate and fraction are those executed flops over its launch time
    (the 8 M K N count of the complex product is reported beside them as
    credited_tflops).  Other precisions: every GEMM launch."""
    if precision == "c64" and agg.get("gemm3m_launches"):
        ms, n = agg["ms_gemm3m"], agg["gemm3m_launches"]
        ex, cr, by = agg["gemm3m_mfma_flops"], agg["gemm3m_flops"], agg["gemm3m_bytes"]
        kname = "k_gemm_3m (complex64 in three real products on FP32 MFMA, 6 M K N executed)"
    else:
        ms, n = agg["ms_gemm"], agg["gemm_launches"]
        ex, cr, by = agg["gemm_mfma_flops"], agg["gemm_flops"], agg["gemm_bytes"]
        kname = {"c64": "k_gemm_c64 MODE 1 (FP32 MFMA, real embedding)",
                 "c128": "k_gemm_f64 (FP64 MFMA)",
                 "c64_bf16x3": "k_gemm_c64 MODE 2 (split-BF16 x3, BF16 MFMA)",
                 "c64_bf16x6": "k_gemm_c64 MODE 3 (split-BF16 x6, BF16 MFMA)"}[precision]
    if not n or not ms:
        return None
    peak = PEAK_TFLOPS[precision]
    # executed MFMA flops over the peak of the instructions that run them
    # (split-BF16: 3 or 6 BF16 products per real product, dense BF16 peak)
    achieved = ex / (ms * 1e-3) / 1e12
    alg_launch = by / n
    src_hash = kernel_source_hash()
    traffic = measured_traffic(src_hash, workload, alg_launch / 2 ** 20) if precision == "c64" else None
    return {"bound": "mfma", "kernel": kname, "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
            "launches": int(n), "avg_launch_ms": round(ms / n, 4),
            "flops_per_launch": ex / n,
            "algorithmic_bytes_per_launch": alg_launch,
            "credited_tflops": round(cr / (ms * 1e-3) / 1e12, 3),
            "credited_flops_per_launch": cr / n,
            "all_gemm_launches": int(agg["gemm_launches"]),
            "all_gemm_ms_share_of_contract": round(agg["ms_gemm"] / agg["ms_contract"], 4)
            if agg.get("ms_contract") else None,
            "kernel_sha": src_hash}


def cpu_baseline_sliced(circ_full, lattice_sub, depth, seed, budget_s=4.0):
    """The oracle's dense complex128 state vector cannot hold 53 qubits
    (2^53 x 16 B = 128 PiB).  It is timed on a bounded sample of the same
    workload -- the first n sites of the same lattice, same depth, gate set
    and seed -- growing n while a pass stays short, once on every host thread
    and once on one thread, and each time is scaled to the full circuit by the
    state vector's own cost law: one pass over 2^N amplitudes per gate, so
    t(N) = t(n) * gates(N) / gates(n) * 2^(N - n)."""
    from oracle import sv
    from circuits import random_circuit
    sv.build()
    threads = sv.max_threads()
    n_full, g_full = circ_full.n, len(circ_full.gates)
    out = {}
    for label, th in (("all", 0), ("one", 1)):
        best = None
        for n in range(16, 31, 2):
            c = random_circuit(lattice_sub(n), depth, seed)
            t = time.perf_counter()
            sv.state(c, th)
            dt = time.perf_counter() - t
            best = (n, len(c.gates), dt)
            if dt * 4.4 > budget_s:   # the next size costs about 4x more
                break
        n, g, dt = best
        est = dt * g_full / g * 2.0 ** (n_full - n)
        out[label] = {"threads": threads if th == 0 else 1, "sample_qubits": n, "sample_gates": g,
                      "sample_s": round(dt, 3), "est_s_per_amp": est}
    a = out["all"]
    return {"value": 1.0 / a["est_s_per_amp"], "unit": "amplitudes/s", "cores": a["threads"],
            "kind": "oracle",
            "sample": (f"dense complex128 state vector of the first {a['sample_qubits']} sites of the "
                       f"same lattice at the same depth and seed ({a['sample_gates']} gates, all "
                       f"amplitudes in one pass) in {a['sample_s']} s on {a['threads']} threads; scaled "
                       f"to {n_full} qubits ({g_full} gates) as t * gates ratio * 2^(qubit difference): "
                       f"{a['est_s_per_amp']:.3e} s per pass, which yields every amplitude but needs "
                       f"2^{n_full} x 16 B of memory, so the oracle cannot run the workload itself"),
            "single_thread": {"value": 1.0 / out["one"]["est_s_per_amp"], **out["one"]},
            "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def headline_sliced(T, ctx, args, torch):
    """One whole amplitude of a sliced workload, its slices spread over the
    timed steps (see the module docstring).  With --open K, the K qubits the
    path absorbs last keep their output bit open: one contraction then yields
    the 2^K amplitudes of all bitstrings that agree elsewhere (a correlated
    batch, 4096 bitstrings at K = 12), computed whole the same way."""
    from circuits import config, diagonal53
    circ, bits = config(args.workload, n_bits=1)
    t = time.perf_counter()
    oq = None
    if args.open:
        base = T.Context(-1).plan(circ, precision=args.precision)
        oq = [int(q) for q in base.info().path[-args.open:]]
        base.close()
    plan = ctx.plan(circ, precision=args.precision, open_qubits=oq)
    t_plan = time.perf_counter() - t
    info = plan.info()
    per = 1 << len(oq or [])
    S, K = int(info.n_slices), args.steps
    if K > S:
        raise SystemExit(f"--steps {K} exceeds the plan's {S} slices: each step takes a range of slices")
    edges = np.linspace(0, S, K + 1).round().astype(int)
    ranges = [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:])]
    print(f"[bench] {args.workload}: {circ.n} qubits, split {info.split_cycle}, cuts "
          f"{info.cut_edges.tolist()}, {S} slices, {info.flops_per_amp:.4e} flop/amp, peak "
          f"{info.peak_elems} elems, plan {t_plan:.2f}s; {K} steps of {ranges[0][1] - ranges[0][0]}"
          f"-{max(b - a for a, b in ranges)} slices", file=sys.stderr, flush=True)

    warm_parts = {}
    for w in range(args.warmup):
        sl = w % S
        warm_parts[sl] = ctx.amplitudes(plan, bits, slices=(sl, sl + 1)).reshape(-1)
        print(f"[bench] warmup {w} (slice {sl}) done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg, amp, per_step = {}, np.zeros(per, np.complex128), []
    for i, (a, b) in enumerate(ranges):
        part, st = ctx.amplitudes(plan, bits, stats=True, slices=(a, b))
        amp += part.reshape(-1)
        for k, v in st.items():
            agg[k] = agg.get(k, 0) + v
        per_step.append(st["ms_total"])
        print(f"[bench] step {i}: slices [{a}, {b}) {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    covered = sum(b - a for a, b in ranges)
    assert covered == S and ranges[0][0] == 0 and ranges[-1][1] == S

    line = {
        "metric": "amplitudes/s + achieved TFLOP/s, c64-MFMA vs c128, 53q depth-12; p50/p99 latency",
        "value": round(per / dt, 8), "unit": "amplitudes/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(dt / K * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c64": "c64 (fp32 mfma)", "c128": "c128 (fp64 mfma)",
                  "c64_bf16x3": "c64 (split-bf16 x3)", "c64_bf16x6": "c64 (split-bf16 x6)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "qubits": circ.n, "cycles": circ.depth,
                   "circuit_seed": 3, "bitstring_seed": 103, "bitstrings": per,
                   "open_qubits": oq or [],
                   "precision": args.precision, "split_cycle": int(info.split_cycle),
                   "cut_edges": info.cut_edges.tolist(), "n_slices": S, "slices_timed": covered,
                   "slices_per_step": [ranges[0][1] - ranges[0][0], max(b - a for a, b in ranges)],
                   "peak_elems": int(info.peak_elems), "flops_per_amp": info.flops_per_amp},
        "s_per_contraction": round(dt, 3),
        "amplitude": [amp[0].real, amp[0].imag] if per == 1 else None,
        "amplitudes_sum_abs2": float(np.sum(np.abs(amp) ** 2)) if per > 1 else None,
        "achieved_tflops_whole_path": round(info.flops_per_amp / dt / 1e12, 3),
        "roofline": gemm_roofline(agg, args.precision, args.workload),
        "cpu_baseline": None,
        "breakdown_ms_per_step": {k: round(agg[k] / K, 3) for k in
                                  ("ms_bra", "ms_merge", "ms_contract", "ms_gemm", "ms_gemm3m",
                                   "ms_permute", "ms_small")},
        "step_ms_min_max": [round(min(per_step), 1), round(max(per_step), 1)],
    }

    if not args.no_compare and 0 in warm_parts and args.precision != "c128":
        # complex128 on the same split, path and cuts: one slice timed, and
        # its partial sum against the complex64 one of the warm-up
        same = dict(split_cycle=int(info.split_cycle), path=info.path.tolist(),
                    cuts=info.cut_edges.tolist(), open_qubits=oq)
        p2 = ctx.plan(circ, precision="c128", **same)
        t = time.perf_counter()
        ref = ctx.amplitudes(p2, bits, slices=(0, 1)).reshape(-1)
        t2 = time.perf_counter() - t
        got = warm_parts[0]
        line["c128"] = {"s_per_slice": round(t2, 3), "est_s_per_contraction": round(t2 * S, 1),
                        "slice0_partial": [ref[0].real, ref[0].imag],
                        "slice0_rel_l2_c64_vs_c128": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))}
        p2.close()
        print(f"[bench] c128 slice 0: {t2:.2f} s", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_sliced(circ, lambda n: diagonal53().sub(n), 12, 3)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    plan.close()
    return line


def slice_range_only(T, ctx, args, torch):
    """Partial sum over one slice range of the headline amplitude (reference
    runs, e.g. complex128 in pieces)."""
    from circuits import config
    circ, bits = config(args.workload, n_bits=1)
    a, b = (int(x) for x in args.slice_range.split(":"))
    plan = ctx.plan(circ, precision=args.precision)
    info = plan.info()
    # in pieces of four slices, each reported as it ends; the pieces' partial
    # sums are added in FP64 in slice order
    t = time.perf_counter()
    total, gf, gms = 0.0 + 0.0j, 0.0, 0.0
    for c0 in range(a, b, 4):
        c1 = min(b, c0 + 4)
        part, st = ctx.amplitudes(plan, bits, stats=True, slices=(c0, c1))
        total += complex(part[0])
        gf += st["gemm_mfma_flops"]
        gms += st["ms_gemm"]
        print(f"[bench] slices [{c0}, {c1}) done, {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - t
    out = {"workload": args.workload, "precision": args.precision, "slices": [a, b],
           "n_slices": int(info.n_slices), "split_cycle": int(info.split_cycle),
           "cut_edges": info.cut_edges.tolist(), "partial": [total.real, total.imag],
           "s": round(dt, 3), "s_per_slice": round(dt / (b - a), 3),
           "gemm_tflops_executed": round(gf / (gms * 1e-3) / 1e12, 2) if gms else None}
    plan.close()
    return out


def bench_batch(T, ctx, args, torch, workload, precision="c64", steps=3, warmup=1, n_bits=None,
                compare=True, cpu=True, compare_bits=128, chunk=0):
    """A bitstring batch per step (workloads that need no cuts, e.g. the
    25-qubit grid): amplitudes/s, GEMM rates, the precision report against
    complex128 and split-BF16 on the first compare_bits bitstrings, and the
    oracle's state vector beside it.  chunk > 0 runs each step's batch in
    calls of that many bitstrings, each reported as it ends (long batches)."""
    from circuits import config
    circ, bits = config(workload, n_bits=n_bits)
    plan = ctx.plan(circ, precision=precision)
    info = plan.info()
    for w in range(warmup):
        ctx.amplitudes(plan, bits)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg, amps = {}, None
    pieces = [(a, min(len(bits), a + chunk)) for a in range(0, len(bits), chunk)] if chunk else [(0, len(bits))]
    for s in range(steps):
        got = []
        for a, b in pieces:
            part, st = ctx.amplitudes(plan, bits[a:b], stats=True)
            got.append(part)
            for k, v in st.items():
                agg[k] = agg.get(k, 0) + v
            if chunk:
                print(f"[bench] {workload} step {s}: bitstrings [{a}, {b}) done, {time.perf_counter() - t0:.1f} s",
                      file=sys.stderr, flush=True)
        amps = np.concatenate(got)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_amp = steps * len(bits)
    out = {"qubits": circ.n, "cycles": circ.depth, "bitstrings_per_step": int(len(bits)),
           "precision": precision, "split_cycle": int(info.split_cycle), "slices": int(info.n_slices),
           "flops_per_amp": info.flops_per_amp, "steps": steps,
           "amps_per_s": round(n_amp / dt, 3), "ms_per_step": round(dt / steps * 1e3, 3),
           "achieved_tflops_whole_path": round(info.flops_per_amp * n_amp / dt / 1e12, 3),
           "roofline": gemm_roofline(agg, precision, workload),
           "breakdown_ms_per_step": {k: round(agg[k] / steps, 3) for k in
                                     ("ms_bra", "ms_merge", "ms_contract", "ms_gemm", "ms_gemm3m",
                                      "ms_permute", "ms_small")}}
    if compare and precision == "c64":
        sub = bits[:min(len(bits), compare_bits)]
        p2 = ctx.plan(circ, precision="c128")
        ctx.amplitudes(p2, sub[:4])
        t = time.perf_counter()
        a2 = ctx.amplitudes(p2, sub)
        out["c128_amps_per_s"] = round(len(sub) / (time.perf_counter() - t), 3)
        p2.close()
        for sp in ("c64_bf16x3", "c64_bf16x6"):
            p3 = ctx.plan(circ, precision=sp)
            ctx.amplitudes(p3, sub[:4])
            t = time.perf_counter()
            a3 = ctx.amplitudes(p3, sub)
            out[sp] = {"amps_per_s": round(len(sub) / (time.perf_counter() - t), 3),
                       "rel_l2_vs_c128": rel_l2(a2, a3), "f_xeb": xeb(a2, a3, circ.n)}
            p3.close()
        a1 = amps[:len(sub)]
        out["c64_vs_c128"] = {"rel_l2": rel_l2(a2, a1),
                              "max_scaled": float(np.abs(a1 - a2).max() / (np.linalg.norm(a2) / np.sqrt(len(a2)))),
                              "f_xeb": xeb(a2, a1, circ.n),
                              "f_ovl": float(abs(np.vdot(a2, a1)) ** 2 / (np.vdot(a2, a2).real * np.vdot(a1, a1).real))}
    if cpu:
        from oracle import sv
        sv.build()
        res = {}
        for label, th in (("all", 0), ("one", 1)):
            t = time.perf_counter()
            ref = sv.amplitudes(circ, bits, th)
            tc = time.perf_counter() - t
            res[label] = {"amps_per_s": round(len(bits) / tc, 3), "s": round(tc, 3),
                          "threads": sv.max_threads() if th == 0 else 1}
        out["cpu_oracle"] = {**res, "cpu_model": cpu_model(),
                             "sample": f"one dense complex128 state-vector pass (all 2^{circ.n} "
                                       f"amplitudes, the {len(bits)} requested read out)"}
        out["oracle_check_rel_l2"] = rel_l2(ref, amps)
    plan.close()
    return out


LEGS = ("grid5x5_d10", "diag53_d10", "diag53_d12_slices", "grid8x13_d8", "serving")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16,
                    help="timed steps; the headline splits its slices over them")
    ap.add_argument("--warmup", type=int, default=1, help="warm-up steps (one slice each on the headline)")
    ap.add_argument("--workload", default="diag53_d12",
                    help="diag53_d12 (headline: one whole sliced amplitude), a batch workload "
                         "(grid3x4_d8, grid5x5_d10, grid8x13_d8), or legs (only the --legs)")
    ap.add_argument("--precision", default="c64", choices=["c64", "c128", "c64_bf16x3", "c64_bf16x6"])
    ap.add_argument("--bits", type=int, default=0, help="bitstrings per step of a batch workload")
    ap.add_argument("--compare-bits", type=int, default=128,
                    help="bitstrings of a batch workload compared against complex128 and split-BF16")
    ap.add_argument("--chunk-bits", type=int, default=0,
                    help="run a batch workload's steps in calls of this many bitstrings, reporting each")
    ap.add_argument("--slice-range", default="", help="A:B -- print the partial sum over slices [A, B) only")
    ap.add_argument("--open", type=int, default=0,
                    help="headline as a correlated batch: the last K qubits of the path left open (2^K amplitudes)")
    ap.add_argument("--legs", default="", help="comma list of extra legs: " + ",".join(LEGS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--d12-slices", type=int, default=2)
    ap.add_argument("--d12-only", action="store_true",
                    help="time only a few 53-qubit depth-12 slices (for kernel traces); prints that leg alone")
    ap.add_argument("--d12-precisions", default="c64,c64_bf16x3,c128")
    ap.add_argument("--d12-legs", default="single,correlated_batch")
    ap.add_argument("--b104-bits", type=int, default=4, help="bitstrings timed on the 104-qubit grid")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB of a plain device copy run first (byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU slice "
              "sharding is not implemented", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]
    for x in legs:
        if x not in LEGS:
            raise SystemExit(f"unknown leg {x}; choose from {','.join(LEGS)}")

    import torch
    import paper_2011_02621_amd as T

    ctx = T.Context(0)
    if args.copy_calibration:
        # a plain device copy of known size, for scaling HBM byte counters
        nbytes = args.copy_calibration << 20
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    if args.d12_only:
        res = bench_53(T, ctx, args, torch)
        print(json.dumps({"metric": "53-qubit depth-12 slice timing (partial contraction)", "n_gpus": 1,
                          "data": "synthetic", **res}))
        ctx.close()
        return
    if args.slice_range:
        print(json.dumps(slice_range_only(T, ctx, args, torch)))
        ctx.close()
        return

    if args.workload == "diag53_d12":
        line = headline_sliced(T, ctx, args, torch)
    elif args.workload == "legs":
        line = {"metric": "extra legs only (no headline)", "n_gpus": 1, "data": "synthetic"}
    else:
        r = bench_batch(T, ctx, args, torch, args.workload, args.precision, args.steps, args.warmup,
                        args.bits or None, compare=not args.no_compare, cpu=not args.no_cpu_baseline,
                        compare_bits=args.compare_bits, chunk=args.chunk_bits)
        cpu = r.pop("cpu_oracle", None)
        line = {"metric": "amplitudes/s + achieved TFLOP/s, c64-MFMA vs c128, 53q depth-12; p50/p99 latency",
                "value": r.pop("amps_per_s"), "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": r.pop("ms_per_step"), "higher_is_better": True,
                "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
                "config": {"workload": args.workload, **{k: r.pop(k) for k in
                           ("qubits", "cycles", "bitstrings_per_step", "precision", "split_cycle",
                            "slices", "flops_per_amp")}},
                "roofline": r.pop("roofline"),
                "cpu_baseline": None if cpu is None else
                {"value": cpu["all"]["amps_per_s"], "unit": "amplitudes/s", "cores": cpu["all"]["threads"],
                 "kind": "oracle", "sample": cpu["sample"] + f", {cpu['all']['s']} s",
                 "single_thread": cpu["one"], "cpu_model": cpu["cpu_model"]},
                **r}

    if "grid5x5_d10" in legs and args.workload != "grid5x5_d10":
        line["grid5x5_d10"] = bench_batch(T, ctx, args, torch, "grid5x5_d10", steps=3, warmup=1)
        print("[bench] grid5x5_d10 done", file=sys.stderr, flush=True)
    if "diag53_d10" in legs or "diag53_d12_slices" in legs:
        args.d12_only = "diag53_d10" not in legs
        args.no_d12 = "diag53_d12_slices" not in legs
        line.update(bench_53(T, ctx, args, torch))
    if "grid8x13_d8" in legs:
        try:
            line.update(bench_104(T, ctx, args, torch))
        except Exception as e:
            line["grid8x13_d8"] = {"error": str(e)}
    if "serving" in legs:
        line["serving"] = serving_run(T, ctx, torch)
        print("[bench] serving done", file=sys.stderr, flush=True)

    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
