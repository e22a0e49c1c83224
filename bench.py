#!/usr/bin/env python3
"""Benchmark: amplitudes/s of the tensor-network-states amplitude path on one
MI355X, with the dominant kernel's roofline and the CPU oracle beside it.

One step = one pass of the whole hot path over one batch of bitstrings:
bra evolution with SVD compression, overlap merge, slice gather, and every
permute + complex GEMM of the contraction path, with the FP64 slice sum.
Inputs are seeded synthetic random circuits (see circuits/); bitstrings are
uploaded as part of each step (they are small), tensors live in HBM.

Prints one JSON line.  Usage:
  python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision c64|c128]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# dense MFMA peaks of MI355X: FP32, FP64; split-BF16 GEMMs are priced against
# the FP32 peak for the same algorithmic (complex64) flops
# dense MFMA peaks: FP32 for complex64, FP64 for complex128; the split-BF16
# forms are priced at the FP32 peak for the same algorithmic flops (their
# executed BF16 rate is reported beside it)
PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6, "c64_bf16x3": 157.3, "c64_bf16x6": 157.3}
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the dominant GEMM, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs scaled by a plain-copy calibration (the summary and commands
# are in profiles/gemm_f32_grid5x5_d10_traffic.md).  Keyed by the sha256
# prefix of the kernel source the counters were taken on, by the plan (split
# cycle, flops per amplitude) and by the algorithmic bytes per launch (units
# per launch): a change to any of them makes the entry stale and the bench
# reports null.
MEASURED_TRAFFIC = {("c64", "grid5x5_d10", "3cef2c90df144854", "split2:4.799972e+11:5422MiB"): 5837.0 * 2 ** 20}


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


def serving_run(T, ctx, torch, n_req=100, pool_size=24, cap_gpu_s=5.0, nominal_tflops=100.0,
                load=0.7, seed=4, max_elems=1 << 32):
    """Continuous batching on the serving mix (complex64).  The pool's plans
    are compiled ahead and stay resident.  Admission: a request whose planned
    work (flops per amplitude x bitstrings) exceeds cap_gpu_s at
    nominal_tflops, or whose circuit needs cuts to fit max_elems, is rejected
    and counted; the library itself rejects requests that do not fit a
    serving slot's memory.  Bitstrings per request are log-uniform in
    1..1024.  Arrivals are Poisson at the rate that gives the stated offered
    load, from service times measured on the device before the run."""
    import math
    from circuits import bitstrings
    pool, rng = serving_pool(T, pool_size, seed)
    pctx = T.Context(-1)
    plans = []
    for name, circ in pool:
        # screen with the unsliced cost (no cut search) on the host planner
        q = pctx.plan(circ, precision="c64", max_intermediate_elems=1 << 62, path_mode="greedy")
        qi = q.info()
        fl, pk = qi.flops_per_amp, int(qi.peak_elems)
        q.close()
        if pk > max_elems or fl / (nominal_tflops * 1e12) > cap_gpu_s:
            plans.append((name, circ, None, fl, None))
            continue
        p = ctx.plan(circ, precision="c64")
        # service-time model o + a * n from one and four bitstrings
        b = bitstrings(circ.n, 4, 9000)
        ctx.amplitudes(p, b[:1])
        torch.cuda.synchronize()
        t = time.perf_counter(); ctx.amplitudes(p, b[:1]); t1 = time.perf_counter() - t
        t = time.perf_counter(); ctx.amplitudes(p, b); t4 = time.perf_counter() - t
        a = max((t4 - t1) / 3, 0.0)
        plans.append((name, circ, p, p.info().flops_per_amp, (max(t1 - a, 0.0), a)))
    pctx.close()
    reqs, rejected_work = [], 0
    for i in range(n_req):
        k = int(rng.integers(len(plans)))
        nb = int(min(1024, max(1, round(math.exp(rng.uniform(0, math.log(1024)))))))
        name, circ, p, fl, model = plans[k]
        if p is None or fl * nb / (nominal_tflops * 1e12) > cap_gpu_s:
            rejected_work += 1
            continue
        reqs.append((k, bitstrings(circ.n, nb, 20000 + i), model[0] + model[1] * nb))
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
            handles.append(ctx.submit(plans[k][2], bits))
        except T.TnsError as e:
            if e.name != "TNS_E_ADMISSION":
                raise
            rejected_mem += 1
    total_amps = 0
    lat = []
    for h in handles:
        h.wait()
        total_amps += h.bits.shape[0]
        lat.append(h.latency_ms()[0])
    wall = time.perf_counter() - t0
    for _, _, p, _, _ in plans:
        if p is not None:
            p.close()
    lat = np.array(lat)
    return {"mix": "20-53 qubits (grid / diagonal lattice), depths 6-12, 1-1024 bitstrings, c64",
            "arrivals": n_req, "served": len(handles), "rejected_work_cap": rejected_work,
            "rejected_memory": rejected_mem, "work_cap_gpu_s": cap_gpu_s,
            "pool": [n for n, _, _, _, _ in plans],
            "pool_rejected": [n for n, _, p, _, _ in plans if p is None],
            "offered_load": load, "mean_service_ms": round(mean_service * 1e3, 2),
            "wall_s": round(wall, 2), "amps_per_s": round(total_amps / wall, 2),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3)}


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
    except Exception as e:
        out["diag53_d12"] = {"error": str(e)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid5x5_d10")
    ap.add_argument("--precision", default="c64", choices=["c64", "c128", "c64_bf16x3", "c64_bf16x6"])
    ap.add_argument("--bits", type=int, default=0, help="bitstrings per step (0 = workload default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-d12", action="store_true", help="skip the 53-qubit depth-12 slice timing")
    ap.add_argument("--d12-slices", type=int, default=2)
    ap.add_argument("--d12-only", action="store_true",
                    help="time only the 53-qubit depth-12 slices (for kernel traces); prints that leg alone")
    ap.add_argument("--d12-precisions", default="c64,c64_bf16x3,c128")
    ap.add_argument("--d12-legs", default="single,correlated_batch")
    ap.add_argument("--no-104", action="store_true", help="skip the 104-qubit grid leg")
    ap.add_argument("--b104-bits", type=int, default=4, help="bitstrings timed on the 104-qubit grid")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="MiB of a plain device copy run first (byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU slice "
              "sharding is not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2011_02621_amd as T
    from circuits import config, random_circuit, diagonal53, bitstrings

    if args.d12_only:
        ctx = T.Context(0)
        res = bench_53(T, ctx, args, torch)
        print(json.dumps({"metric": "53-qubit depth-12 slice timing (partial contraction)", "n_gpus": 1,
                          "data": "synthetic", **res}))
        ctx.close()
        return

    if args.copy_calibration:
        # a plain device copy of known size, for scaling HBM byte counters
        nbytes = args.copy_calibration << 20
        x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    circ, bits = config(args.workload, n_bits=args.bits or None)
    n_q = circ.n
    ctx = T.Context(0)
    t_plan = time.perf_counter()
    plan = ctx.plan(circ, precision=args.precision)
    t_plan = time.perf_counter() - t_plan
    info = plan.info()
    print(f"[bench] {args.workload}: {n_q} qubits, {len(bits)} bitstrings, split {info.split_cycle}, "
          f"{info.flops_per_amp:.3e} flop/amp, {info.n_slices} slices, peak {info.peak_elems} elems, "
          f"plan {t_plan:.2f}s", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        ctx.amplitudes(plan, bits)
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg = {}
    amps = None
    for s in range(args.steps):
        amps, st = ctx.amplitudes(plan, bits, stats=True)
        for k, v in st.items():
            agg[k] = agg.get(k, 0) + v
        print(f"[bench] step {s}: {st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_amp = args.steps * len(bits)
    value = n_amp / dt
    tflops = info.flops_per_amp * n_amp / dt / 1e12

    # algorithmic rate (8 M K N per complex product, the path's flop count,
    # also credited to the three-multiplication form) and, beside it, the rate
    # of the flops the MFMA instructions execute (6 M K N for that form)
    gemm_tflops = agg["gemm_flops"] / (agg["ms_gemm"] * 1e-3) / 1e12 if agg.get("ms_gemm") else 0.0
    mfma_tflops = agg["gemm_mfma_flops"] / (agg["ms_gemm"] * 1e-3) / 1e12 if agg.get("ms_gemm") else 0.0
    avg_gemm_ms = agg["ms_gemm"] / max(agg["gemm_launches"], 1)
    kname = {"c64": "k_gemm_3m + k_gemm_c64 MODE 1 (FP32 MFMA; three-multiplication form on the wide steps)",
             "c128": "k_gemm_f64 (FP64 MFMA)",
             "c64_bf16x3": "k_gemm_c64 (MODE 2, split-BF16 x3, BF16 MFMA)",
             "c64_bf16x6": "k_gemm_c64 (MODE 3, split-BF16 x6, BF16 MFMA)"}[args.precision]
    import hashlib
    src = os.path.join(ROOT, "paper_2011_02621_amd", "csrc", "kernels_contract.hip")
    src_hash = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    alg_launch = agg["gemm_bytes"] / max(agg["gemm_launches"], 1)
    plan_key = f"split{info.split_cycle}:{info.flops_per_amp:.6e}:{alg_launch / 2 ** 20:.0f}MiB"
    traffic = MEASURED_TRAFFIC.get((args.precision, args.workload, src_hash, plan_key))
    roofline = {"bound": "mfma", "kernel": kname,
                "achieved": round(gemm_tflops, 3), "peak": PEAK_TFLOPS[args.precision],
                "unit": "TFLOP/s", "frac": round(gemm_tflops / PEAK_TFLOPS[args.precision], 4),
                "traffic": traffic,
                "executed_tflops": round(mfma_tflops, 3),
                "executed_frac": round(mfma_tflops / PEAK_TFLOPS[args.precision], 4),
                "algorithmic_bytes_per_launch": agg["gemm_bytes"] / max(agg["gemm_launches"], 1),
                "avg_launch_ms": round(avg_gemm_ms, 4),
                "launches": int(agg["gemm_launches"]),
                "flops_per_launch": agg["gemm_flops"] / max(agg["gemm_launches"], 1),
                "mfma_flops_per_launch": agg["gemm_mfma_flops"] / max(agg["gemm_launches"], 1)}
    breakdown = {k: round(agg[k] / args.steps, 3) for k in
                 ("ms_bra", "ms_merge", "ms_contract", "ms_gemm", "ms_permute", "ms_small")}
    if agg.get("ms_permute"):
        breakdown["permute_GBps"] = round(agg["permute_bytes"] / (agg["ms_permute"] * 1e-3) / 1e9, 1)

    extra = {}
    if not args.no_compare:
        # c128 reference on a subset: precision report and c128 throughput
        other = "c128" if args.precision == "c64" else "c64"
        sub = bits[:min(len(bits), 128)]
        p2 = ctx.plan(circ, precision=other)
        ctx.amplitudes(p2, sub[:4])
        t = time.perf_counter()
        a2 = ctx.amplitudes(p2, sub)
        t2 = time.perf_counter() - t
        a1 = amps[:len(sub)]
        ref, test = (a2, a1) if other == "c128" else (a1, a2)
        extra[f"{other}_amps_per_s"] = round(len(sub) / t2, 3)
        if args.precision == "c64":
            for sp in ("c64_bf16x3", "c64_bf16x6"):
                p3 = ctx.plan(circ, precision=sp)
                ctx.amplitudes(p3, sub[:4])
                t = time.perf_counter()
                a3 = ctx.amplitudes(p3, sub)
                t3 = time.perf_counter() - t
                extra[sp] = {"amps_per_s": round(len(sub) / t3, 3), "rel_l2_vs_c128": rel_l2(a2, a3),
                             "f_xeb": xeb(a2, a3, n_q)}
                p3.close()
        extra["c64_vs_c128"] = {"rel_l2": rel_l2(ref, test),
                                "max_scaled": float(np.abs(test - ref).max() / (np.linalg.norm(ref) / np.sqrt(len(ref)))),
                                "f_xeb": xeb(ref, test, n_q),
                                "f_ovl": float(abs(np.vdot(ref, test)) ** 2 / (np.vdot(ref, ref).real * np.vdot(test, test).real))}
        print(f"[bench] {other} done", file=sys.stderr, flush=True)

    if not args.no_d12:
        extra.update(bench_53(T, ctx, args, torch))

    if not args.no_104:
        try:
            extra.update(bench_104(T, ctx, args, torch))
        except Exception as e:
            extra["grid8x13_d8"] = {"error": str(e)}

    if not args.no_serving:
        extra["serving"] = serving_run(T, ctx, torch)
        print(f"[bench] serving done", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import sv
        sv.build()
        threads = sv.max_threads()
        t = time.perf_counter()
        ref = sv.amplitudes(circ, bits)
        tc = time.perf_counter() - t
        cpu = {"value": round(len(bits) / tc, 3), "unit": "amplitudes/s", "cores": threads,
               "kind": "oracle",
               "sample": f"one dense complex128 state-vector pass over {args.workload} "
                         f"(all 2^{n_q} amplitudes, the {len(bits)} requested read out), {tc:.2f} s"}
        extra["oracle_check_rel_l2"] = rel_l2(ref, amps)

    line = {
        "metric": "amplitudes/s + achieved TFLOP/s, c64-MFMA vs c128, 53q depth-12; p50/p99 latency",
        "value": round(value, 4), "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"c64": "c64 (fp32 mfma)", "c128": "c128 (fp64 mfma)",
                  "c64_bf16x3": "c64 (split-bf16 x3)", "c64_bf16x6": "c64 (split-bf16 x6)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "qubits": n_q, "cycles": circ.depth,
                   "bitstrings_per_step": int(len(bits)), "precision": args.precision,
                   "split_cycle": int(info.split_cycle), "slices": int(info.n_slices),
                   "flops_per_amp": info.flops_per_amp},
        "achieved_tflops_whole_path": round(tflops, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "breakdown_ms_per_step": breakdown,
        **extra,
    }
    print(json.dumps(line))
    plan.close()
    ctx.close()


if __name__ == "__main__":
    main()
