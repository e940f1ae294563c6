#!/usr/bin/env python3
"""Benchmark of the twisted-mass Wilson Dslash and its Krylov solves on one MI355X.

One step is one pass of the whole hot path on one synthetic workload (default:
48^3 x 12 lattice, exp(i eps H) links at eps = 0.4, kappa = 0.16, a mu = 0.005,
periodic space / antiperiodic time, one Gaussian source):

  * a burst of even-odd Dslash hops in FP64/18, FP32/12 and FP16/12 storage,
    timed with HIP events on the stream they run on (the roofline kernel);
  * the plain FP64 even-odd CGNR solve to a true residual of 1e-10;
  * the mixed-precision solves (FP32/12 and FP16/12 inner Dslash, FP64
    reliable updates) to the same true residual.

`value` is whole-step throughput in the metric's unit: compulsory Dslash
bytes moved by every hop of the step (microbenchmark hops and every hop the
solvers applied, each at its own precision) divided by the step wall time.
The JSON line also carries the roofline of the FP64 Dslash kernel, the
time-to-solution of each solve and the FP64 CPU oracle's throughput on a
bounded sample of the same solve.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Wilson-tm Dslash GB/s (% HBM peak); mixed vs FP64 CG time to 1e-10 resid"
HBM_PEAK_GBS = 8000.0
# compulsory bytes per output site of one even-odd hop: input spinor, 8 links, output spinor
HOP_BYTES = {(64, 18): 192 + 8 * 144 + 192, (64, 12): 192 + 8 * 96 + 192,
             (32, 18): 96 + 8 * 72 + 96, (32, 12): 96 + 8 * 48 + 96, (16, 12): 52 + 8 * 24 + 52}
WORKLOADS = {
    "48x12": (48, 48, 48, 12),
    "32x8": (32, 32, 32, 8),
    "24x8": (24, 24, 24, 8),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(U, b, L, theta, kappa, mu, budget_s):
    """The oracle's FP64 even-odd CGNR on the same inputs, for as many
    iterations as fit the budget; reported as compulsory FP64 Dslash bytes per
    second with the same accounting as the GPU (4 hops of V/2 sites per
    iteration)."""
    import numpy as np

    from oracle import solvers as S
    from oracle import wilson as W

    A = lambda v: W.schur(U, v, L, theta, kappa, mu)  # noqa: E731
    Ah = lambda v: W.schur(U, v, L, theta, kappa, mu, dagger=True)  # noqa: E731
    bhat = W.eo_source(U, b, L, theta, kappa, mu)
    bn = float(np.linalg.norm(b.ravel()))
    t0 = time.perf_counter()
    S.cgnr(A, Ah, bhat, 1e-300, 1, bn, residual=lambda x: 1.0)
    t_one = time.perf_counter() - t0  # start (2 Schur) + 1 iteration (2 Schur)
    n = max(1, int(budget_s / max(t_one / 2, 1e-3)) - 1)
    t0 = time.perf_counter()
    S.cgnr(A, Ah, bhat, 1e-300, n, bn, residual=lambda x: 1.0)
    t = time.perf_counter() - t0
    t_iter = t / (n + 1)  # the start (residual, Mhat^+ r) costs the same 2 Schur applications as an iteration
    Vh = int(np.prod(L)) // 2
    gbs = 4 * Vh * HOP_BYTES[(64, 18)] / t_iter / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": W.num_threads(), "kind": "oracle",
            "sample": f"oracle FP64 even-odd CGNR on the same {L[0]}^3x{L[3]} inputs: start + {n} iterations "
                      f"in {t:.1f} s ({t_iter:.2f} s per iteration); FP64/18 Dslash bytes per iteration / time",
            "cpu_model": cpu_model()}


def recorded_traffic(workload):
    """HBM bytes per launch of the FP64 hop from the committed counter passes
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading for
    a 1 GiB copy), or None when they were taken on other kernel sources."""
    from paper_1411_5219_amd.profiling import kernel_source_digest

    path = os.path.join(ROOT, "profiles", f"dslash_fp64_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None, "no counter passes recorded for this workload"
    vals = {}
    for line in open(path):
        if " = " in line:
            k, v = line.split(" = ", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_digest") != kernel_source_digest():
        return None, "counters were taken on an older kernel"
    t = float(vals["read_bytes"]) + float(vals["write_bytes"])
    return t, f"{os.path.relpath(path, ROOT)}: read {float(vals['read_bytes']):.4g} B + write {float(vals['write_bytes']):.4g} B"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="48x12", choices=sorted(WORKLOADS))
    ap.add_argument("--hops", type=int, default=40, help="Dslash hops per precision per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--profile-hops", action="store_true",
                    help="only run the Dslash hops of each precision and a 1 GiB copy (for counter passes)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "the one-GPU kernel runs at the real per-GPU shape and the sharding design is documented.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from lattice_inputs import gauge_field, gaussian_spinor
    from paper_1411_5219_amd import fields, lqcd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    L = WORKLOADS[args.workload]
    theta = (0.0, 0.0, 0.0, math.pi)
    kappa, mu, eps, tol = 0.16, 0.005, 0.4, 1e-10
    V = int(np.prod(L))
    Vh = V // 2
    log(f"workload {L} V={V}; generating inputs")
    t0 = time.perf_counter()
    U = gauge_field(L, "exp", eps=eps, seed=1002)
    b = gaussian_spinor(L, seed=2002)
    log(f"inputs ready in {time.perf_counter() - t0:.1f}s")

    dev = torch.device("cuda:0")
    lat = fields.Lattice(L, theta, device=dev)
    Ug = {(64, 18): lat.gauge(U, 64, 18), (32, 12): lat.gauge(U, 32, 12), (16, 12): lat.gauge(U, 16, 12)}
    bd = lat.spinor(b)
    hop_in = {k: lat.parity_view(lat.spinor(b, k[0]), 1, k[0]) for k in Ug}
    hop_out = {k: lat.empty(lqcd.FIELD_SPINOR_PARITY, k[0]) for k in Ug}
    ops = {k: lqcd.op(kappa, mu, k[0], k[1]) for k in Ug}
    solves = {
        "fp64": lqcd.solve_params(tol=tol, maxiter=100000, eo=1, inner_prec=64),
        "mixed_fp32": lqcd.solve_params(tol=tol, maxiter=100000, eo=1, inner_prec=32, inner_recon=12),
        "mixed_fp16": lqcd.solve_params(tol=tol, maxiter=100000, eo=1, inner_prec=16, inner_recon=12),
    }
    o64 = ops[(64, 18)]
    ws = {n: lat.workspace(o64, p) for n, p in solves.items()}
    xs = {n: lat.zeros(lqcd.FIELD_SPINOR_FULL, 64) for n in solves}
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    def step(rec):
        byts = 0.0
        for k, Uk in Ug.items():
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(args.hops):
                lqcd.dslash_eo_apply(lat.g, ops[k], Uk, hop_in[k], hop_out[k], 0, lqcd.OP_HOP, 0, stream=stream)
            e1.record(stream)
            rec["hops"].setdefault(k, []).append((e0, e1))
            byts += args.hops * Vh * HOP_BYTES[k]
        for n, p in solves.items():
            fn = lqcd.cg_solve
            rc, info = fn(lat.g, o64, Ug[(64, 18)], bd, xs[n], p, ws[n], stream=stream)
            i = info[0]
            if rc != 0:
                raise RuntimeError(f"solve {n} failed: rc={rc} info={i}")
            rec["solves"].setdefault(n, []).append(i)
            inner = (p.inner_prec, p.inner_recon)
            byts += i["hops_outer"] * Vh * HOP_BYTES[(64, 18)]
            if p.inner_prec != 64:
                byts += i["hops_inner"] * Vh * HOP_BYTES[inner]
        return byts

    if args.profile_hops:
        # the roofline kernels, then a plain copy of known size that calibrates the byte counters
        for k, Uk in Ug.items():
            for _ in range(5):
                lqcd.dslash_eo_apply(lat.g, ops[k], Uk, hop_in[k], hop_out[k], 0, lqcd.OP_HOP, 0, stream=stream)
        a = torch.empty((1 << 30) // 4, dtype=torch.float32, device=dev)
        c = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_hops": True, "workload": list(L), "copy_bytes": 1 << 30}), flush=True)
        return

    log(f"warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        step({"hops": {}, "solves": {}})
    torch.cuda.synchronize()

    rec = {"hops": {}, "solves": {}}
    log(f"timing {args.steps} step(s)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_bytes = 0.0
    for s in range(args.steps):
        total_bytes += step(rec)
        log(f"step {s + 1}/{args.steps} enqueued/done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3

    hop_stats = {}
    for k, evs in rec["hops"].items():
        ms = sum(a.elapsed_time(b) for a, b in evs) / (len(evs) * args.hops)
        bpl = Vh * HOP_BYTES[k]
        gbs = bpl / (ms * 1e-3) / 1e9
        hop_stats[f"fp{k[0]}_{k[1]}"] = {"avg_launch_us": ms * 1e3, "bytes_per_launch": bpl, "GBps": gbs,
                                         "frac_hbm_peak": gbs / HBM_PEAK_GBS}
    main_k = hop_stats["fp64_18"]
    traffic, traffic_note = recorded_traffic(args.workload)
    solve_stats = {}
    for n, infos in rec["solves"].items():
        secs = [i["seconds"] for i in infos]
        solve_stats[n] = {"seconds_median": float(np.median(secs)), "iters": infos[-1]["iters"],
                          "reliable_updates": infos[-1]["reliable_updates"],
                          "true_resid": infos[-1]["true_resid"], "restarts": infos[-1]["restarts"]}
    if "fp64" in solve_stats:
        for n in ("mixed_fp32", "mixed_fp16"):
            if n in solve_stats:
                solve_stats[n]["speedup_vs_fp64"] = solve_stats["fp64"]["seconds_median"] / solve_stats[n]["seconds_median"]

    result = {
        "metric": METRIC,
        "value": total_bytes / elapsed / 1e9,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"twisted-mass Wilson even-odd Dslash + CGNR solves (FP64; mixed FP32/12 and "
                               f"FP16/12 with FP64 reliable updates) on {L[0]}^3x{L[3]}",
                   "lattice": list(L), "kappa": kappa, "mu": mu, "links": f"exp(i eps H), eps={eps}",
                   "bc": "periodic space, antiperiodic time", "tol": tol, "sources": 1,
                   "hops_per_precision_per_step": args.hops},
        "roofline": {"bound": "hbm", "kernel": "k_dslash_eo<64,18> (FP64 even-odd hop)",
                     "achieved": main_k["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": main_k["GBps"] / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_note": traffic_note,
                     "bytes_per_launch": main_k["bytes_per_launch"], "avg_launch_us": main_k["avg_launch_us"]},
        "dslash": hop_stats,
        "solves": solve_stats,
        "device": torch.cuda.get_device_properties(0).name,
    }
    if not args.no_cpu_baseline:
        log(f"CPU oracle baseline (budget {args.cpu_budget:.0f}s)")
        result["cpu_baseline"] = cpu_baseline(U, b, L, theta, kappa, mu, args.cpu_budget)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
