"""Benchmark: one step = one full ChASE solve (Lanczos, filter, QR,
Rayleigh-Ritz, residuals, locking) of the planted-spectrum Hermitian
problem, inputs resident in HBM before timing starts.

Default workload: n=20000 complex128, lowest 1200 eigenvalues geometric
(-1 + 10^(-4(1-i/1200))), the rest uniform in [0,1], Haar Q; nev=1000,
nex=300, degree 20, tol 1e-10; FP64 filter (and, as a second measurement on
the same matrix, the mixed FP32/FP64 filter).

Prints one JSON line (see the README of the bench contract in the design doc).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve s @resid≤1e-10 & filter TFLOP/s (% MFMA peak), FP64 vs mixed"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}

WORKLOADS = {
    "geometric20k": dict(kind="geometric", n=20000, nev=1000, nex=300, deg=20, tol=1e-10),
    "cluster121_30k": dict(kind="cluster121", n=30000, nev=1500, nex=500, deg=20, tol=1e-10),
    "uniform8k": dict(kind="uniform", n=8000, nev=200, nex=60, deg=20, tol=1e-10),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(H_host, V0_host, st, n, budget_s=20.0):
    """Time the CPU oracle's filter (numpy FP64) on a bounded sample of the
    same matrix: a block of columns of the start block at a fixed degree,
    grown until it costs a few seconds, then extrapolated to the solve's
    total filter work (the GPU run's Matvecs).  The extrapolation covers the
    filter only, so it is a lower bound on the oracle's solve time."""
    import numpy as np
    import threadpoolctl

    import oracle

    info = threadpoolctl.threadpool_info()
    threads = max([d.get("num_threads", 1) for d in info if d.get("user_api") == "blas"] or [1])
    cols, deg = 32, 2
    spent = 0.0
    rate = None
    total_mv = 0
    t_total = 0.0
    while spent < budget_s:
        x = V0_host[:, :cols]
        degs = np.full(cols, deg)
        t0 = time.perf_counter()
        _, mv = oracle.chebyshev_filter(H_host, x, degs, st["b_sup"], st["mu_1"], st["mu_ne"])
        dt = time.perf_counter() - t0
        spent += dt
        total_mv += mv
        t_total += dt
        rate = total_mv / t_total
        if dt * 3 > budget_s - spent:
            break
        cols = min(cols * 2, V0_host.shape[1])
    mv_full = st["matvecs_fp64"] + st["matvecs_low"]
    flops_per_mv = 8.0 * n * n
    return {
        "value": mv_full / rate,
        "unit": "s (filter part of the solve, extrapolated)",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"oracle.chebyshev_filter on the benchmark matrix, {total_mv} matrix-vector "
                  f"products (column blocks of the start block, degree {deg}) in {t_total:.1f} s; "
                  f"scaled to the GPU solve's {mv_full} Matvecs",
        "filter_gflops": rate * flops_per_mv / 1e9,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="geometric20k", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="both", choices=["fp64", "fp32", "both"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_2205_02491_amd as pk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pk.lib()
    wl = WORKLOADS[args.workload]
    n, nev, nex = wl["n"], wl["nev"], wl["nex"]
    t0 = time.perf_counter()
    prob = gen.make_torch(wl["kind"], n, nev, nex, device="cuda")
    torch.cuda.synchronize()
    log(f"generated {args.workload} n={n} in {time.perf_counter() - t0:.1f} s")
    H, V0, S = prob["H"].contiguous(), prob["V0"], prob["S"]
    lam = prob["lam"]
    norm = max(abs(lam[0]), abs(lam[-1]))

    precs = ["fp64", "fp32"] if args.prec == "both" else [args.prec]
    results = {}
    for prec in precs:
        opts = pk.default_opts(filter_prec=pk.PREC_FP32 if prec == "fp32" else pk.PREC_FP64,
                               verbose=1 if args.verbose else 0)
        handle = pk.Handle(n, nev, nex, H.dtype, opts)
        for w in range(args.warmup):
            ev, vec, res, st = pk.chase_solve(H, nev, nex, wl["tol"], wl["deg"], V0, S,
                                              handle=handle)
            log(f"{prec} warmup {w}: {st['t_all']:.2f} s, {st['iterations']} it")
        torch.cuda.synchronize()
        times, stats = [], []
        t_start = time.perf_counter()
        for k in range(args.steps):
            ts = time.perf_counter()
            ev, vec, res, st = pk.chase_solve(H, nev, nex, wl["tol"], wl["deg"], V0, S,
                                              handle=handle)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
            stats.append(st)
            log(f"{prec} step {k}: {times[-1]:.2f} s, it={st['iterations']} "
                f"mv64={st['matvecs_fp64']} mvlow={st['matvecs_low']} "
                f"filter {st['filter_flops'] / st['t_filter_kernels'] / 1e12:.1f} TF")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        err = float(np.max(np.abs(ev - lam[:nev])))
        fl = sum(s["filter_flops"] for s in stats)
        kt = sum(s["t_filter_kernels"] for s in stats)
        launches = sum(s["filter_launches"] for s in stats)
        results[prec] = dict(
            solve_s=elapsed / args.steps, converged=bool(st["converged"]),
            max_resid=float(res.max()), max_eig_err_rel=err / norm,
            iterations=st["iterations"], matvecs_fp64=st["matvecs_fp64"],
            matvecs_low=st["matvecs_low"],
            filter_tflops=fl / kt / 1e12, filter_kernel_s=kt / args.steps,
            filter_launches=launches // args.steps,
            avg_launch_ms=kt / launches * 1e3, flops_per_launch=fl / launches,
            phases={k: st[k] for k in ("t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid")},
            qr_shifted=st["qr_shifted"], qr_householder=st["qr_householder"],
            stats=st)
        handle.close()

    main_prec = "fp64" if "fp64" in results else precs[0]
    r = results[main_prec]
    peak = PEAK_TFLOPS["fp64"]
    # dominant kernel: the FP64 Chebyshev-step GEMM (all FP64 filter launches)
    roof = {"bound": "mfma", "achieved": r["filter_tflops"], "peak": peak, "unit": "TFLOP/s",
            "frac": r["filter_tflops"] / peak, "traffic": None,
            "kernel": "gemm_kernel<c128,FP64,N,N,CHEB>",
            "avg_launch_ms": r["avg_launch_ms"], "flops_per_launch": r["flops_per_launch"]}
    out = {
        "metric": METRIC, "value": r["solve_s"], "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["solve_s"] * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if main_prec == "fp64" else "c64/c128",
        "data": "synthetic planted-spectrum Hermitian (seeded, generated on the GPU)",
        "config": {"workload": f"{args.workload}", "n": n, "nev": nev, "nex": nex,
                   "degree": wl["deg"], "tol": wl["tol"], "filter": main_prec,
                   "parallelism": "single GPU"},
        "filter_tflops": r["filter_tflops"], "filter_frac_peak": r["filter_tflops"] / peak,
        "iterations": r["iterations"], "matvecs": r["matvecs_fp64"] + r["matvecs_low"],
        "converged": r["converged"], "max_resid": r["max_resid"],
        "max_eig_err_rel": r["max_eig_err_rel"], "phases_s": r["phases"],
        "roofline": roof,
    }
    if "fp32" in results and main_prec != "fp32":
        m = results["fp32"]
        out["mixed"] = {k: m[k] for k in ("solve_s", "converged", "max_resid", "max_eig_err_rel",
                                          "iterations", "matvecs_fp64", "matvecs_low",
                                          "filter_tflops", "phases")}
        out["mixed"]["speedup_vs_fp64"] = r["solve_s"] / m["solve_s"]
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        Hh = H.cpu().numpy()
        V0h = V0.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(Hh, V0h, r["stats"], n)
        log(f"cpu baseline done in {time.perf_counter() - t0:.1f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
