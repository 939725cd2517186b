"""Benchmark: one step = one full ChASE solve (Lanczos, filter, QR,
Rayleigh-Ritz, residuals, locking) of the planted-spectrum Hermitian
problem, inputs resident in HBM before timing starts.

Default workload: n=20000 complex128, lowest 1200 eigenvalues geometric
(-1 + 10^(-4(1-i/1200))), the rest uniform in [0,1], Haar Q; nev=1000,
nex=300, degree 20, tol 1e-10; FP64 filter (and, as further measurements on
the same matrix, the mixed filters: FP32 products, split-BF16 products with
three terms, and the two-term split-BF16 mode).

Prints one JSON line: the FP64 solve time as the value, the filter's
algorithmic TFLOP/s against the FP64 MFMA peak (roofline), the Lanczos block
GEMV's GB/s against the HBM peak, the mixed-precision solves on the same
matrix, the CPU oracle timed on the same host (its solve estimated from timed
pieces of the same matrix, and a complete small solve beside the library's),
the vendor's own GEMM rates on the same GPU (hipBLASLt BF16, rocBLAS FP64
and complex128) as the practical ceiling beside the published peaks, and a
second block on the mixed-precision workload: n=30000 complex128, lowest 2000
eigenvalues those of the (1-2-1) matrix of order 30000, the rest uniform up
to 10, nev=1500, nex=500, solved once in each filter mode.
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
# dense MFMA peaks of one MI355X (TFLOP/s) for the arithmetic each filter
# mode executes: FP64, FP32, BF16 (split-BF16 runs on the BF16 matrix cores)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16x2": 2500.0,
               # FP64-accurate products on the INT8 matrix cores: the algorithmic
               # rate is set against the FP64 peak it replaces
               "fp64i8": 78.6, "bf16x2i8": 2500.0}
# FP64 filter products on the INT8 matrix cores (chase_opts.fp64_emulation):
# the moduli of each mode, the INT8 operations per algorithmic FLOP
# (complex: three real products per modulus, 2 n^2 k each, against 8 n^2 k)
# and the dense INT8 peak
EMU_MODULI = {"fp64i8": 14, "bf16x2i8": 14}
INT8_PEAK_TOPS = 5000.0
# executed MFMA FLOPs per algorithmic FLOP (8 per complex multiply-add):
# three real products per complex product (Gauss) for FP64/FP32, twelve BF16
# products (four real products x hi*hi, hi*lo, lo*hi) for split-BF16, eight
# for its two-term form (the block as bf16: hi*hi, lo*hi)
EXEC_PER_ALGO = {"fp64": 0.75, "fp32": 0.75, "bf16x3": 3.0, "bf16x2": 2.0,
                 "fp64i8": 3 * 14 * 2 / 8.0, "bf16x2i8": 2.0}
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x2": 3, "fp64i8": 0, "bf16x2i8": 3}
# dense eigensolver of the Rayleigh-Ritz step (chase_opts.eig_solver)
EIG_CODE = {"auto": 0, "library": 1, "jacobi": 2}
EIG_CHOICE = "auto"
KERNEL_NAME = {
    "fp64": "gemm_kernel<double,double,complex,N,N,CHEB,8,Gauss,128x64> (FP64 MFMA 16x16x4)",
    "fp32": "gemm_kernel<float,float,complex,N,N,CHEB,16,Gauss,128x64> (FP32 MFMA 16x16x4)",
    "bf16x3": "gemm_bf16x3_kernel<complex, 3 terms> (BF16 MFMA 32x32x16, 256x128 tiles)",
    "bf16x2": "gemm_bf16x3_kernel<complex, 2 terms; start pass 3 terms> (BF16 MFMA 32x32x16, "
              "256x128 tiles)",
    "fp64i8": "FP64 step on INT8: 42 rocBLAS INT8 GEMMs (14 moduli x 3 Gauss products) + "
              "crt_cheb_k (Garner reconstruction, Chebyshev epilogue); executed = INT8 ops",
    "bf16x2i8": "gemm_bf16x3_kernel<complex, 2 terms; start pass 3 terms> (BF16 MFMA 32x32x16); "
                "FP64 steps and Rayleigh-Ritz H Q on INT8 (14 moduli)",
}

# HBM bytes per filter launch from rocprofv3 PMC runs (FETCH_SIZE x 2.0 and
# WRITE_SIZE x 1.0, calibrated on a 1 GiB copy), valid only for the GEMM
# source they were measured on (sha256 prefix of csrc/gemm.hip).
MEASURED_TRAFFIC = {
    ("geometric20k", "fp64"): {"fetch_gb": 54.55, "write_gb": 0.416, "columns": 1300,
                               "gemm_sha256": "c0bdc1127171d3e2",
                               "source": "profiles/filter_fp64_geometric20k_hbm_traffic.md"},
}

WORKLOADS = {
    "geometric20k": dict(kind="geometric", n=20000, nev=1000, nex=300, deg=20, tol=1e-10),
    "cluster121_30k": dict(kind="cluster121", n=30000, nev=1500, nex=500, deg=20, tol=1e-10),
    "reflectors100k": dict(kind="reflectors", n=100000, nev=2000, nex=600, deg=20, tol=1e-10),
    "diff8k": dict(kind="uniform", n=8000, nev=200, nex=60, deg=20, tol=1e-10),
    "table2": dict(kind="table2", n=20000, nev=1500, nex=500, deg=20, tol=1e-10),
}

# The paper's eigen-type tests (Table 2, GPU rows: one node of 4 NVIDIA A100,
# FP64, real symmetric n=20000, nev=1500, nex=500): iterations, Matvecs and
# seconds for All, Lanczos, Filter, QR, RR and Resid, as context for the
# table2 workload (the same matrix types on one MI355X).
PAPER_TABLE2_GPU = {
    "121": (13, 466614, 31.39, 0.58, 14.38, 2.59, 8.41, 5.24),
    "geometric": (8, 285192, 18.57, 0.58, 8.76, 1.58, 4.58, 2.96),
    "uniform": (5, 163562, 11.79, 0.58, 5.06, 1.00, 3.11, 1.96),
    "wilkinson": (8, 246924, 17.22, 0.57, 7.63, 1.59, 4.45, 2.90),
}


def exec_per_algo(prec, st, deg, ne, cplx=True):
    """Executed MFMA FLOPs per algorithmic FLOP over a solve's filter launches
    of its own precision.  The two-term split-BF16 mode runs the start block's
    low-precision steps with three terms (deg - fp64_tail steps over all ne
    columns) and the defect-form passes with two."""
    if prec == "fp64i8" and not cplx:
        return float(EMU_MODULI[prec])  # one real product per modulus, 2 n^2 k each
    if prec not in ("bf16x2", "bf16x2i8") or st["matvecs_low"] == 0:
        return EXEC_PER_ALGO[prec]
    d0 = deg + (deg & 1)
    start = min(st["matvecs_low"], (d0 - st["fp64_tail"]) * ne)
    return (EXEC_PER_ALGO["bf16x3"] * start
            + EXEC_PER_ALGO["bf16x2"] * (st["matvecs_low"] - start)) / st["matvecs_low"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    """CPU model, logical CPU count and BLAS thread pool of the host that runs
    the oracle."""
    import threadpoolctl

    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = [{k: d.get(k) for k in ("internal_api", "num_threads", "version", "architecture")}
            for d in threadpoolctl.threadpool_info() if d.get("user_api") == "blas"]
    threads = max([b["num_threads"] or 1 for b in blas] or [1])
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "blas": blas}, int(threads)


def cpu_baseline(H_host, V0_host, S_host, st, n, ne, budget_s=12.0):
    """The CPU oracle (numpy FP64) timed on the same matrix.  A full oracle
    solve of this size takes minutes, so its pieces are timed once each and
    added up as the solve runs them:
    - filter: oracle.chebyshev_filter on column blocks of the start block at
      degree 2, grown until the sample costs about budget_s, then scaled to
      the GPU solve's matrix-vector products;
    - Lanczos: a 3-step run from one start vector, scaled to the solve's
      runs x steps products;
    - QR, Rayleigh-Ritz and residual: one full-size call each
      (oracle.qr_locked on the n x ne start block, oracle.rayleigh_ritz on the
      result, oracle.residual_norms on the Ritz vectors), times the GPU solve's
      iterations (exact for a one-iteration solve; later iterations of a
      longer solve work on fewer active columns)."""
    import numpy as np

    import oracle

    info, threads = host_info()
    cols, deg = min(32, V0_host.shape[1]), 2
    spent = 0.0
    total_mv = 0
    t_total = 0.0
    while spent < budget_s:
        x = V0_host[:, :cols]
        degs = np.full(x.shape[1], deg)
        t0 = time.perf_counter()
        _, mv = oracle.chebyshev_filter(H_host, x, degs, st["b_sup"], st["mu_1"], st["mu_ne"])
        dt = time.perf_counter() - t0
        spent += dt
        total_mv += mv
        t_total += dt
        if dt * 3 > budget_s - spent:
            break
        cols = min(cols * 2, V0_host.shape[1])
    rate = total_mv / t_total
    mv_full = st["matvecs_fp64"] + st["matvecs_low"]
    t_filter = mv_full / rate
    t0 = time.perf_counter()
    oracle.lanczos_runs(H_host, S_host[:, :1], 3)
    t_lz = (time.perf_counter() - t0) / 3 * 4 * 25
    t0 = time.perf_counter()
    q = oracle.qr_locked(V0_host[:, :0], V0_host[:, :ne])
    t1 = time.perf_counter()
    theta, va = oracle.rayleigh_ritz(H_host, q)
    t2 = time.perf_counter()
    oracle.residual_norms(H_host, va, theta, 1.0)
    t3 = time.perf_counter()
    t_iter = t3 - t0
    it = st["iterations"]
    est = t_lz + t_filter + it * t_iter
    flops_per_mv = 8.0 * n * n
    return {
        "value": est,
        "unit": "s (oracle solve, estimated from timed pieces)",
        "cores": threads,
        "kind": "oracle",
        "sample": f"oracle pieces on the benchmark matrix: chebyshev_filter {total_mv} "
                  f"matrix-vector products (column blocks of the start block, degree {deg}) in "
                  f"{t_total:.1f} s, scaled to the GPU solve's {mv_full} Matvecs "
                  f"({t_filter:.1f} s); Lanczos 3 steps scaled to 4 x 25 ({t_lz:.1f} s); one "
                  f"full-size qr_locked + rayleigh_ritz + residual_norms ({t_iter:.1f} s) x "
                  f"{it} iteration(s)",
        "filter_gflops": rate * flops_per_mv / 1e9,
        "pieces_s": {"filter": t_filter, "lanczos": t_lz, "qr": t1 - t0, "rr": t2 - t1,
                     "resid": t3 - t2},
        "host": info,
    }


def small_solve_pair(pk):
    """The oracle's complete solve of the small workload (n=1000 complex128,
    lambda i.i.d. uniform in [-1, 1], nev=100, nex=40, degree 20, tol 1e-10)
    timed beside the library's solve of the same bytes (median of 5 after one
    warm-up)."""
    import numpy as np
    import torch

    import gen
    import oracle

    p = gen.make_uniform(n=1000, nev=100, nex=40)
    t0 = time.perf_counter()
    ev_o, _, _, st_o = oracle.solve(p.H, p.nev, p.nex, p.tol, p.deg, p.V0, p.S)
    t_oracle = time.perf_counter() - t0
    Hd = torch.from_numpy(p.H).cuda()
    V0, S = torch.from_numpy(p.V0).cuda(), torch.from_numpy(p.S).cuda()
    h = pk.Handle(p.H.shape[0], p.nev, p.nex, Hd.dtype, pk.default_opts())
    ts = []
    for k in range(6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, _, res, st = pk.chase_solve(Hd, p.nev, p.nex, p.tol, p.deg, V0, S, handle=h)
        torch.cuda.synchronize()
        if k:
            ts.append(time.perf_counter() - t0)
    h.close()
    norm = max(abs(p.lam[0]), abs(p.lam[-1]))
    return {"workload": "small (n=1000 c128, nev 100, nex 40)", "oracle_solve_s": t_oracle,
            "oracle_iterations": st_o.iterations, "oracle_matvecs": st_o.matvecs,
            "gpu_solve_s": float(np.median(ts)), "gpu_iterations": st["iterations"],
            "gpu_matvecs": st["matvecs_fp64"] + st["matvecs_low"],
            "max_eig_diff_rel": float(np.max(np.abs(ev - ev_o)) / norm),
            "max_resid": float(res.max())}


def independent_residual(H, vec, ev, prob):
    """max_a ||H v_a - lambda_a v_a||_2 computed without the library: with the
    factored form of Q for the reflector workload (H itself never read), else
    with torch's GEMM on the stored H."""
    import torch

    import gen
    lam_t = torch.tensor(ev, dtype=torch.float64, device=vec.device)
    v = vec.contiguous()
    if "U" in prob:
        planted = torch.tensor(prob["lam"], dtype=torch.float64, device=vec.device)
        hv = gen.apply_q(planted[:, None] * gen.apply_q(v, prob["U"], adjoint=True), prob["U"],
                         adjoint=False)
    else:
        hv = torch.matmul(H, v)
    r = hv - v * lam_t[None, :]
    return float(torch.linalg.vector_norm(r, dim=0).max())


def bench_diff(args, wl):
    """Differentiation workload: loss = sum_i w_i lambda_i + ||Y^H B||_F^2 with
    lambda from the solve and Y the filtered start block at frozen bounds and
    degrees; forward + backward time, and a central-difference check of the
    gradient along seeded Hermitian directions.  Second case per dtype: the
    same loss with Y the eigenvector block (eigenvector adjoint), checked
    against the planted first-order reference gradient."""
    import numpy as np
    import torch

    import gen
    import paper_2205_02491_amd as pk

    n, nev, nex = wl["n"], wl["nev"], wl["nex"]
    out = {"metric": "fwd+bwd s (differentiation workload)", "unit": "s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "higher_is_better": False,
           "data": "synthetic planted-spectrum (seeded numpy)", "vs_baseline": None,
           "config": {"workload": "diff8k", "n": n, "nev": nev, "nex": nex}, "cases": {}}
    for cplx in (True, False):
        p = gen.make_uniform(n=n, nev=nev, nex=nex, cplx=cplx, cfg=gen.CFG_DIFF8K)
        w, B = gen.loss_weights(gen.CFG_DIFF8K, nev, 16, n, cplx)
        Hd = torch.from_numpy(p.H).cuda()
        V0, S = torch.from_numpy(p.V0).cuda(), torch.from_numpy(p.S).cuda()
        Bt, wt = torch.from_numpy(B).cuda(), torch.from_numpy(w).cuda()
        _, _, _, st = pk.chase_solve(Hd, nev, nex, wl["tol"], wl["deg"], V0, S)
        frozen = (st["b_sup"], st["mu_1"], st["mu_ne"])
        deg = np.full(nev + nex, wl["deg"], dtype=np.int32)

        def loss_fn(Hx):
            lam, _ = pk.chase_eigh(Hx, nev, nex, wl["tol"], wl["deg"], V0, S)
            Y = pk.filtered_block(Hx, V0, deg, *frozen)
            return (wt * lam).sum() + torch.linalg.matrix_norm(Y.mH @ Bt) ** 2

        tf, tb = [], []
        for k in range(args.warmup + args.steps):
            H = Hd.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L = loss_fn(H)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if k >= args.warmup:
                tf.append(t1 - t0)
                tb.append(t2 - t1)
        G = H.grad
        errs = []
        h = 1e-6
        for sd in range(3):
            gE = np.random.Generator(np.random.PCG64(900 + sd))
            E = gen.gaussian(gE, (n, n), cplx)
            E = (E + E.conj().T) / 2
            E /= np.linalg.norm(E)
            Et = torch.from_numpy(E).cuda()
            with torch.no_grad():
                lp = float(loss_fn(Hd + h * Et))
                lm = float(loss_fn(Hd - h * Et))
            fd = (lp - lm) / (2 * h)
            an = float(torch.real(torch.sum(torch.conj(G) * Et)))
            errs.append(abs(fd - an) / max(abs(an), 1e-300))
        out["cases"]["c128" if cplx else "f64"] = {
            "fwd_s": float(np.median(tf)), "bwd_s": float(np.median(tb)),
            "fwd_bwd_s": float(np.median(tf) + np.median(tb)),
            "fd_rel_err_max": float(max(errs)), "iterations": st["iterations"]}
        log(f"diff {'c128' if cplx else 'f64'}: {out['cases']['c128' if cplx else 'f64']}")

        # the same loss with V the eigenvector block itself:
        # L = sum_i w_i lam_i + ||V^H B||_F^2 (phase invariant), backward through
        # chase_eigval_adjoint + chase_eigvec_adjoint; checked against the
        # first-order formula evaluated from the planted eigendecomposition
        def loss_vec(Hx):
            lam, V = pk.chase_eigh(Hx, nev, nex, wl["tol"], wl["deg"], V0, S)
            return (wt * lam).sum() + torch.linalg.matrix_norm(V.mH @ Bt) ** 2

        tf, tb = [], []
        for k in range(args.warmup + args.steps):
            H = Hd.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L = loss_vec(H)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            if k >= args.warmup:
                tf.append(t1 - t0)
                tb.append(t2 - t1)
        G = H.grad
        Q = torch.from_numpy(p.Q).cuda()
        lamt = torch.from_numpy(p.lam).cuda()
        Vq = Q[:, :nev]
        Gv = 2.0 * Bt @ (Bt.mH @ Vq)
        C = Q.mH @ Gv
        den = lamt[:nev][None, :] - lamt[:, None]
        idx = torch.arange(nev, device="cuda")
        den[idx, idx] = 1.0
        D = C / den
        D[idx, idx] = 0.0
        A = Q @ (D @ Vq.mH) + (Vq * wt[None, :].to(Vq.dtype)) @ Vq.mH
        ref = (A + A.mH) / 2
        ref_err = float(torch.linalg.matrix_norm(G - ref) / torch.linalg.matrix_norm(ref))
        out["cases"][("c128" if cplx else "f64") + "_eigvec"] = {
            "fwd_s": float(np.median(tf)), "bwd_s": float(np.median(tb)),
            "fwd_bwd_s": float(np.median(tf) + np.median(tb)),
            "ref_rel_err": ref_err}
        log(f"diff eigvec {'c128' if cplx else 'f64'}: "
            f"{out['cases'][('c128' if cplx else 'f64') + '_eigvec']}")
    out["value"] = out["cases"]["c128"]["fwd_bwd_s"]
    out["ms_per_step"] = out["value"] * 1e3
    return out


def warm_start_step(pk, H, vec, V0, S, nev, nex, wl, norm, handle):
    """One step of a sequence of related problems (the use case the method is
    built for): H2 = H + E with a seeded Hermitian E of spectral norm
    1e-5 ||H||_2, solved from the cold start block and from [eigenvectors of
    H | last nex columns of the cold start block]."""
    import torch

    n = H.shape[0]
    if n > 40000:
        return {"skipped": "the perturbed copy needs two more n x n buffers"}
    g = torch.Generator(device=H.device)
    g.manual_seed(20250502)
    E = torch.randn((n, n), generator=g, dtype=H.dtype, device=H.device)
    E = (E + E.mH) / 2
    # ||E||_2 of a Gaussian Hermitian matrix is about sqrt(2 n) times its
    # entry scale (semicircle edge); a few power steps pin it down
    x = torch.randn((n, 1), generator=g, dtype=H.dtype, device=H.device)
    for _ in range(30):
        x = E @ x
        x = x / torch.linalg.vector_norm(x)
    e2 = float(torch.linalg.vector_norm(E @ x))
    H2 = H + (1e-5 * norm / e2) * E
    del E
    v0w = torch.cat([vec, V0[:, nev:]], dim=1).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, rc, stc = pk.chase_solve(H2, nev, nex, wl["tol"], wl["deg"], V0, S, handle=handle)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    evw, _, rw, stw = pk.chase_solve(H2, nev, nex, wl["tol"], wl["deg"], v0w, S, handle=handle)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # the same warm start with Rayleigh-Ritz on the start block (initial_rr)
    opts_rr = pk.Opts.from_buffer_copy(handle.opts)
    opts_rr.initial_rr = 1
    hrr = pk.Handle(n, nev, nex, H.dtype, opts_rr)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    _, _, rr_res, strr = pk.chase_solve(H2, nev, nex, wl["tol"], wl["deg"], v0w, S, handle=hrr)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    hrr.close()
    del H2
    return {"perturbation": "||E||_2 = 1e-5 ||H||_2", "cold_s": t1 - t0, "warm_s": t2 - t1,
            "speedup": (t1 - t0) / (t2 - t1), "iterations_cold": stc["iterations"],
            "iterations_warm": stw["iterations"],
            "matvecs_cold": stc["matvecs_fp64"] + stc["matvecs_low"],
            "matvecs_warm": stw["matvecs_fp64"] + stw["matvecs_low"],
            "converged": bool(stc["converged"] and stw["converged"] and strr["converged"]),
            "max_resid_warm": float(rw.max()),
            "warm_initial_rr_s": t4 - t3, "speedup_initial_rr": (t1 - t0) / (t4 - t3),
            "iterations_warm_initial_rr": strr["iterations"],
            "matvecs_warm_initial_rr": strr["matvecs_fp64"] + strr["matvecs_low"],
            "max_resid_warm_initial_rr": float(rr_res.max())}


def time_modes(pk, prob, wl, precs, steps, warmup, label, verbose=False, max_deg=None,
               warm_start=False):
    """Time `steps` solves (after `warmup` untimed ones) of the problem in
    each filter mode, one handle per mode; returns per-mode results."""
    import numpy as np
    import torch

    n, nev, nex = wl["n"], wl["nev"], wl["nex"]
    H, V0, S = prob["H"].contiguous(), prob["V0"], prob["S"]
    lam = prob["lam"]
    norm = max(abs(lam[0]), abs(lam[-1]))
    results = {}
    for prec in precs:
        opts = pk.default_opts(filter_prec=PREC_CODE[prec], verbose=1 if verbose else 0,
                               eig_solver=EIG_CODE[EIG_CHOICE],
                               fp64_emulation=EMU_MODULI.get(prec, 0))
        if max_deg is not None:
            opts.max_deg = max_deg
        handle = pk.Handle(n, nev, nex, H.dtype, opts)
        for w in range(warmup):
            ev, vec, res, st = pk.chase_solve(H, nev, nex, wl["tol"], wl["deg"], V0, S,
                                              handle=handle)
            log(f"{label} {prec} warmup {w}: {st['t_all']:.2f} s, {st['iterations']} it")
        torch.cuda.synchronize()
        times, stats = [], []
        t_start = time.perf_counter()
        for k in range(steps):
            ts = time.perf_counter()
            ev, vec, res, st = pk.chase_solve(H, nev, nex, wl["tol"], wl["deg"], V0, S,
                                              handle=handle)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
            stats.append(st)
            log(f"{label} {prec} step {k}: {times[-1]:.2f} s, it={st['iterations']} "
                f"mv64={st['matvecs_fp64']} mvlow={st['matvecs_low']} "
                f"filter {st['filter_flops'] / st['t_filter_kernels'] / 1e12:.1f} TF")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        err = float(np.max(np.abs(ev - lam[:nev])))
        indep = independent_residual(H, vec, ev, prob) / norm
        # the filter launches of this mode's precision (a mixed solve also
        # runs FP64 filter steps: the start block's FP64 tail, FP64 ranks)
        per_mv = (8.0 if H.is_complex() else 2.0) * n * n
        if prec in ("fp64", "fp64i8"):
            fl = sum(s["filter_flops"] for s in stats)
            kt = sum(s["t_filter_kernels"] for s in stats)
            launches = sum(s["filter_launches"] for s in stats)
        else:
            fl = per_mv * sum(s["matvecs_low"] for s in stats)
            kt = sum(s["t_filter_kernels_low"] for s in stats)
            launches = sum(s["filter_launches_low"] for s in stats)
        lz_b = sum(s["lanczos_gemv_bytes"] for s in stats)
        lz_t = sum(s["t_lanczos_gemv"] for s in stats)
        results[prec] = dict(
            lanczos_gemv_gbs=lz_b / lz_t / 1e9 if lz_t > 0 else None,
            lanczos_gemv_ms=lz_t / max(1, sum(s["lanczos_gemv_launches"] for s in stats)) * 1e3,
            solve_s=elapsed / steps, converged=bool(st["converged"]),
            max_resid=float(res.max()), max_eig_err_rel=err / norm,
            max_resid_independent=indep,
            iterations=st["iterations"], matvecs_fp64=st["matvecs_fp64"],
            matvecs_low=st["matvecs_low"], fp64_tail=st["fp64_tail"],
            exec_per_algo=exec_per_algo(prec, st, wl["deg"], nev + nex, H.is_complex()),
            filter_tflops=fl / kt / 1e12, filter_kernel_s=kt / steps,
            filter_launches=launches // steps,
            avg_launch_ms=kt / launches * 1e3, flops_per_launch=fl / launches,
            phases={k: st[k] for k in ("t_lanczos", "t_filter", "t_qr", "t_rr", "t_rr_eig",
                                       "t_resid")},
            qr_shifted=st["qr_shifted"], qr_householder=st["qr_householder"],
            eig_jacobi_calls=st["eig_jacobi_calls"], eig_jacobi_sweeps=st["eig_jacobi_sweeps"],
            steps=steps, warmup=warmup, stats=st, evals=ev)
        if warm_start:
            results[prec]["warm_start"] = warm_start_step(pk, H, vec, V0, S, nev, nex, wl, norm,
                                                          handle)
            log(f"{label} {prec} warm start: {results[prec]['warm_start']}")
        del vec
        handle.close()
    return results


MODE_KEYS = ("solve_s", "converged", "max_resid", "max_eig_err_rel", "max_resid_independent",
             "iterations", "matvecs_fp64", "matvecs_low", "fp64_tail", "filter_tflops", "phases",
             "qr_shifted", "qr_householder", "eig_jacobi_calls", "eig_jacobi_sweeps", "steps",
             "warmup")


def mode_summary(m, prec, fp64_solve_s):
    out = {k: m[k] for k in MODE_KEYS}
    out["filter_frac_peak"] = m["filter_tflops"] / PEAK_TFLOPS[prec]
    out["filter_executed_frac"] = m["exec_per_algo"] * m["filter_tflops"] / PEAK_TFLOPS[prec]
    if prec == "fp64i8":
        # FP64-accurate products on INT8: the algorithmic rate against the
        # FP64 peak (above 1 when faster than the FP64 matrix cores can be),
        # the executed INT8 operations against the INT8 peak
        out["filter_executed_frac"] = m["exec_per_algo"] * m["filter_tflops"] / INT8_PEAK_TOPS
        out["filter_executed_unit"] = "INT8 TOPS / %g" % INT8_PEAK_TOPS
    if prec in EMU_MODULI:
        out["fp64_emulation_moduli"] = EMU_MODULI[prec]
    out["avg_launch_ms"] = m["avg_launch_ms"]
    if fp64_solve_s is not None and prec != "fp64":
        out["speedup_vs_fp64"] = fp64_solve_s / m["solve_s"]
    return out


def eigensolver_block(pk, k, reps=2):
    """The Rayleigh-Ritz step's dense eigensolve on its own (chase_heev):
    the library's Jacobi against rocSOLVER's divide and conquer on seeded
    complex Hermitian k x k matrices, dense (a random projected matrix, as in
    the first iteration) and diag(lambda) + E with ||E||_F = 1e-1, 1e-2, 1e-4
    of ||lambda|| (the later iterations).  Mean of `reps` timed calls after
    one untimed call; eigenvalue difference relative to max |lambda|."""
    import torch

    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    a = torch.randn((k, k), dtype=torch.complex128, device="cuda", generator=g)
    dense = (a + a.mH) / 2
    lam = torch.sort(torch.rand(k, dtype=torch.float64, device="cuda", generator=g) * 2 - 1).values
    e = dense / torch.linalg.norm(dense) * torch.linalg.norm(lam)
    cases = {"dense": dense}
    for off in (1e-1, 1e-2, 1e-4):
        cases[f"near_diagonal_{off:g}"] = torch.diag(lam).to(e.dtype) + off * e
    h = pk.Handle(k, k - 1, 1, torch.complex128)
    out = {"k": k, "dtype": "c128", "cases": {}}
    for name, G in cases.items():
        G = G.contiguous()
        row = {}
        for meth, code in (("jacobi", pk.EIG_JACOBI), ("library", pk.EIG_LIBRARY)):
            pk.chase_heev(G, method=code, handle=h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ev, W, sw = pk.chase_heev(G, method=code, handle=h)
            torch.cuda.synchronize()
            row[meth + "_ms"] = (time.perf_counter() - t0) / reps * 1e3
            row[meth + "_evals"] = ev
            if meth == "jacobi":
                row["jacobi_sweeps"] = sw
        row["eig_diff_rel"] = float(abs(row.pop("jacobi_evals") - row["library_evals"]).max()
                                    / abs(row.pop("library_evals")).max())
        out["cases"][name] = row
        log(f"eigensolver k={k} {name}: {row}")
    h.close()
    return out


def cholesky_block(pk, k, reps=10):
    """The Cholesky factor of the QR step's Cholesky passes on its own
    (chase_cholesky) on B^H B, B a seeded (2k + 8) x k Gaussian block,
    complex and real: the library's kernels timed with HIP events on the
    stream they run on (median of `reps` calls after two untimed ones, the
    matrix restored before each), torch.linalg.cholesky on the same matrix
    timed the same way, and the backward error max|R^H R - A| / max|A|."""
    import ctypes

    import numpy as np
    import torch

    L = pk.lib()
    out = {"k": k, "cases": {}}
    for dt, name in ((torch.complex128, "c128"), (torch.float64, "f64")):
        g = torch.Generator(device="cuda")
        g.manual_seed(k)
        b = torch.randn((2 * k + 8, k), dtype=dt, device="cuda", generator=g)
        a0 = (b.mH @ b).contiguous()
        del b
        buf = torch.empty_like(a0)
        h = pk.Handle(2, 1, 1, dt)
        info = ctypes.c_int()

        def timed(fn):
            ts = []
            for r in range(reps + 2):
                buf.copy_(a0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                torch.cuda.synchronize()
                if r >= 2:
                    ts.append(e0.elapsed_time(e1))
            return float(np.median(ts))

        def lib_call():
            rc = L.chase_cholesky(h.ptr, ctypes.c_void_p(buf.data_ptr()), k, k,
                                  ctypes.byref(info), pk._stream())
            if rc != 0 or info.value != 0:
                raise RuntimeError(f"chase_cholesky: status {rc}, info {info.value}")

        lib_ms = timed(lib_call)
        # buf (row-major) is the column-major A^T = conj(A); R^H R = conj(A) there
        R = torch.triu(buf.transpose(0, 1))
        err = ((R.mH @ R - a0.transpose(0, 1)).abs().max() / a0.abs().max()).item()
        torch_ms = timed(lambda: torch.linalg.cholesky(buf, upper=True))
        h.close()
        row = {"library_ms": lib_ms, "torch_linalg_cholesky_ms": torch_ms,
               "speedup": torch_ms / lib_ms, "backward_err": err}
        out["cases"][name] = row
        log(f"cholesky k={k} {name}: {row}")
    return out


def library_gemm_reference():
    """Rates of the vendor's own GEMMs on this GPU (torch -> hipBLASLt /
    rocBLAS), timed the same way as the library's kernels, as the practical
    ceiling beside the published peaks: a BF16 GEMM of 30000 x 30000 times
    30000 x 8000 with N(0, 1) and with zero operands (the chip's clock under
    MFMA load depends on the data), an FP64 GEMM and a complex128 GEMM of the
    n=20000 filter step's shape (20000 x 20000 times 20000 x 1300)."""
    import torch

    def rate(a, b, reps, flops):
        for _ in range(2):
            c = a @ b
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c = a @ b
        torch.cuda.synchronize()
        del c
        return flops / ((time.perf_counter() - t0) / reps) / 1e12

    out = {"source": "torch.matmul (hipBLASLt / rocBLAS)", "unit": "TFLOP/s"}
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    n, k = 30000, 8000
    a = torch.randn((n, n), device="cuda", dtype=torch.bfloat16, generator=g)
    b = torch.randn((n, k), device="cuda", dtype=torch.bfloat16, generator=g)
    out["bf16_random"] = rate(a, b, 10, 2.0 * n * n * k)
    a.zero_()
    b.zero_()
    out["bf16_zeros"] = rate(a, b, 10, 2.0 * n * n * k)
    del a, b
    torch.cuda.empty_cache()
    n, k = 20000, 1300
    for dt, key, per in ((torch.float64, "fp64", 2.0), (torch.complex128, "complex128", 8.0)):
        a = torch.randn((n, n), device="cuda", dtype=dt, generator=g)
        b = torch.randn((n, k), device="cuda", dtype=dt, generator=g)
        out[key] = rate(a, b, 3, per * n * n * k)
        del a, b
        torch.cuda.empty_cache()
    out["shapes"] = ("bf16: 30000x30000 @ 30000x8000; fp64 and complex128: 20000x20000 @ "
                     "20000x1300 (complex counted as 8 n^2 k)")
    return out


def mixed_workload_block(pk, precs, steps, warmup):
    """FP64 versus mixed-precision solves on the n=30000 workload (lowest 2000
    eigenvalues those of the (1-2-1) matrix, the rest uniform up to 10;
    nev=1500, nex=500): every mode solves the same matrix; the FP64 one is the
    reference for the speedups and the eigenvalue differences."""
    import numpy as np
    import torch

    import gen

    wl = WORKLOADS["cluster121_30k"]
    t0 = time.perf_counter()
    prob = gen.make_torch(wl["kind"], wl["n"], wl["nev"], wl["nex"], device="cuda")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"generated cluster121_30k n={wl['n']} in {time.perf_counter() - t0:.1f} s")
    res = time_modes(pk, prob, wl, precs, steps, warmup, "cluster121_30k")
    lam = prob["lam"]
    norm = max(abs(lam[0]), abs(lam[-1]))
    fp64_s = res["fp64"]["solve_s"] if "fp64" in res else None
    out = {"workload": "cluster121_30k", "n": wl["n"], "nev": wl["nev"], "nex": wl["nex"],
           "degree": wl["deg"], "tol": wl["tol"], "steps": steps, "warmup": warmup}
    for prec in precs:
        out[prec] = mode_summary(res[prec], prec, fp64_s)
        if "fp64" in res and prec != "fp64":
            out[prec]["max_eig_diff_vs_fp64_rel"] = float(
                np.max(np.abs(res[prec]["evals"] - res["fp64"]["evals"])) / norm)
    del prob
    torch.cuda.empty_cache()
    return out


def table2_block(pk, precs, steps, warmup):
    """The paper's matrix types (Table 1: Uniform, Geometric, (1-2-1),
    Wilkinson spectra) as dense real symmetric n=20000 matrices Q diag(lam)
    Q^T with a Haar Q, nev=1500, nex=500, degree 20, tol 1e-10: one MI355X
    beside the paper's one node of 4 A100 (Table 2, FP64)."""
    import torch

    import gen

    wl = WORKLOADS["table2"]
    out = {}
    for kind in ("uniform", "geometric", "121", "wilkinson"):
        t0 = time.perf_counter()
        prob = gen.make_torch(kind, wl["n"], wl["nev"], wl["nex"], device="cuda", cplx=False,
                              cfg=gen.CFG_TABLE2, lam=gen.spectrum_table1(kind, wl["n"]))
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        log(f"generated table2 {kind} in {time.perf_counter() - t0:.1f} s")
        res = time_modes(pk, prob, wl, precs, steps, warmup, f"table2 {kind}")
        fp64_s = res["fp64"]["solve_s"] if "fp64" in res else None
        it, mv, *secs = PAPER_TABLE2_GPU[kind]
        out[kind] = {p: mode_summary(res[p], p, fp64_s) for p in precs}
        out[kind]["paper_gpu_node"] = {
            "iterations": it, "matvecs": mv,
            "seconds": dict(zip(("all", "lanczos", "filter", "qr", "rr", "resid"), secs))}
        del prob, res
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="geometric20k", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="all",
                    choices=["fp64", "fp32", "bf16x3", "bf16x2", "fp64i8", "bf16x2i8", "both",
                             "all", "int8"],
                    help="filter modes to time: both = fp64 + fp32, all = every mode; fp64i8 "
                         "and bf16x2i8 run the FP64 products on the INT8 matrix cores "
                         "(14 moduli)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed-workload", action="store_true",
                    help="skip the n=30000 FP64-versus-mixed block of the default workload")
    ap.add_argument("--no-library-reference", action="store_true",
                    help="skip the vendor GEMM rates printed beside the roofline")
    ap.add_argument("--library-reference", action="store_true",
                    help="only time the vendor GEMMs (torch -> hipBLASLt / rocBLAS)")
    ap.add_argument("--extra-steps", type=int, default=5,
                    help="timed solves of each mode other than the main (FP64) one at most "
                         "(warm-ups at most 2)")
    ap.add_argument("--mixed-extra", nargs="*", default=[], choices=["fp64i8"],
                    help="further modes for the n=30000 block (fp64i8: every FP64 product "
                         "on INT8, about 40 s more)")
    ap.add_argument("--mixed-steps", type=int, default=1,
                    help="timed solves per mode in the n=30000 block")
    ap.add_argument("--mixed-warmup", type=int, default=0,
                    help="untimed solves per mode in the n=30000 block")
    ap.add_argument("--warm-start", action="store_true",
                    help="also time a sequence step: H + E (||E||_2 = 1e-5 ||H||_2, seeded "
                         "Hermitian) solved cold and warm-started from the previous "
                         "eigenvectors, in each timed filter mode")
    ap.add_argument("--eig-solver", default="auto", choices=sorted(EIG_CODE),
                    help="dense eigensolver of the Rayleigh-Ritz step: auto (the library's "
                         "Jacobi once the projected matrix is near diagonal, else rocSOLVER), "
                         "library (rocSOLVER) or jacobi")
    ap.add_argument("--moduli", type=int, default=None, choices=[8, 10, 12, 14, 16],
                    help="moduli of the INT8 FP64-product modes (default 14)")
    ap.add_argument("--eigensolver", type=int, default=None, metavar="K",
                    help="only time the Rayleigh-Ritz eigensolve (Jacobi and rocSOLVER) "
                         "on K x K complex Hermitian matrices")
    ap.add_argument("--cholesky", type=int, default=None, metavar="K",
                    help="only time the QR passes' Cholesky factorisation (the library's "
                         "and torch.linalg.cholesky) on K x K positive definite matrices")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--max-deg", type=int, default=None,
                    help="cap of the optimised filter degree (library default 36)")
    ap.add_argument("--gen-elementary", action="store_true",
                    help="build Q from 64 elementary reflectors (no factorization) with the "
                         "workload's spectrum; for counter-collection runs, where rocprofv3 "
                         "--pmc crashes inside the dense QR of the usual generator")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte "
                         "counters of rocprofv3 --pmc)")
    args = ap.parse_args()
    global EIG_CHOICE
    EIG_CHOICE = args.eig_solver
    if args.moduli is not None:
        for key in EMU_MODULI:
            EMU_MODULI[key] = args.moduli
        EXEC_PER_ALGO["fp64i8"] = 3 * args.moduli * 2 / 8.0
    if args.library_reference:
        print(json.dumps(library_gemm_reference()), flush=True)
        return
    if args.eigensolver is not None:
        import paper_2205_02491_amd as pk
        print(json.dumps(eigensolver_block(pk, args.eigensolver)), flush=True)
        return
    if args.cholesky is not None:
        import paper_2205_02491_amd as pk
        print(json.dumps(cholesky_block(pk, args.cholesky)), flush=True)
        return
    if args.calib_copy:
        import torch
        x = torch.ones(2**27, dtype=torch.float64, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": 2**30, "launches": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import gen
    import paper_2205_02491_amd as pk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    pk.lib()
    wl = WORKLOADS[args.workload]
    n, nev, nex = wl["n"], wl["nev"], wl["nex"]
    if args.workload == "diff8k":
        print(json.dumps(bench_diff(args, wl)), flush=True)
        return
    if args.workload == "table2":
        precs = {"both": ["fp64", "fp32"], "all": ["fp64", "fp32", "bf16x3", "bf16x2"],
                 "int8": ["fp64", "fp64i8", "bf16x2", "bf16x2i8"]}.get(args.prec, [args.prec])
        if "fp64" not in precs:
            precs = ["fp64"] + precs
        t2 = table2_block(pk, precs, args.steps, args.warmup)
        print(json.dumps({"metric": "solve s per matrix type (Table 2 suite, n=20000 float64)",
                          "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                          "higher_is_better": False, "data": "synthetic (Table 1 spectra, Haar Q)",
                          "config": {"workload": "table2", "n": n, "nev": nev, "nex": nex,
                                     "degree": wl["deg"], "tol": wl["tol"]},
                          "value": t2["121"]["fp64"]["solve_s"], "vs_baseline": None,
                          "table2": t2}), flush=True)
        return
    t0 = time.perf_counter()
    if wl["kind"] == "reflectors":
        prob = gen.make_torch_reflectors(n, nev, nex, device="cuda")
    elif args.gen_elementary:
        lam_w = {"geometric": lambda: gen.spectrum_geometric_low(
                     n, gen.rng(gen.CFG_GEO20K, gen.SLOT_LAMBDA), 1200 if n == 20000 else (nev + nex) * 12 // 13),
                 "cluster121": lambda: gen.spectrum_121_cluster(
                     n, gen.rng(gen.CFG_MIXED30K, gen.SLOT_LAMBDA), nev + nex)}[wl["kind"]]()
        prob = gen.make_torch_reflectors(n, nev, nex, nrefl=64, width=1, device="cuda", lam=lam_w)
    else:
        prob = gen.make_torch(wl["kind"], n, nev, nex, device="cuda")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"generated {args.workload} n={n} in {time.perf_counter() - t0:.1f} s")

    precs = {"both": ["fp64", "fp32"],
             "all": ["fp64", "fp32", "bf16x3", "bf16x2", "fp64i8", "bf16x2i8"],
             "int8": ["fp64", "fp64i8", "bf16x2", "bf16x2i8"]}.get(args.prec, [args.prec])
    # the main mode takes the requested steps; the other modes, reported
    # beside it, at most --extra-steps (their rates settle within a few solves)
    main_first = "fp64" if "fp64" in precs else precs[0]
    results = time_modes(pk, prob, wl, [main_first], args.steps, args.warmup, args.workload,
                         verbose=args.verbose, max_deg=args.max_deg, warm_start=args.warm_start)
    rest = [p for p in precs if p != main_first]
    if rest:
        results.update(time_modes(pk, prob, wl, rest, min(args.steps, args.extra_steps),
                                  min(args.warmup, 2), args.workload, verbose=args.verbose,
                                  max_deg=args.max_deg, warm_start=args.warm_start))
    H = prob["H"]

    main_prec = "fp64" if "fp64" in results else precs[0]
    r = results[main_prec]
    peak = PEAK_TFLOPS[main_prec]
    # dominant kernel: the Chebyshev-step GEMM of the filter (all filter
    # launches of the timed solves; HIP events around each launch)
    roof = {"bound": "mfma", "achieved": r["filter_tflops"], "peak": peak, "unit": "TFLOP/s",
            "frac": r["filter_tflops"] / peak, "traffic": None,
            "kernel": KERNEL_NAME[main_prec] + "; executed MFMA FLOPs = %g x algorithmic"
                      % r["exec_per_algo"],
            "avg_launch_ms": r["avg_launch_ms"], "flops_per_launch": r["flops_per_launch"]}
    roof["executed_frac"] = r["exec_per_algo"] * r["filter_tflops"] / peak
    tr = MEASURED_TRAFFIC.get((args.workload, main_prec))
    if tr is not None:
        import hashlib
        src = os.path.join(ROOT, "paper_2205_02491_amd", "csrc", "gemm.hip")
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if sha == tr["gemm_sha256"]:
            roof["traffic"] = (tr["fetch_gb"] + tr["write_gb"]) * 1e9
            roof["traffic_unit"] = "bytes per launch (%d columns)" % tr["columns"]
            roof["traffic_source"] = tr["source"]
    out = {
        "metric": METRIC, "value": r["solve_s"], "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["solve_s"] * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "c128", "fp32": "c64/c128", "bf16x3": "bf16x3/c128",
                  "bf16x2": "bf16x2/c128", "fp64i8": "int8-crt/c128",
                  "bf16x2i8": "bf16x2/int8-crt/c128"}[main_prec],
        "data": "synthetic planted-spectrum Hermitian (seeded, generated on the GPU)",
        "config": {"workload": f"{args.workload}", "n": n, "nev": nev, "nex": nex,
                   "degree": wl["deg"], "tol": wl["tol"], "filter": main_prec,
                   "max_deg": args.max_deg if args.max_deg is not None else 36,
                   "parallelism": "single GPU"},
        "filter_tflops": r["filter_tflops"], "filter_frac_peak": r["filter_tflops"] / peak,
        "filter_peak_tflops": peak,
        "iterations": r["iterations"], "matvecs": r["matvecs_fp64"] + r["matvecs_low"],
        "converged": r["converged"], "max_resid": r["max_resid"],
        "max_resid_independent": r["max_resid_independent"],
        "max_eig_err_rel": r["max_eig_err_rel"], "phases_s": r["phases"],
        "qr_shifted_passes": r["qr_shifted"], "qr_householder": r["qr_householder"],
        "eig_solver": EIG_CHOICE, "eig_jacobi_calls": r["eig_jacobi_calls"],
        "eig_jacobi_sweeps": r["eig_jacobi_sweeps"],
        "roofline": roof,
        # memory-bound step: the Lanczos block GEMV (H read once per launch,
        # 4 vectors), HIP events around each launch of the timed solves
        "memory_bound": {"kernel": "lz_gemv_k (Lanczos block GEMV, 4 vectors)", "bound": "hbm",
                         "achieved": r["lanczos_gemv_gbs"], "peak": 8000.0, "unit": "GB/s",
                         "frac": (r["lanczos_gemv_gbs"] / 8000.0
                                  if r["lanczos_gemv_gbs"] else None),
                         "avg_launch_ms": r["lanczos_gemv_ms"],
                         "bytes_per_launch": n * n * (16 if H.is_complex() else 8)},
    }
    for low, key in (("fp32", "mixed"), ("bf16x3", "mixed_bf16x3"), ("bf16x2", "mixed_bf16x2"),
                     ("fp64i8", "fp64_on_int8"), ("bf16x2i8", "mixed_bf16x2_int8")):
        if low not in results or main_prec == low:
            continue
        out[key] = mode_summary(results[low], low, r["solve_s"])
    if args.warm_start:
        out["warm_start"] = {p: results[p]["warm_start"] for p in results}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        Hh = H.cpu().numpy()
        V0h = prob["V0"].cpu().numpy()
        Sh = prob["S"].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(Hh, V0h, Sh, r["stats"], n, nev + nex)
        del Hh, V0h, Sh
        out["cpu_baseline"]["small_solve"] = small_solve_pair(pk)
        log(f"cpu baseline done in {time.perf_counter() - t0:.1f} s: "
            f"{out['cpu_baseline']['pieces_s']}, small {out['cpu_baseline']['small_solve']}")
    del H, prob, results
    torch.cuda.empty_cache()
    if not args.no_library_reference:
        out["library_gemm_reference"] = library_gemm_reference()
        log(f"library GEMM reference: {out['library_gemm_reference']}")
    if args.workload == "geometric20k" and not (args.no_mixed_workload or args.gen_elementary):
        # the metric's FP64-versus-mixed comparison on the workload where the
        # mixed-precision policy does its work (many iterations, defect form)
        out["mixed_workload"] = mixed_workload_block(
            pk, ["fp64", "fp32", "bf16x3", "bf16x2", "bf16x2i8"] + args.mixed_extra,
            args.mixed_steps, args.mixed_warmup)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
