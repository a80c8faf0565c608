"""Benchmark: preconditioned batch Krylov sampler on one MI355X.

Workload (one "step" = one pass of the whole sampling path over one batch):
  512 x 512 lattice, second-order precision Q = (kappa2 I + L)^2 (13-point, free boundary),
  kappa2 = 0.01, block-circulant preconditioner M = periodic version of Q applied with 2D
  FFTs, 32 seeded N(0, I) right-hand sides.  The step is z -> z_hat -> Lanczos steps ->
  T^{-1/2} e_1 -> x = M^{-1/2} u_m for all 32 columns.

Headline value: samples/s at <= 1e-5 relative error.  With this preconditioner the operator
keeps cond(A) ~ 1.7e4, so 1e-5 needs m ~ 480 steps (rho <= 1e-5) in FP64 storage; FP32
storage floors near 8e-5 on this operator and m_max = 300 stops near 3e-4.  Those runs are
reported beside the headline ("at_m_max_300", "fp32").  The relative error of column 0 is
measured against the CPU oracle's converged sample (full reorthogonalisation, rho <= 1e-10).

Roofline: the dominant kernel of the step (the preconditioned step kernel) is timed alone with
HIP events on the stream it runs on; its algorithmic bytes per launch are 3 s n k (read v_j and
v_{j-1}, write w_j; s = 8 bytes, n = 512^2, k = 32).  cpu_baseline: the oracle (NumPy/SciPy FP64)
on one column of the same workload with the same stopping rule.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

HBM_PEAK_GBS = 8000.0
DOMINANT_KERNEL = "lz_step"      # largest share of the step in the committed rocprofv3 summary
COPY_BYTES = 512 << 20           # reference read / copy of the counter runs (--only counters)
# HBM bytes per launch of the dominant kernel from the committed counter summary: FETCH_SIZE x 2 +
# WRITE_SIZE x 1 (KiB per dispatch, scaled by the reference copy's readings); None if the kernel changed
TRAFFIC_BYTES = 225610752      # k_step<double, 64, true>, 512x512, 32 fields (profiles/k_step_precond_512x512_32rhs_fp64.md)
TOL_HEADLINE = 1e-5              # stopping rule of the headline (rho_m <= tol)
ERR_HEADLINE = 1e-5              # a headline sample counts when its relative error is within this
REF_TOL, REF_M_MAX = 1e-10, 1024 # converged FP64 reference of the headline columns
INFINITY_CACHE_BYTES = 256 << 20
BW_BYTES = 1 << 30               # array size of the achievable-bandwidth kernels (beyond the Infinity Cache)
SERVE_RATES = (50, 100, 150, 200, 256)  # offered requests/s of the serving leg, raised until the server falls behind
SERVE_WARMUP_S = 2.0             # arrivals in the first 2 s of each window are served but not counted
SERVE_TOL, SERVE_M_MAX = 1e-5, 600   # served samples: FP32 storage at the headline's 1e-5
SERVE_LOGDET_M = 80
M_MAX_HEADLINE = 600


def _ensure_built():
    from paper_1312_1476_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs (profiling runs)")
    ap.add_argument("--only", default="", help="profiling: run only this leg (headline|counters|lgcp|logdet|ichol|plain|uneven|serve)")
    ap.add_argument("--no-ref", action="store_true",
                    help="profiling: skip the converged reference run of the headline (value is then null)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-lgcp", action="store_true", help="skip the log-Gaussian Cox process leg")
    ap.add_argument("--no-logdet", action="store_true", help="skip the log-determinant leg")
    ap.add_argument("--no-ichol", action="store_true", help="skip the incomplete-Cholesky leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain 64x64 and uneven-batch legs")
    ap.add_argument("--kernel", default="", help="counters leg: kernel to run (default: the dominant one)")
    ap.add_argument("--storage", default="f64", help="counters leg: storage dtype (f64|f32)")
    ap.add_argument("--side", type=int, default=512, help="counters leg: lattice side of the operator (spmv)")
    ap.add_argument("--dim", type=int, default=2, help="counters leg: 2 (13-point) or 3 (7-point) lattice (spmv)")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="arrival window per serving rate")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (samples, probes and "
              "fields shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)
    _ensure_built()
    import torch
    import paper_1312_1476_amd as gm

    c = workloads.C1
    sp = c.lattice
    k = c.k
    Zh = workloads.gaussian_block(sp.n, k, 1, 0)
    Z = torch.from_numpy(np.ascontiguousarray(Zh.T)).to("cuda:0")
    stream = torch.cuda.current_stream()

    def make(storage):
        return gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, storage).set_circulant_precond()

    op64 = make("f64")

    if args.only == "counters":
        # workload of the hardware-counter runs: one kernel alone (the dominant one unless --kernel names
        # another: spmv = the 13-point operator alone), then a plain device copy of known size whose
        # FETCH_SIZE / WRITE_SIZE readings scale the counters to bytes
        name = args.kernel or DOMINANT_KERNEL
        if name in ("lgcp_rows", "lgcp_cols"):   # the LGCP passes at 512 x 512 (periodic prior, diagonal H)
            spec = workloads.lgcp_prior(args.side)
            op = gm.Operator.lattice(spec.shape, 2, spec.kappa2, spec.tau, "periodic", args.storage)
            op.set_diagonal(workloads.lgcp_diagonal(args.side))
            op.set_circulant_precond()
        elif name != "spmv":
            op = make(args.storage)
        elif args.dim == 3:      # the 3D 7-point operator (first order) of the serving pool's 3D lattices
            op = gm.Operator.lattice((args.side,) * 3, 1, 0.05, 1.0, "free", args.storage)
        else:
            op = gm.Operator.lattice((args.side, args.side), sp.order, sp.kappa2, sp.tau, sp.boundary, args.storage)
        if name in ("spmv", "lz2d"):
            gm.autotune(op, k, reps=20, stream=stream)     # count the kernel with the launch options it runs with
        r = gm.kernel_bench(op, name, k, reps=50, stream=stream)
        # references of known size: the library's read kernel (FETCH_SIZE) and copy kernel (WRITE_SIZE) over
        # arrays of COPY_BYTES, 5 + 2 launches each
        gm.bandwidth_bench("read", COPY_BYTES, reps=5, stream=stream)
        gm.bandwidth_bench("copy", COPY_BYTES, reps=5, stream=stream)
        torch.cuda.synchronize()
        print(json.dumps({"kernel": name, "storage": args.storage, "avg_us": r["avg_us"], "bytes": r["bytes"],
                          "reference_bytes": COPY_BYTES}))
        return

    def step(op, tol, m_max):
        return op.sample(Z, tol=tol, m_max=m_max, reorth=False)

    if args.only == "lgcp":
        print(json.dumps({"lgcp": lgcp_leg(gm, torch, stream)}))
        return
    if args.only == "logdet":
        print(json.dumps({"logdet": logdet_leg(gm, torch)}))
        return
    if args.only == "ichol":
        print(json.dumps({"ichol": ichol_leg(gm, torch)}))
        return
    if args.only == "plain":
        print(json.dumps({"plain_64x64": _public(plain_leg(gm, torch))}))
        return
    if args.only == "serve":
        print(json.dumps({"serving": serving_leg(gm, torch, args.serve_seconds)}))
        return
    if args.only == "uneven":
        print(json.dumps({"uneven_batch": _public(uneven_leg(gm, torch))}))
        return

    # ---- headline: FP64 storage, stop at rho <= 1e-5 ---------------------------------------------
    for _ in range(args.warmup):
        step(op64, TOL_HEADLINE, M_MAX_HEADLINE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        X, info = step(op64, TOL_HEADLINE, M_MAX_HEADLINE)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    m_used = [i["m_used"] for i in info]
    x0 = X[0].cpu().numpy()
    # every column against the same columns run to convergence (FP64, rho <= 1e-10, m_max = 1024; the
    # full-size parity test pins this run to the oracle at 1e-8): only samples within 1e-5 count
    if args.no_ref:
        Xref, iref = X, info
    else:
        Xref, iref = step(op64, REF_TOL, REF_M_MAX)
    torch.cuda.synchronize()
    errs = ((X - Xref).norm(dim=1) / Xref.norm(dim=1)).cpu().numpy()
    n_ok = int(np.sum(errs <= ERR_HEADLINE))
    xref0 = Xref[0].cpu().numpy()
    result = {
        "metric": "samples/s at 1e-5 rel err, batched/served vs plain; SpMV HBM GB/s; p99 latency",
        "value": None if args.no_ref else round(n_ok / dt, 2),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * dt, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded N(0, I) right-hand sides on a synthetic lattice precision",
        "config": {"workload": "preconditioned batch: 512x512 lattice, 13-point second-order Q, kappa2=0.01, "
                               "free boundary, periodic block-circulant preconditioner (2D FFT), 32 RHS",
                   "n": sp.n, "rhs": k, "storage": "f64", "tol_rho": TOL_HEADLINE, "m_max": M_MAX_HEADLINE,
                   "m_used_max": max(m_used), "m_used_min": min(m_used), "reorth": False,
                   "parallelism": "single GPU, RHS-batched"},
        "headline_accuracy": {
            "reference": f"the same 32 columns, FP64, rho <= {REF_TOL:g} (m = {min(i['m_used'] for i in iref)}-"
                         f"{max(i['m_used'] for i in iref)}), all converged: "
                         f"{all(i['status'] == 'OK' for i in iref)}",
            "within_1e-5": n_ok, "of": k, "max_rel_err": float(errs.max()),
            "median_rel_err": float(np.median(errs))},
    }
    if args.only == "headline":
        print(json.dumps(result))
        return

    # ---- literal m_max = 300 runs (FP64 and FP32 storage) ------------------------------------------
    extra = {}
    op32 = make("f32")
    for name, op in (("f64", op64), ("f32", op32)):
        step(op, c.tol, c.m_max)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps // 2)):
            Xl, il = step(op, c.tol, c.m_max)
        torch.cuda.synchronize()
        dtl = (time.perf_counter() - t0) / max(1, args.steps // 2)
        extra[name] = {"samples_per_s": round(k / dtl, 2), "ms_per_step": round(1000 * dtl, 3),
                       "m_used": il[0]["m_used"], "rho": il[0]["rel_residual"], "x_col0": Xl[0].cpu().numpy()}
    # plain single-sample FP64 Lanczos on the same operator and stopping rule (k = 1)
    Z1 = Z[:1].contiguous()
    op64.sample(Z1, tol=TOL_HEADLINE, m_max=M_MAX_HEADLINE)
    torch.cuda.synchronize()
    nplain = 4
    t0 = time.perf_counter()
    for r in range(nplain):
        op64.sample(Z[r:r + 1].contiguous(), tol=TOL_HEADLINE, m_max=M_MAX_HEADLINE)
    torch.cuda.synchronize()
    dtp = (time.perf_counter() - t0) / nplain
    result["plain_single_sample_fp64"] = {"samples_per_s": round(1.0 / dtp, 2), "ms_per_sample": round(1000 * dtp, 3),
                                          "batched_speedup": round((k / dt) * dtp, 2)}
    # two-pass sampler (no stored basis: three Krylov slots instead of m_max + 1) on the same batch and rule
    op64.sample_two_pass(Z, tol=TOL_HEADLINE, m_max=M_MAX_HEADLINE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X2p, i2p = op64.sample_two_pass(Z, tol=TOL_HEADLINE, m_max=M_MAX_HEADLINE)
    torch.cuda.synchronize()
    dt2 = time.perf_counter() - t0
    vec = k * sp.n * 8
    result["two_pass_fp64"] = {"samples_per_s": round(k / dt2, 2), "ms_per_step": round(1000 * dt2, 3),
                               "m_used_max": max(i["m_used"] for i in i2p),
                               "basis_bytes_one_pass": (M_MAX_HEADLINE + 1) * vec, "basis_bytes_two_pass": 3 * vec,
                               "max_abs_diff_vs_one_pass": float((X2p - X).abs().max())}
    # the same batch without the preconditioner at the workload's m_max = 300: it stops at m_max far from
    # 1e-5, which is what the preconditioner is for
    opq = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, "f64")
    step(opq, TOL_HEADLINE, c.m_max)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xu, iu = step(opq, TOL_HEADLINE, c.m_max)
    torch.cuda.synchronize()
    dtu = time.perf_counter() - t0
    extra["unprec"] = {"samples_per_s": round(k / dtu, 2), "ms_per_step": round(1000 * dtu, 3),
                       "m_used": iu[0]["m_used"], "status": iu[0]["status"], "rho": iu[0]["rel_residual"],
                       "x_col0": Xu[0].cpu().numpy()}
    opq.close()
    # FP32 storage with the headline stopping rule (reaches its accuracy floor)
    step(op32, TOL_HEADLINE, M_MAX_HEADLINE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X32, i32 = step(op32, TOL_HEADLINE, M_MAX_HEADLINE)
    torch.cuda.synchronize()
    dt32 = time.perf_counter() - t0
    extra["f32_tol"] = {"samples_per_s": round(k / dt32, 2), "m_used": i32[0]["m_used"],
                        "rho": i32[0]["rel_residual"], "x_col0": X32[0].cpu().numpy()}

    # ---- roofline: dominant kernel timed alone -----------------------------------------------------
    roof = gm.kernel_bench(op64, DOMINANT_KERNEL, k, reps=50, stream=stream)
    result["roofline"] = {"bound": "hbm", "achieved": round(roof["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(roof["achieved_gbs"] / HBM_PEAK_GBS, 4),
                          "traffic": TRAFFIC_BYTES, "kernel": roof["kernel"], "avg_us": round(roof["avg_us"], 2),
                          "bytes_per_launch": roof["bytes"],
                          # the launch's vectors fit the 256 MB Infinity Cache (as they do in the sampling loop,
                          # where v_j and v_{j-1} were written one and two steps before)
                          "cache_resident": roof["bytes"] < INFINITY_CACHE_BYTES}
    # achievable HBM bandwidth on this part (hand-written read / copy / triad kernels over 1 GiB arrays)
    ach = {kind: round(gm.bandwidth_bench(kind, BW_BYTES, reps=10, stream=stream)["gbs"], 1)
           for kind in ("read", "copy", "triad")}
    result["roofline"]["achievable_gbs"] = ach
    # the step kernel reads two vectors and writes one: the triad's mix
    result["roofline"]["frac_of_achievable_triad"] = round(roof["achieved_gbs"] / ach["triad"], 4)
    kern = {}
    for name in ("lz_band", "lz_dots"):
        r = gm.kernel_bench(op64, name, k, reps=50, stream=stream)
        kern[name] = {"avg_us": round(r["avg_us"], 2), "gbs": round(r["achieved_gbs"], 1)}
    result["other_kernels"] = kern
    # the SpMV/SpMM metric: the 13-point stencil over 32 columns, FP64 and FP32 storage, with the launch options
    # the autotuner picks (tile order, store policy; no option changes a result bit)
    spmv = {}
    for name, op in (("f64", op64), ("f32", op32)):
        gm.autotune(op, k, reps=20, stream=stream)
        r = gm.kernel_bench(op, "spmv", k, reps=50, stream=stream)
        spmv[name] = {"achieved_gbs": round(r["achieved_gbs"], 1), "frac_of_peak": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                      "avg_us": round(r["avg_us"], 2), "bytes_per_launch": r["bytes"]}
    result["spmv_13pt_32rhs"] = spmv
    # the same operator on 1024 x 1024 (537 MB per FP64 launch, beyond the 256 MB Infinity Cache): HBM-resident
    spmv_big = {}
    for storage in ("f64", "f32"):
        opb = gm.Operator.lattice((1024, 1024), sp.order, sp.kappa2, sp.tau, sp.boundary, storage)
        gm.autotune(opb, k, reps=10, stream=stream)
        r = gm.kernel_bench(opb, "spmv", k, reps=20, stream=stream)
        spmv_big[storage] = {"achieved_gbs": round(r["achieved_gbs"], 1),
                             "frac_of_peak": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                             "avg_us": round(r["avg_us"], 2), "bytes_per_launch": r["bytes"],
                             "cache_resident": r["bytes"] < INFINITY_CACHE_BYTES}
        opb.close()
    result["spmv_13pt_1024x1024_32rhs"] = spmv_big
    # the unpreconditioned one-pass Lanczos step (the C2/C3 and 2D serving kernel) on a large single field:
    # 5-point, 2048 x 2048, 8 columns, 3 s n k bytes per step (805 MB FP64), tuned launch options
    lz = {}
    for storage in ("f64", "f32"):
        opl = gm.Operator.lattice((2048, 2048), 1, 0.05, 1.0, "free", storage)
        gm.autotune(opl, 8, reps=10, stream=stream)
        r = gm.kernel_bench(opl, "lz2d", 8, reps=20, stream=stream)
        lz[storage] = {"achieved_gbs": round(r["achieved_gbs"], 1), "frac_of_peak": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                       "avg_us": round(r["avg_us"], 2), "bytes_per_launch": r["bytes"]}
        opl.close()
    result["lanczos2d_5pt_2048x2048_8rhs"] = lz
    # the 3D 7-point operator (z-marching kernel), 128^3 x 32: 1074 MB FP64 per launch
    sp3 = {}
    for storage in ("f64", "f32"):
        op3 = gm.Operator.lattice((128, 128, 128), 1, 0.05, 1.0, "free", storage)
        r = gm.kernel_bench(op3, "spmv", 32, reps=20, stream=stream)
        sp3[storage] = {"achieved_gbs": round(r["achieved_gbs"], 1), "frac_of_peak": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                        "avg_us": round(r["avg_us"], 2), "bytes_per_launch": r["bytes"]}
        op3.close()
    result["spmv_7pt_128cubed_32rhs"] = sp3
    # the general CSR operator (gmrf_op_create_csr) holding the same 13-point Q on 512 x 512, 32 columns:
    # each row's entries are read once for 8 right-hand sides
    Pc = lattice_csr(512, 2, sp.kappa2)
    opc = gm.Operator.csr(Pc.shape[0], Pc.indptr, Pc.indices, Pc.data)
    r = gm.kernel_bench(opc, "spmv", 32, reps=20, stream=stream)
    result["spmv_csr_13pt_512x512_32rhs"] = {"avg_us": round(r["avg_us"], 2), "nnz": int(Pc.nnz),
                                             "bytes_per_launch": r["bytes"],   # X, Y and the matrix once
                                             "achieved_gbs": round(r["achieved_gbs"], 1)}
    opc.close()

    # ---- log-Gaussian Cox process proposal (Q + H, M = Q): Table 1 and throughput --------------------
    if not args.no_lgcp:
        result["lgcp"] = lgcp_leg(gm, torch, stream)

    # ---- Hutchinson log det (workload C3), plain and coloured ------------------------------------------
    if not args.no_logdet:
        result["logdet"] = logdet_leg(gm, torch)

    # ---- incomplete-Cholesky preconditioning (Section 5.2, Figure 3) ------------------------------------
    if not args.no_ichol:
        result["ichol"] = ichol_leg(gm, torch)

    # ---- plain FP64 single sample (64 x 64) and the uneven batch of 256 fields ---------------------------
    if not args.no_plain:
        result["plain_64x64"] = plain_leg(gm, torch)
        result["uneven_batch"] = uneven_leg(gm, torch)

    # ---- serving: Poisson request stream over a pool of 64 resident operators ---------------------------
    if not args.no_serve:
        result["serving"] = serving_leg(gm, torch, args.serve_seconds)

    # the launch options the autotuner chose (kernel, lattice class, columns class -> options)
    result["autotune"] = [f"{r['kernel']} order {r['order']} {r['storage']} 2^{r['log2_n1']}x2^{r['log2_n2']} "
                          f"k<=2^{r['log2_k']}: {'+'.join(r['options']) or 'none'}" for r in gm.tune_table()]

    # ---- oracle legs ----------------------------------------------------------------------------------
    if not args.no_cpu:
        from oracle import lattice as olat, precond as opre
        Q = olat.lattice_precision(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary)
        cores = len(os.sched_getaffinity(0))
        t0 = time.perf_counter()
        ro = opre.sample(Q, sp.shape, sp.order, sp.kappa2, sp.tau, Zh[:, 0], M_MAX_HEADLINE, tol=TOL_HEADLINE)
        tcpu = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(1.0 / tcpu, 4), "unit": "samples/s", "cores": cores, "kind": "oracle",
                                  "sample": f"column 0 of the 32-column batch, same stopping rule (m = {ro.m}); "
                                            f"{tcpu:.1f} s"}
        ref = opre.sample(Q, sp.shape, sp.order, sp.kappa2, sp.tau, Zh[:, 0], 700, tol=1e-10, reorth=True)
        nref = np.linalg.norm(ref.x)
        rel = lambda x: float(np.linalg.norm(x - ref.x) / nref)
        result["accuracy"] = {
            "reference": f"oracle, full reorthogonalisation, rho = {ref.rho[-1]:.1e} (m = {ref.m})",
            "headline_rel_err_col0": rel(x0),
            # the GPU's converged reference (no reorthogonalisation) against the oracle's (CGS2): both
            # converged, so they differ by truncation only
            "gpu_reference_col0_vs_oracle_reference": rel(xref0),
            # both sides stop at rho <= 1e-5, before convergence, where the iterate moves by far more than
            # rounding under a rounding-level change of the operator; tight parity is taken at convergence
            "parity_vs_oracle_same_rule_col0": float(np.linalg.norm(x0 - ro.x) / np.linalg.norm(ro.x)),
        }
        for key in ("f64", "f32", "f32_tol", "unprec"):
            extra[key]["rel_err_col0"] = rel(extra[key]["x_col0"])
        if "plain_64x64" in result:
            from oracle import closed_form as ocf
            c0 = workloads.C0
            sp0 = c0.lattice
            z0 = workloads.gaussian_block(sp0.n, 1, 0, 0)[:, 0]
            ex = ocf.exact_sample_free(sp0.shape, sp0.order, sp0.kappa2, sp0.tau, z0)
            result["plain_64x64"]["rel_err_vs_exact"] = float(np.linalg.norm(result["plain_64x64"]["_x"] - ex)
                                                              / np.linalg.norm(ex))
        if "logdet" in result:
            from oracle import closed_form as ocf
            sp3 = workloads.C3_LATTICE
            ex = ocf.exact_logdet(sp3.shape, sp3.order, sp3.kappa2, sp3.tau, sp3.boundary)
            result["logdet"]["exact"] = ex
            for v in result["logdet"]["variants"].values():
                v["z_score"] = (v["estimate"] - ex) / v["std_err"]
        if "uneven_batch" in result:
            from oracle import closed_form as ocf
            errs = []
            for f, ((side, k2), Zf, Xf) in result["uneven_batch"]["_x"].items():
                ex = ocf.exact_sample_free((side, side), 1, k2, 1.0, Zf.T)
                errs += [float(np.linalg.norm(Xf[r] - ex[:, r]) / np.linalg.norm(ex[:, r])) for r in range(Zf.shape[0])]
            result["uneven_batch"]["accuracy"] = {
                "sample": "8 fields across the kappa2 range x 8 columns, vs the exact DCT sample",
                "max_rel_err": max(errs), "median_rel_err": float(np.median(errs)),
                "within_1e-5": sum(e <= 1e-5 for e in errs), "of": len(errs)}
    for key in extra:
        extra[key].pop("x_col0", None)
    for key in ("plain_64x64", "uneven_batch"):
        if key in result:
            result[key] = _public(result[key])
    result["at_m_max_300"] = {"f64": extra["f64"], "f32": extra["f32"]}
    result["fp32_storage_at_tol"] = extra["f32_tol"]
    result["unpreconditioned_at_m_max_300"] = extra["unprec"]
    print(json.dumps(result))


def _public(d):
    """The leg's record without its private arrays (keys starting with an underscore)."""
    return {k: v for k, v in d.items() if not k.startswith("_")}


LGCP_TOL = 1e-8                  # Table 1's accuracy
LGCP_TABLE_N = (16, 32, 64, 128, 256, 512, 1024, 2048, 4096)
LGCP_BATCH = (512, 32)           # side, right-hand sides of the throughput line
LGCP_UNPRE_N = (16, 32, 64, 128)   # Table 1's unpreconditioned row (the Krylov dimension grows with N)
LGCP_UNPRE_M_MAX = 16384


def lgcp_leg(gm, torch, stream):
    """The sMMALA proposal of the log-Gaussian Cox process on the unit torus (workload C5): Q + H with
    the periodic prior as preconditioner (two 2D FFTs per step).  Table 1's preconditioned row (Krylov
    dimension at rho <= 1e-8, one right-hand side, FP64) from 16^2 to 4096^2, the time of one such
    sample, the batch throughput at 512^2 x 32, and the two passes of the step timed alone."""
    out = {"workload": "LGCP proposal: periodic 13-point prior tau = N^2, kappa2 = 100 / N^2 on the unit "
                       "torus, H = h^2 exp(x) at a smooth synthetic log-intensity; M = prior; FP64",
           "tol_rho": LGCP_TOL, "table1_preconditioned_m": {}, "ms_per_sample_k1": {}}
    for N in LGCP_TABLE_N:
        spec = workloads.lgcp_prior(N)
        op = gm.Operator.lattice(spec.shape, 2, spec.kappa2, spec.tau, "periodic", "f64")
        op.set_diagonal(workloads.lgcp_diagonal(N))
        op.set_circulant_precond()
        Z1 = torch.from_numpy(np.ascontiguousarray(workloads.gaussian_block(N * N, 1, 5, 1).T)).to("cuda:0")
        op.sample(Z1, tol=LGCP_TOL, m_max=40)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            X, info = op.sample(Z1, tol=LGCP_TOL, m_max=40)
        torch.cuda.synchronize()
        out["table1_preconditioned_m"][str(N)] = info[0]["m_used"]
        out["ms_per_sample_k1"][str(N)] = round(1000 * (time.perf_counter() - t0) / reps, 3)
        op.close()
        del X, Z1
    # Table 1's unpreconditioned row: Algorithm 1 on Q + H itself (CSR operator), the same column and tolerance
    out["table1_unpreconditioned_m"], out["ms_per_sample_k1_unpreconditioned"] = {}, {}
    for N in LGCP_UNPRE_N:
        spec = workloads.lgcp_prior(N)
        P = lgcp_posterior_csr(N, spec, workloads.lgcp_diagonal(N))
        op = gm.Operator.csr(P.shape[0], P.indptr, P.indices, P.data)
        Z1 = torch.from_numpy(np.ascontiguousarray(workloads.gaussian_block(N * N, 1, 5, 1).T)).to("cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = op.sample(Z1, tol=LGCP_TOL, m_max=LGCP_UNPRE_M_MAX)
        torch.cuda.synchronize()
        out["table1_unpreconditioned_m"][str(N)] = info[0]["m_used"] if info[0]["status"] == "OK" else None
        out["ms_per_sample_k1_unpreconditioned"][str(N)] = round(1000 * (time.perf_counter() - t0), 1)
        op.close()
        del X, Z1
    N, k = LGCP_BATCH
    spec = workloads.lgcp_prior(N)
    op = gm.Operator.lattice(spec.shape, 2, spec.kappa2, spec.tau, "periodic", "f64")
    op.set_diagonal(workloads.lgcp_diagonal(N))
    op.set_circulant_precond()
    Zb = torch.from_numpy(np.ascontiguousarray(workloads.gaussian_block(N * N, k, 5, 2).T)).to("cuda:0")
    op.sample(Zb, tol=LGCP_TOL, m_max=40)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        X, info = op.sample(Zb, tol=LGCP_TOL, m_max=40)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out["batch"] = {"side": N, "rhs": k, "samples_per_s": round(k / dt, 1), "ms_per_call": round(1000 * dt, 3),
                    "m_used_max": max(i["m_used"] for i in info)}
    kern = {}
    for name in ("lgcp_rows", "lgcp_cols"):
        r = gm.kernel_bench(op, name, k, reps=50, stream=stream)
        kern[name] = {"avg_us": round(r["avg_us"], 2), "bytes_per_launch": r["bytes"],
                      "achieved_gbs": round(r["achieved_gbs"], 1), "frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4)}
    out["kernels_512x512_32rhs"] = kern
    op.close()
    return out


LOGDET_COLUMNS = 64             # Lanczos columns per estimate (probes x colour classes), all variants


def logdet_leg(gm, torch):
    """Section 6 on workload C3 (1024^2, 13-point, kappa2 = 0.05, m = 80, FP32 storage): the plain
    Hutchinson estimate with 64 probes, and the coloured estimate of Section 6.1 for distance-p
    colourings (p = 1, 2) at the same number of Lanczos columns (probes = 64 / classes).  The
    variance per column (SE^2 x columns) compares the estimators at equal cost."""
    sp = workloads.C3_LATTICE
    seed = workloads.c3_probe_seed()
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, "f32")
    gm.autotune(op, LOGDET_COLUMNS, reps=5)   # the variants' 64, 63 and 54 columns share one columns class
    out = {"workload": "1024x1024 13-point lattice, kappa2 = 0.05, free boundary, m = 80, FP32 storage",
           "columns": LOGDET_COLUMNS, "m": workloads.C3_M, "variants": {}}
    for p in (0, 1, 2):
        col = op.distance_colouring(p)
        K = int(col.max()) + 1
        npb = max(2, LOGDET_COLUMNS // K)
        run = (lambda: op.logdet(npb, workloads.C3_M, seed=seed)) if p == 0 else \
              (lambda: op.logdet_coloured(npb, workloads.C3_M, col, seed=seed))
        run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mean, se, per = run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out["variants"][f"p{p}"] = {"classes": K, "probes": npb, "columns": npb * K, "estimate": mean,
                                    "std_err": se, "var_per_column": se * se * npb * K,
                                    "ms": round(1000 * dt, 2), "columns_per_s": round(npb * K / dt, 1)}
        if p == 2:
            # the same probes with twice the quadrature steps: the change is the m = 80 quadrature's bias,
            # which the standard error (probe variance only) does not see
            mean2, se2, _ = op.logdet_coloured(npb, 2 * workloads.C3_M, col, seed=seed)
            out["variants"]["p2_m160"] = {"classes": K, "probes": npb, "m": 2 * workloads.C3_M, "estimate": mean2,
                                          "std_err": se2}
    op.close()
    return out


ICHOL_DROPTOLS = (None, -1.0, 1e-2, 1e-3, 1e-4, 1e-5)   # None: no preconditioner; -1: IC(0)


def lattice_csr(N, order, kappa2):
    """Q = (kappa2 I + L)^order as CSR, L the 5-point graph Laplacian of the free N x N grid."""
    import scipy.sparse as sps
    T = sps.diags([-np.ones(N - 1), np.r_[1.0, 2 * np.ones(N - 2), 1.0], -np.ones(N - 1)], [-1, 0, 1])
    K = kappa2 * sps.identity(N * N) + sps.kron(T, sps.identity(N)) + sps.kron(sps.identity(N), T)
    P = sps.csr_matrix(K @ K if order == 2 else K)
    P.sort_indices()
    return P


def lgcp_posterior_csr(N, spec, d):
    """Q + diag(d) as CSR: Q = tau (kappa2 I + L)^2, L the 5-point graph Laplacian of the N x N torus
    (the LGCP prior of Section 3 with the Fisher information of the counts on the diagonal)."""
    import scipy.sparse as sps
    T = sps.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1]).tolil()
    T[0, N - 1] = T[N - 1, 0] = -1.0
    L = sps.kron(T, sps.identity(N)) + sps.kron(sps.identity(N), T)
    K = spec.kappa2 * sps.identity(N * N) + L
    P = sps.csr_matrix(spec.tau * (K @ K) + sps.diags(np.asarray(d, dtype=np.float64)))
    P.sort_indices()
    return P


def section52_matrix():
    """Q = (31^2 P_30)^2, P_30 the 5-point Dirichlet Laplacian on a 30 x 30 grid (n = 900), CSR."""
    import scipy.sparse as sps
    T = sps.diags([-np.ones(29), 2 * np.ones(30), -np.ones(29)], [-1, 0, 1])
    P = 31.0 ** 2 * (sps.kron(T, sps.identity(30)) + sps.kron(sps.identity(30), T))
    return sps.csr_matrix(P @ P)


def ichol_leg(gm, torch):
    """Figure 3's experiment on the GPU: Section 5.2's 900-point matrix, sampled with incomplete-Cholesky
    preconditioners (IC(0) and drop thresholds 1e-2 .. 1e-5) and without: Krylov dimension at
    rho <= 1e-8 (one right-hand side, CGS2, FP64), factor size and solve levels, and the time of a
    32-sample batch at that tolerance without reorthogonalisation."""
    Q = section52_matrix()
    n = Q.shape[0]
    z1 = torch.from_numpy(np.ascontiguousarray(workloads.gaussian_block(n, 1, 8, 0).T)).to("cuda:0")
    zb = torch.from_numpy(np.ascontiguousarray(workloads.gaussian_block(n, 32, 8, 1).T)).to("cuda:0")
    out = {"matrix": "(31^2 P_30)^2, n = 900 (Section 5.2)", "tol_rho": 1e-8, "variants": {}}
    for dt in ICHOL_DROPTOLS:
        op = gm.Operator.csr(n, Q.indptr, Q.indices, Q.data, "f64")
        rec = {}
        if dt is not None:
            rec["shift"] = op.set_ichol_precond(dt)
            rec["nnz_L"], rec["levels"], _ = op.ichol_info()
        _, info = op.sample(z1, tol=1e-8, m_max=900, reorth=True)
        rec["m_cgs2"] = info[0]["m_used"]
        op.sample(zb, tol=1e-8, m_max=900)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ib = op.sample(zb, tol=1e-8, m_max=900)
        torch.cuda.synchronize()
        rec["batch32_ms"] = round(1000 * (time.perf_counter() - t0), 2)
        rec["batch32_m_max"] = max(i["m_used"] for i in ib)
        out["variants"]["none" if dt is None else ("ic0" if dt < 0 else f"{dt:g}")] = rec
        op.close()
    return out


def plain_leg(gm, torch, reps=20):
    """Plain FP64 Lanczos, one sample (workload C0): 64 x 64 first-order lattice, kappa2 = 0.1, free
    boundary, full reorthogonalisation (CGS2), m_max = 200, stop at rho <= 1e-8.  Launch-bound at this
    size (n = 4096): the time is the latency of one request."""
    c = workloads.C0
    sp = c.lattice
    op = gm.Operator.lattice(sp.shape, sp.order, sp.kappa2, sp.tau, sp.boundary, "f64")
    Z = torch.from_numpy(np.ascontiguousarray(workloads.gaussian_block(sp.n, 1, 0, 0).T)).to("cuda:0")
    op.sample(Z, tol=c.tol, m_max=c.m_max, reorth=c.reorth)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        X, info = op.sample(Z, tol=c.tol, m_max=c.m_max, reorth=c.reorth)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out = {"samples_per_s": round(1.0 / dt, 2), "ms_per_sample": round(1000 * dt, 3),
           "us_per_iteration": round(1e6 * dt / max(1, info[0]["m_used"]), 1), "m_used": info[0]["m_used"],
           "rho": info[0]["rel_residual"], "status": info[0]["status"], "reorth": "CGS2",
           "_x": X[0].cpu().numpy()}   # for the accuracy check beside the oracle leg (removed before printing)
    op.close()
    return out


UNEVEN_TOL, UNEVEN_M_MAX = 1e-5, 600


def uneven_leg(gm, torch):
    """Uneven batch (workload C2): 256 first-order fields, side uniform in 32..256, kappa2 log-uniform
    in [1e-3, 1], 8 right-hand sides each, FP32 storage (FP64 scalars), all fields in one set of
    launches per Lanczos step; against the same fields sampled one call each, and against plain FP64
    Lanczos one sample at a time (column 0 of every field, same stopping rule)."""
    fields = workloads.uneven_fields()
    ops = [gm.Operator.lattice((s, s), 1, k2, 1.0, "free", "f32") for s, k2 in fields]
    Zs = [torch.from_numpy(np.ascontiguousarray(workloads.uneven_field_rhs(f, s).T)).to("cuda:0")
          for f, (s, _) in enumerate(fields)]
    ncol = sum(int(Z.shape[0]) for Z in Zs)
    tuned = set()
    for op, (s, _) in zip(ops, fields):      # one field per lattice class (ceil(log2) of the side)
        c = int(np.ceil(np.log2(s)))
        if c not in tuned:
            gm.autotune(op, 8, reps=5)
            tuned.add(c)
    gm.sample_batch(ops, Zs, tol=UNEVEN_TOL, m_max=UNEVEN_M_MAX)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xs, info = gm.sample_batch(ops, Zs, tol=UNEVEN_TOL, m_max=UNEVEN_M_MAX)
    torch.cuda.synchronize()
    dtb = time.perf_counter() - t0
    for _ in range(2):   # the first pass over the fields sizes the library's scratch pool, the second is timed
        t0 = time.perf_counter()
        for op, Z in zip(ops, Zs):
            op.sample(Z, tol=UNEVEN_TOL, m_max=UNEVEN_M_MAX)
        torch.cuda.synchronize()
        dts = time.perf_counter() - t0
    # plain FP64, k = 1: column 0 of every field
    ops64 = [gm.Operator.lattice((s, s), 1, k2, 1.0, "free", "f64") for s, k2 in fields]
    Z1 = [Z[:1].contiguous() for Z in Zs]
    for op, z in zip(ops64[:8], Z1[:8]):
        op.sample(z, tol=UNEVEN_TOL, m_max=UNEVEN_M_MAX)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for op, z in zip(ops64, Z1):
        op.sample(z, tol=UNEVEN_TOL, m_max=UNEVEN_M_MAX)
    torch.cuda.synchronize()
    dtp = time.perf_counter() - t0
    for op in ops64:
        op.close()
    ms = [i["m_used"] for i in info]
    col_n = [int(Z.shape[1]) for Z in Zs for _ in range(int(Z.shape[0]))]
    order = np.argsort([k2 for _, k2 in fields])
    picks = [int(order[(len(order) - 1) * q // 7]) for q in range(8)]   # 8 fields across the kappa2 range
    out = {"fields": len(fields), "columns": ncol, "unknowns": int(sum(s * s for s, _ in fields)), "storage": "f32",
           "tol_rho": UNEVEN_TOL, "m_max": UNEVEN_M_MAX, "m_used_min": min(ms), "m_used_max": max(ms),
           "not_converged": sum(i["status"] != "OK" for i in info),
           "batched_samples_per_s": round(ncol / dtb, 1), "batched_s": round(dtb, 3),
           "one_call_per_field_samples_per_s": round(ncol / dts, 1), "one_call_per_field_s": round(dts, 3),
           "batch_speedup": round(dts / dtb, 2),
           # algorithmic bytes: the one-pass step reads v_j, v_{j-1} and writes w_j (3 s n per column and
           # step); the final combination reads each column's m basis vectors once (s n m)
           "step_bytes": 3 * 4 * sum(i["m_used"] * n for i, n in zip(info, col_n)),
           "combine_bytes": 4 * sum(i["m_used"] * n for i, n in zip(info, col_n)),
           "plain_fp64_k1_samples_per_s": round(len(fields) / dtp, 1),
           "speedup_vs_plain_fp64_k1": round((ncol / dtb) / (len(fields) / dtp), 1),
           "_x": {f: (fields[f], Zs[f].cpu().numpy(), Xs[f].cpu().numpy()) for f in picks}}
    for op in ops:
        op.close()
    return out


def serving_leg(gm, torch, seconds):
    """Continuous batching (serve.Server: 4 worker streams, HBM budget = 80% of free memory) of the
    seeded Poisson request stream over 64 resident operators: 2D first-order lattices (side
    log-uniform on [64, 2048]) and 3D 7-point lattices (side 16..128), kappa2 log-uniform on
    [1e-3, 1], k uniform on 1..32; 75% samples, 25% log-det estimates.  Samples are served from
    FP32-storage operators at tol 1e-5 (m_max 600) and count only when their status is OK; log-dets
    (m = 80) run on the same FP32-storage operators with FP64 scalars, as the 1024^2 log-det estimate does.  Each offered rate gets an arrival window
    of `seconds` after a 2 s warm-up whose requests are served but not counted; the rates rise until the
    server falls behind (the queue does not drain within max(2 s, 10% of the window) after the last
    arrival).  The sustainable rate is the highest one it kept up with; latency runs from arrival to
    result."""
    from paper_1312_1476_amd import serve
    pool = workloads.serving_pool()
    ops = [gm.Operator.lattice(p.shape, p.order, p.kappa2, p.tau, "free", "f32") for p in pool]
    gm.set_hbm_budget(0)           # returns the scratch the earlier legs left cached in the library's pool
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    t0 = time.perf_counter()
    gm.pool_reserve(budget)        # one region for all scratch: no device allocation while serving
    t_reserve = time.perf_counter() - t0
    out = {"pool": "64 lattices: 2D 5-point (80%), 3D 7-point (20%); FP32 storage, FP64 scalars",
           "workers": 4, "hbm_budget_gb": round(budget / 1e9, 1), "reserved_region_s": round(t_reserve, 2),
           "arrival_window_s": seconds, "warmup_s": SERVE_WARMUP_S,
           "sample_tol": SERVE_TOL, "sample_m_max": SERVE_M_MAX, "logdet_m": SERVE_LOGDET_M, "rates": {}}
    sustainable = None
    for rate in SERVE_RATES:
        trace = workloads.serving_trace(rate=rate, duration=seconds + SERVE_WARMUP_S)
        reqs = [serve.ServeRequest(i, r.kind, r.op_index, r.k, r.seed,
                                   tol=SERVE_TOL, m_max=(SERVE_M_MAX if r.kind == "sample" else SERVE_LOGDET_M),
                                   t_arrival=r.t_arrival) for i, r in enumerate(trace)]
        counted = [q for q, r in zip(reqs, trace) if r.t_arrival >= SERVE_WARMUP_S]
        last_arrival = max(r.t_arrival for r in reqs)
        a0 = gm.pool_info()["device_allocs"]
        srv = serve.Server(ops, budget, workers=4, keep_results=False).start()
        t_start = time.perf_counter()
        st_all = srv.run_trace(reqs)
        srv.stop()
        device_allocs = gm.pool_info()["device_allocs"] - a0
        # the counted window: from the end of the warm-up to the last counted result
        wall = max(q.t_done for q in counted) - (t_start + SERVE_WARMUP_S)
        st = serve.stats(counted, wall)
        st["jobs"], st["retries"] = st_all["jobs"], st_all["retries"]
        drain = st_all["wall_s"] - last_arrival
        kept_up = drain <= max(2.0, 0.1 * seconds) and st["rejected"] == 0
        n_samples = sum(r.k for r in counted if r.kind == "sample")
        out["rates"][f"{rate}_req_per_s"] = {
            "requests": st["requests"], "completed": st["completed"], "rejected": st["rejected"],
            "two_pass": st["two_pass"], "batched": st["batched"], "jobs": st["jobs"], "retries": st["retries"],
            "pool_device_allocs": device_allocs,
            "wall_s": round(st["wall_s"], 2), "drain_s": round(drain, 2), "kept_up": kept_up,
            "completed_per_s": round(st["completed_per_s"], 2),
            "p50_latency_s": round(st["p50_latency_s"], 4), "p99_latency_s": round(st["p99_latency_s"], 4),
            "samples_ok": st["samples_ok"], "samples_not_ok": n_samples - st["samples_ok"],
            "samples_ok_per_s": round(st["samples_per_s"], 2), "probes_per_s": round(st["probes_per_s"], 2)}
        print(f"serving {rate} req/s: {st['completed']}/{st['requests']} counted in {st['wall_s']:.1f} s, "
              f"p99 {st['p99_latency_s']:.3f} s, kept up {kept_up}", file=sys.stderr, flush=True)
        if not kept_up:
            break
        sustainable = rate
    out["sustainable_rate_req_per_s"] = sustainable
    if sustainable is not None:
        r = out["rates"][f"{sustainable}_req_per_s"]
        out["at_sustainable_rate"] = {k: r[k] for k in ("p50_latency_s", "p99_latency_s", "samples_ok_per_s",
                                                        "probes_per_s", "completed_per_s")}
    gm.pool_reserve(0)
    for op in ops:
        op.close()
    return out


if __name__ == "__main__":
    main()
