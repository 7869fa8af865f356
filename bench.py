"""Benchmark: one ChFSI pass on the production-size FP64 workload on one MI355X.

Default workload (c1; synthetic, seeded): periodic cube L = 48 bohr, 24^3
cells of order p = 6 (M = 144^3 = 2,985,984 nodes, 343 nodes per cell), 64
Gaussian atoms (minimum separation 2 bohr) with local potentials and 4 s/p
projectors each, N = 256 wanted states, column blocks of B = 128, Chebyshev
degree m = 30.

A step is one pass of the hot path: the Chebyshev filter of every column
block (cell-wise H~.X with nonlocal projectors, fused recurrence), the
Cholesky-Gram-Schmidt orthonormalisation and the Rayleigh-Ritz step with
residual norms, all on inputs already resident in HBM.

Prints one JSON line.  ``value`` is the pass's algorithmic flop rate
(cell products, nonlocal products and subspace GEMMs counted without
padding) in GFLOP/s; ``ms_per_step`` is the pass time.  The ``roofline``
object reports the dominant kernel (the cell H~.X kernel) against the FP64
MFMA peak, timed with HIP events on the library's stream, with the HBM
traffic per launch from the committed rocprofv3 counter summary when it was
taken on the current kernel source.  The ``cpu_baseline`` object times the
FP64 oracle (numpy/scipy) on a bounded sample of the same workload on the
host cores.

Other workloads (``--workload``), each printing one JSON line of its own:
c2 (time to Delta E <= 1e-6 Ha at N = 1024 for FP64, FP32, BF16 and the
mixed schedule), c3 (32 batched complex k-point problems, sequential vs
persistent launch vs hipGraph, complex128 vs complex64), c4 (learned warm
start: training on solver output, passes saved on held-out configurations)
kernels (one 128-column filter step per precision), density (electron
density of the c2 block at the nodes and at the Gauss points of every cell,
with the Fermi level) and rrgep (the spectrum-splitting Rayleigh-Ritz step in
FP64 and in the paper's mixed precision: time at the c2 block size, accuracy
on a converged c4 problem) and scf (the self-consistent field loop on a
c4 system: Hartree potential, LDA exchange, one ChFSI pass per step,
Fermi level, density, Anderson mixing).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ChFSI pass time & cell H·X GFLOP/s; mixed/learned vs FP64 at ΔE≤1e-6 Ha"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0


def pass_flops(M, E, mcell, npairs, N, m, cplx=False):
    """Algorithmic flops of one pass (padding excluded)."""
    cf = 4.0 if cplx else 1.0
    cols = N * m + N                      # filter + W = H X_o of Rayleigh-Ritz
    cell = cols * 2.0 * mcell * mcell * E * cf
    nonlocal_ = cols * 2.0 * 2.0 * mcell * 4.0 * npairs * cf
    sub = (3.0 * M * N * (N + 1) + 4.0 * M * N * N) * cf
    return cell, nonlocal_, sub


def profiled_traffic(profile="cell_hx_c1_fp64.md", source="kernels_hx.hip"):
    """HBM bytes per launch of a kernel (by default the cell kernel's
    128-column filter step), from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source (else None)."""
    import hashlib
    import re
    prof = os.path.join(ROOT, "profiles", profile)
    src = os.path.join(ROOT, "paper_2203_07820_amd", "csrc", source)
    try:
        text = open(prof).read()
        m = re.search(r"```json\s*(\{.*?\})\s*```", text, re.S)
        rec = json.loads(m.group(1))
        if rec["source_sha256"] != hashlib.sha256(open(src, "rb").read()).hexdigest():
            return None
        return float(rec["traffic_bytes_per_launch"])
    except (OSError, AttributeError, KeyError, ValueError):
        return None


def cpu_baseline(sys_, B, seed):
    """Oracle cell-wise H~.X of one B-column block at full size, timed."""
    import numpy as np

    from oracle import fe
    cores = len(os.sched_getaffinity(0))
    op = fe.build_operator(sys_)
    X = np.random.default_rng(seed).standard_normal((op.M, B))
    t0 = time.perf_counter()
    fe.apply_cellwise(op, X, chunk=256)
    dt = time.perf_counter() - t0
    npairs_est = 0  # the oracle applies projectors at node level; count the cell products only
    fl = 2.0 * op.cells.shape[1] ** 2 * op.E * B + npairs_est
    return {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"one cell-wise H~X of a {B}-column FP64 block on the full workload "
                      f"(oracle.fe.apply_cellwise, numpy/scipy, {dt:.1f} s)",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--deterministic", action="store_true",
                    help="c1: assemble H~X colour class by colour class (chfsi_set_deterministic)")
    ap.add_argument("--workload", default="c1",
                    choices=["c0", "c1", "c2", "c3", "c4", "kernels", "density", "rrgep", "scf", "scf_k", "small_batch"],
                    help="c1: FP64 pass at production size (the headline line); c2: mixed precision "
                         "time-to-accuracy at N=1024; c3: batched k-point solves; c4: learned warm start; "
                         "kernels: one 128-column filter step per precision; density: electron density "
                         "of the c2 block; rrgep: spectrum-splitting Rayleigh-Ritz, FP64 vs mixed; "
                         "scf: self-consistent field loop on a c4 system (scf_k: at 8 k-points); small_batch: 64 small complex "
                         "problems batched vs one at a time")
    ap.add_argument("--out", default=None, help="write per-pass histories (npz) here")
    ap.add_argument("--max-passes", type=int, default=0, help="c2: pass cap per run (0: default)")
    ap.add_argument("--c2-runs", default="f32,mixed,f32_split_rr,bf16", help="c2: runs beside the FP64 reference")
    ap.add_argument("--c4-train", type=int, default=200, help="c4: training configurations solved")
    ap.add_argument("--c4-test", type=int, default=40, help="c4: held-out configurations")
    ap.add_argument("--c4-epochs", type=int, default=40, help="c4: passes over the training set")
    ap.add_argument("--c4-phase", default="all", choices=["all", "train", "eval"],
                    help="c4: all in one run, or one training chunk / the evaluation (network state in --c4-state)")
    ap.add_argument("--c4-range", default=None, help="c4 train phase: configurations a:b of this chunk")
    ap.add_argument("--c4-state", default=None, help="c4: network state file (npz) read and written by the phases")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    if args.workload == "c2":
        return run_c2(args)
    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "small_batch":
        return run_small_batch(args)
    if args.workload == "scf_k":
        return run_scf_k(args)
    if args.workload == "kernels":
        return run_kernels(args)
    if args.workload == "density":
        return run_density(args)
    if args.workload == "rrgep":
        return run_rrgep(args)
    if args.workload == "scf":
        return run_scf(args)
    if args.workload == "c0":
        return run_c0(args)
    return run_c1(args)


def run_c1(args):
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    sys_ = workloads.config("c1")
    N, B, m = 256, 128, 30
    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    if args.deterministic:
        ctx.set_deterministic(True)
    t0 = time.perf_counter()
    op = lib.Operator(ctx, sys_)
    t_build = time.perf_counter() - t0
    g = torch.Generator(device="cuda")
    g.manual_seed(sys_.seed + 1_000_000)
    X = torch.randn(op.M, N, dtype=torch.float64, device="cuda", generator=g)
    b, _ = op.bounds(20, seed=sys_.seed + 2_000_000)
    op.orthonormalize(X)
    th, r = op.rayleigh_ritz(X)
    a, aL = th[-1], th[0]
    print(f"# setup: M={op.M} E={op.E} pairs={op.npairs} build={t_build:.1f}s b={b:.3f} a={a:.4f} aL={aL:.4f}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        th, r = op.one_pass(X, N, m, B, a, b, aL)
        a, aL = th[-1], th[0]
        print(f"# warmup pass: max r={np.max(r):.3e}", file=sys.stderr, flush=True)
    ctx.set_timing(True)
    ctx.kernel_time(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        th, r = op.one_pass(X, N, m, B, a, b, aL)
        a, aL = th[-1], th[0]
        print(f"# pass {k}: max r={np.max(r):.3e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches, kfl = ctx.kernel_time(reset=True)
    ctx.set_timing(False)
    pass_s = (t1 - t0) / args.steps
    cell, nl, sub = pass_flops(op.M, op.E, op.mcell, op.npairs, N, m)
    total = cell + nl + sub
    achieved = kfl / (kms * 1e-3) / 1e12 if kms > 0 else None
    out = {
        "metric": METRIC,
        "value": total / pass_s / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": pass_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c1: FP64 Gamma-point ChFSI pass, 24^3 cells p=6 (M=2985984), 64 Gaussian "
                               "atoms with s/p projectors, N=256, B=128, m=30",
                   "M": op.M, "E": op.E, "mcell": op.mcell, "npairs": op.npairs, "N": N, "block": B,
                   "degree": m, "assembly": "colour classes" if args.deterministic else "atomic"},
        "pass_time_s": pass_s,
        "hx_kernel_tflops": achieved,
        "hx_kernel_ms_avg": kms / launches if launches else None,
        "hx_kernel_launches": launches,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": (achieved / PEAK_FP64_TFLOPS) if achieved else None,
                     "traffic": None if args.deterministic else profiled_traffic(),
                     "traffic_unit": "HBM bytes per 128-column launch"},
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(sys_, 64, seed=sys_.seed + 3_000_000)
        except Exception as e:  # the GPU figure stands on its own
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


def run_c0(args):
    """The small plain FP64 workload (4^3 cells, p = 4, M = 4096, 2 atoms, no
    projectors, N = B = 32, m = 20, 10 passes after the initial
    Rayleigh-Ritz): launch-bound.  Reports microseconds per pass of
    chfsi_solve (filter, CholGS, Rayleigh-Ritz, residuals) and of the same
    solve through chfsi_solve_batched with the filter captured in a hipGraph,
    the eigenvalues against the oracle's iteration, and the oracle timed on
    the host: the whole 10-pass solve with all cores and with one thread,
    and the gather / cell GEMM / scatter split of one 32-column H~X."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_limits

    import paper_2203_07820_amd as lib
    import workloads
    from oracle import chfsi as ochfsi
    from oracle import fe

    cfg = workloads.CONFIGS["c0"]
    s = workloads.config("c0")
    N, m, passes = cfg.nwanted, cfg.degree, cfg.passes
    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    op = lib.Operator(ctx, s)
    X0 = workloads.start_block(op.M, N, seed=s.seed + 1_000_000)
    v0 = workloads.lanczos_start(op.M, seed=s.seed + 2_000_000)
    b, _ = op.bounds(20, v0=torch.from_numpy(v0).cuda())
    runs = {}
    for name, graph in (("solve", False), ("solve_batched_graph", True)):
        per = []
        for rep in range(max(2, args.steps)):
            X = torch.from_numpy(X0).cuda()
            torch.cuda.synchronize()
            if graph:
                th, rs, st = ctx.solve_batched([op], [X], N, m=m, block=N, filter_prec=lib.F64,
                                               fixed_passes=passes, b_upper=b, use_graph=True, history=True)
                th, st = th[0], st[0]
            else:
                th, r, st = op.solve(X, N, m=m, block=N, fixed_passes=passes, b_upper=b, history=True)
            t = np.asarray(st["history"]["time_ms"])
            per.append(np.diff(t))
            split = {k: st[k] / passes * 1e3 for k in ("t_filter", "t_cholgs", "t_rr") if k in st}
        per = np.concatenate(per[1:])            # the first repetition warms up
        runs[name] = {"us_per_pass_median": float(np.median(per) * 1e3),
                      "us_per_pass_min": float(np.min(per) * 1e3), "passes_timed": int(per.size),
                      "us_per_pass_by_step": split, "theta": [float(x) for x in th]}
        log(f"# c0 {name}: {np.median(per) * 1e3:.0f} us per pass")
    # the oracle's iteration on the same inputs (and its time)
    ref_op = fe.build_operator(s)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    ref = ochfsi.solve(lambda v: fe.apply_cellwise(ref_op, v), X0, N, m=m, block=N, v0=v0, passes=passes, b=b)
    t_all = time.perf_counter() - t0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ochfsi.solve(lambda v: fe.apply_cellwise(ref_op, v), X0, N, m=m, block=N, v0=v0, passes=passes, b=b)
        t_one = time.perf_counter() - t0
    dtheta = max(float(np.max(np.abs(np.asarray(runs[k]["theta"]) - ref.theta))) for k in runs)
    # gather / GEMM / scatter of the oracle's cell-wise product on one block
    import scipy.sparse as sp
    A0 = ref_op.cell_matrix()
    X = X0.copy()
    t0 = time.perf_counter()
    Xc = (ref_op.D[:, None] * X)[ref_op.cells]
    t_g = time.perf_counter() - t0
    t0 = time.perf_counter()
    Yc = np.einsum("ij,cjb->cib", A0, Xc, optimize=True)
    t_m = time.perf_counter() - t0
    idx = ref_op.cells.ravel()
    S = sp.csr_matrix((np.ones(idx.size), (idx, np.arange(idx.size))), shape=(ref_op.M, idx.size))
    t0 = time.perf_counter()
    S @ Yc.reshape(-1, N)
    t_s = time.perf_counter() - t0
    fl_hx = 2.0 * op.mcell ** 2 * op.E * N
    fl_pass = (m + 1) * fl_hx
    us = runs["solve"]["us_per_pass_median"]
    out = {"metric": "ChFSI pass time, small FP64 workload", "value": us, "unit": "us", "n_gpus": 1,
           "steps": passes, "warmup": 1, "ms_per_step": us / 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "c0: 4^3 cells p=4 (M=4096), 2 Gaussian atoms, N=B=32, m=20, 10 passes",
                      "M": op.M, "E": op.E, "N": N, "degree": m},
           "runs": runs, "max_abs_theta_vs_oracle": dtheta,
           "floor_us_per_pass_fp64_mfma": fl_pass / (PEAK_FP64_TFLOPS * 1e12) * 1e6,
           "cpu_baseline": {"value": t_all / passes * 1e6, "unit": "us per pass", "cores": cores, "kind": "oracle",
                            "sample": f"oracle.chfsi.solve, {passes} passes with oracle.fe.apply_cellwise "
                                      f"({t_all:.2f} s)",
                            "single_thread_us_per_pass": t_one / passes * 1e6,
                            "hx_split_ms": {"gather": t_g * 1e3, "cell_gemm": t_m * 1e3, "scatter": t_s * 1e3,
                                            "gemm_GFLOPs": fl_hx / t_m / 1e9}}}
    print(json.dumps(out), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_c2(args):
    """Mixed precision at N = 1024 on the c1 operator: time to Delta E <= 1e-6 Ha
    for FP64, FP32, BF16 and the BF16 -> FP32 -> FP64 schedule, against an FP64
    reference run converged to max r <= 1e-9."""
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    sys_ = workloads.config("c1")
    N, nb, B, m = 1024, 128, 128, 30
    nfr = 128   # Ritz vectors rotated by the spectrum-splitting Rayleigh-Ritz of the split run
    cap = args.max_passes or 80
    ref_tol, target = 1e-9, 1e-6
    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    op = lib.Operator(ctx, sys_)
    b, _ = op.bounds(20, seed=sys_.seed + 2_000_000)
    log(f"# c2: M={op.M} N={N}+{nb} B={B} m={m} b={b:.3f}")

    def start():
        g = torch.Generator(device="cuda")
        g.manual_seed(sys_.seed + 1_000_000)
        return torch.randn(op.M, N + nb, dtype=torch.float64, device="cuda", generator=g)

    def run(name, prec0, switch, limit, stop, split=None):
        """split ("f64" or "mixed"): each pass is the filter followed by the
        paper's spectrum-splitting Rayleigh-Ritz (Algorithm 2) in FP64 or in
        its mixed precision (X then holds the orthonormal basis Psi_o, the
        Ritz values come from the generalised eigenproblem, no residuals);
        one full FP64 Rayleigh-Ritz at the end, timed, gives the Ritz
        vectors."""
        X = start()
        Pfr = torch.empty(op.M, nfr, dtype=torch.float64, device="cuda") if split else None
        torch.cuda.synchronize()
        ctx.set_timing(True)
        ctx.kernel_time(reset=True)
        t0 = time.perf_counter()
        op.orthonormalize(X)
        th, r = op.rayleigh_ritz(X)
        rec = {"t": [time.perf_counter() - t0], "prec": [-1], "maxr": [float(np.max(r[:N]))], "theta": [th.copy()]}
        prec = prec0
        for k in range(1, limit + 1):
            if split:
                op.filter(X, m, th[-1], b, th[0], prec=prec, block=B)
                th = op.rayleigh_ritz_split(X, nfr, Pfr, mixed=(split == "mixed"))
                r = np.full(N + nb, np.nan)
            else:
                th, r = op.one_pass(X, N, m, B, th[-1], b, th[0], n_buf=nb, filter_prec=prec)
            rec["t"].append(time.perf_counter() - t0)
            rec["prec"].append(prec)
            rec["maxr"].append(float(np.max(r[:N])))
            rec["theta"].append(th.copy())
            log(f"# {name} pass {k}: prec={prec} max r={rec['maxr'][-1]:.3e} t={rec['t'][-1]:.1f}s")
            if stop(th, r):
                break
            if switch:
                prec = lib.next_prec(prec, rec["maxr"], b)
        if split:
            th, r = op.rayleigh_ritz(X)
            torch.cuda.synchronize()
            rec["t"][-1] = time.perf_counter() - t0
            rec["maxr"][-1] = float(np.max(r[:N]))
            rec["theta"][-1] = th.copy()
        kms, launches, kfl = ctx.kernel_time(reset=True)
        ctx.set_timing(False)
        rec["hx_tflops"] = kfl / (kms * 1e-3) / 1e12 if kms > 0 else None
        rec = {k: (np.array(v) if isinstance(v, list) else v) for k, v in rec.items()}
        return X, rec

    # FP64 reference (also the FP64 metric run)
    Xref, ref = run("f64", lib.F64, False, cap, lambda th, r: np.max(r[:N]) <= ref_tol)
    # refine the reference with higher-degree FP64 passes (not part of any timing)
    th_ref = ref["theta"][-1].copy()
    r_ref = ref["maxr"][-1]
    for k in range(10):
        if r_ref <= ref_tol:
            break
        th_ref, rr = op.one_pass(Xref, N, 3 * m, B, th_ref[-1], b, th_ref[0], n_buf=nb)
        r_ref = float(np.max(rr[:N]))
        log(f"# reference refinement {k + 1} (degree {3 * m}): max r={r_ref:.3e}")
    lam = th_ref[:N].copy()
    gaps = np.diff(th_ref)[:N]
    # gap-separated prefixes [0, k): the largest k <= N whose gap to state k exceeds the threshold
    prefixes = {g: int(np.nonzero(gaps[:N - 1] > g)[0].max()) + 1 for g in (1e-6, 1e-4, 1e-3)}

    def dE(th):
        return float(np.max(np.abs(th[:N] - lam)))

    def sin_angle(X, k):
        C = Xref[:, :k].T @ X[:, :k]
        R = X[:, :k].clone()
        R.addmm_(Xref[:, :k], C, alpha=-1.0)
        G = (R.T @ R).cpu().numpy()
        del R
        return float(np.sqrt(max(np.linalg.eigvalsh(G)[-1], 0.0)))

    def summarize(rec, X):
        de = np.array([dE(t) for t in rec["theta"]])
        hit = np.nonzero(de <= target)[0]
        k = int(hit[0]) if hit.size else None
        out = {"passes_to_target": k, "time_to_target_s": float(rec["t"][k]) if k is not None else None,
               "final_dE": float(de[-1]), "min_dE": float(de.min()), "final_max_resid": float(rec["maxr"][-1]),
               "passes": int(len(rec["t"]) - 1), "sec_per_pass": float(np.median(np.diff(rec["t"]))),
               "hx_tflops": rec["hx_tflops"], "prec_per_pass": [int(p) for p in rec["prec"][1:]],
               "sin_subspace": {f"gap>{g:g} (k={k})": sin_angle(X, k) for g, k in prefixes.items()}}
        rec["dE"] = de
        return out

    results = {"f64": summarize(ref, Xref)}
    k64 = results["f64"]["passes_to_target"]
    results["f64"]["max_resid_at_target"] = float(ref["maxr"][k64]) if k64 is not None else None
    hists = {"f64": ref}
    stop_target = lambda th, r: dE(th) <= target  # noqa: E731
    wanted = set(args.c2_runs.split(",")) if args.c2_runs else set()
    plan = (("f32", lib.F32, False, cap, stop_target, None), ("mixed", lib.BF16, True, cap, stop_target, None),
            ("f32_split_rr", lib.F32, False, cap, stop_target, "f64"),
            ("f32_split_rr_mixed", lib.F32, False, cap, stop_target, "mixed"),
            ("bf16", lib.BF16, False, 8, lambda th, r: False, None))
    for name, prec0, switch, limit, stop, split in plan:
        if name not in wanted:
            continue
        X, rec = run(name, prec0, switch, limit, stop, split)
        results[name] = summarize(rec, X)
        hists[name] = rec
        del X
    t64 = results["f64"]["time_to_target_s"]
    tmix = results.get("mixed", {}).get("time_to_target_s")
    t32 = results.get("f32", {}).get("time_to_target_s")
    tsp = results.get("f32_split_rr", {}).get("time_to_target_s")
    # the headline is the fastest reduced-precision route that reaches the
    # target (every route's figures stay in "runs")
    routes = {n: r["time_to_target_s"] for n, r in results.items()
              if n not in ("f64", "bf16") and r.get("time_to_target_s") is not None}
    best = min(routes, key=routes.get) if routes else None
    dtypes = {"f32": "f32 filter, f64 subspace", "mixed": "bf16/f32 filter, f64 subspace",
              "f32_split_rr": "f32 filter, f64 spectrum-split Rayleigh-Ritz",
              "f32_split_rr_mixed": "f32 filter, mixed spectrum-split Rayleigh-Ritz"}
    out = {
        "metric": "time to Delta E <= 1e-6 Ha, mixed precision vs FP64 (c2)",
        "value": routes.get(best), "unit": "s", "n_gpus": 1,
        "steps": results.get(best, {}).get("passes"), "warmup": 0,
        "ms_per_step": 1e3 * results.get(best, results["f64"])["sec_per_pass"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": dtypes.get(best, "f64"), "data": "synthetic",
        "route": best,
        "config": {"workload": "c2: c1 operator (24^3 cells p=6, M=2985984, 64 atoms with projectors), N=1024 "
                               "+ 128 buffer columns, B=128, m=30, start N(0,1) seeded",
                   "N": N, "n_buf": nb, "block": B, "degree": m, "b_upper": b,
                   "reference": f"FP64 run (the f64 run, then up to 10 degree-{3 * m} passes) to max r <= {ref_tol:g}",
                   "reference_max_resid": r_ref, "gap_prefixes": {f"{g:g}": k for g, k in prefixes.items()}},
        "speedup_vs_f64": {"f32": (t64 / t32) if (t64 and t32) else None,
                           "mixed": (t64 / tmix) if (t64 and tmix) else None,
                           "f32_split_rr": (t64 / tsp) if (t64 and tsp) else None,
                           "best": (t64 / routes[best]) if (t64 and best) else None},
        "runs": results,
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = c2_oracle_sample(sys_, Xref, th_ref, ref_tol)
        except Exception as e:  # the GPU figures stand on their own
            out["cpu_baseline"] = {"error": repr(e)}
    if args.out:
        np.savez_compressed(args.out, **{f"{n}_{k}": v for n, h in hists.items() for k, v in h.items()
                                         if isinstance(v, np.ndarray)})
    print(json.dumps(out), flush=True)


def run_c3(args):
    """Batched uneven k-point solves: 8 periodic p = 5 systems x 4 Monkhorst-Pack
    k-points (32 complex Bloch operators).  Per pass: each problem solved on
    its own (complex128) against one batched solve (persistent launch per
    Chebyshev step, without and with the hipGraph) in complex128 and complex64,
    tile shapes from the autotuner."""
    import tempfile

    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    m, B, K = 30, 128, max(1, args.steps)
    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    systems, Ns, tags = [], [], []
    for i, (nc, na, nw) in enumerate(workloads.C3_SYSTEMS):
        base = workloads.config("c3", i)
        for j, kp in enumerate(workloads.kpoints_mp4(base.L)):
            systems.append(base.with_k(kp))
            Ns.append(nw)
            tags.append((i, j))
    t0 = time.perf_counter()
    ops = [lib.Operator(ctx, s) for s in systems]
    log(f"# c3: {len(ops)} operators built in {time.perf_counter() - t0:.1f}s; sum M={sum(o.M for o in ops)}")
    bs = [ops[q].bounds(20, seed=3000 + tags[q][0] + 2_000_000 + 10 * tags[q][1])[0] for q in range(len(ops))]
    cell = nl = sub = 0.0
    for q, o in enumerate(ops):
        c_, n_, s_ = pass_flops(o.M, o.E, o.mcell, o.npairs, Ns[q], m, cplx=True)
        cell, nl, sub = cell + c_, nl + n_, sub + s_
    total = cell + nl + sub

    def fill():
        Xs = []
        for q, o in enumerate(ops):
            g = torch.Generator(device="cuda")
            g.manual_seed(3000 + tags[q][0] + 1_000_000 + 10 * tags[q][1])
            Xs.append(torch.randn(o.M, Ns[q], dtype=torch.complex128, device="cuda", generator=g))
        torch.cuda.synchronize()
        return Xs

    def per_pass_ms(h):
        return float(np.median(np.diff(h["time_ms"])))

    tune_path = os.path.join(tempfile.gettempdir(), "chfsi_tuning_c3.json")
    tuning = {}
    for name, prec in (("c128", lib.C128), ("c64", lib.C64)):
        t1 = time.perf_counter()
        tuning[name] = ctx.autotune(5, prec, B, cache_json=tune_path)
        log(f"# autotune {name}: {tuning[name]} ({time.perf_counter() - t1:.1f}s)")

    modes = {}
    # each problem on its own, complex128 (cell-kernel launches timed with HIP events)
    Xs = fill()
    ctx.set_timing(True)
    ctx.kernel_time(reset=True)
    seq_ms, seq_filter_ms, seq_theta = 0.0, 0.0, []
    for q, o in enumerate(ops):
        th, r, st = o.solve(Xs[q], Ns[q], m, B, fixed_passes=K, filter_prec=lib.C128, b_upper=bs[q], history=True)
        seq_ms += per_pass_ms(st["history"])
        seq_filter_ms += st["t_filter"] / K
        seq_theta.append(th)
        if q % 4 == 3:
            log(f"# sequential: system {tags[q][0]} done, running pass time {seq_ms:.0f} ms")
    kms_seq, n_seq, kfl_seq = ctx.kernel_time(reset=True)
    ctx.set_timing(False)
    modes["sequential_c128"] = {"pass_ms": seq_ms, "filter_ms_per_pass": seq_filter_ms,
                                "tflops": total / (seq_ms * 1e-3) / 1e12,
                                "cell_kernel_ms_per_pass": kms_seq / K, "cell_kernel_launches": n_seq,
                                "cell_kernel_tflops": kfl_seq / (kms_seq * 1e-3) / 1e12}
    del Xs
    thetas = {}
    for name, prec, graph in (("batched_c128", lib.C128, False), ("batched_graph_c128", lib.C128, True),
                              ("batched_graph_c64", lib.C64, True)):
        Xs = fill()
        t1 = time.perf_counter()
        timed = not graph   # the graph's launches are not timed one by one
        ctx.set_timing(timed)
        ctx.kernel_time(reset=True)
        th, rs, st = ctx.solve_batched(ops, Xs, Ns, m, B, prec, fixed_passes=K, b_upper=bs, use_graph=graph,
                                       history=True)
        kms_b, n_b, kfl_b = ctx.kernel_time(reset=True)
        ctx.set_timing(False)
        big = int(np.argmax([o.M * Ns[q] for q, o in enumerate(ops)]))
        pm = per_pass_ms(st[big]["history"])
        modes[name] = {"pass_ms": pm, "filter_ms_per_pass": st[big]["t_filter"] / K,
                       "tflops": total / (pm * 1e-3) / 1e12,
                       "max_resid": float(max(np.max(rs[q][:Ns[q]]) for q in range(len(ops))))}
        if timed:
            modes[name].update(cell_kernel_ms_per_pass=kms_b / K, cell_kernel_launches=n_b,
                               cell_kernel_tflops=kfl_b / (kms_b * 1e-3) / 1e12)
        thetas[name] = th
        log(f"# {name}: {pm:.0f} ms per pass ({time.perf_counter() - t1:.1f}s)")
        del Xs
    d_seq = max(float(np.max(np.abs(thetas["batched_graph_c128"][q] - seq_theta[q]))) for q in range(len(ops)))
    d_c64 = max(float(np.max(np.abs(thetas["batched_graph_c64"][q][:Ns[q]] - thetas["batched_graph_c128"][q][:Ns[q]])))
                for q in range(len(ops)))
    pm = modes["batched_graph_c128"]["pass_ms"]
    out = {
        "metric": "batched k-point ChFSI pass (c3): algorithmic GFLOP/s of one pass over 32 problems",
        "value": total / (pm * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": K, "warmup": 0,
        "ms_per_step": pm, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128", "data": "synthetic",
        "config": {"workload": "c3: 8 periodic p=5 systems (8^3..20^3 cells, 8..48 atoms with projectors, "
                               "N=64..384) x 4 Monkhorst-Pack k-points, m=30, B=min(N,128)",
                   "problems": len(ops), "sum_M": int(sum(o.M for o in ops)), "degree": m, "block": B,
                   "pass_flops": total},
        "modes": modes,
        "speedup_batched_graph_vs_sequential": modes["sequential_c128"]["pass_ms"] / pm,
        # the same cell-kernel work (filter steps and Rayleigh-Ritz products of
        # all 32 problems) in one launch per step against one launch per
        # problem and step: > 1 means the batched launch keeps the GPU busier
        "load_balance_efficiency": (modes["sequential_c128"]["cell_kernel_ms_per_pass"] /
                                    modes["batched_c128"]["cell_kernel_ms_per_pass"]),
        "speedup_c64_vs_c128": pm / modes["batched_graph_c64"]["pass_ms"],
        "max_dtheta_batched_vs_sequential": d_seq,
        "max_dtheta_c64_vs_c128_after_same_passes": d_c64,
        "tuning": tuning,
    }
    print(json.dumps(out), flush=True)


def run_small_batch(args):
    """Many small problems: 16 periodic p = 5 boxes of 3^3 .. 6^3 cells (M =
    3,375 .. 27,000, 2 .. 6 atoms with projectors, N = 16 .. 48) at the 4
    Monkhorst-Pack k-points, 64 complex problems, m = 20, one block each.
    One at a time, no launch fills the GPU (at most 432 workgroups per step);
    the batched filter runs every problem's step in one launch (three with the
    projections).  Reports the pass time over all problems for each problem
    solved alone and for the batched solve without and with the hipGraph."""
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    m, K = 20, max(1, args.steps)
    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    systems, Ns, tags = [], [], []
    for i, (nc, na, nw) in enumerate(workloads.SMALL_BATCH_SYSTEMS):
        base = workloads.config("small_batch", i)
        for j, kp in enumerate(workloads.kpoints_mp4(base.L)):
            systems.append(base.with_k(kp))
            Ns.append(nw)
            tags.append((i, j))
    ops = [lib.Operator(ctx, s) for s in systems]
    B = max(Ns)
    bs = [ops[q].bounds(20, seed=6000 + tags[q][0] + 2_000_000 + 10 * tags[q][1])[0] for q in range(len(ops))]
    total = 0.0
    for q, o in enumerate(ops):
        total += sum(pass_flops(o.M, o.E, o.mcell, o.npairs, Ns[q], m, cplx=True))

    def fill():
        Xs = []
        for q, o in enumerate(ops):
            g = torch.Generator(device="cuda")
            g.manual_seed(6000 + tags[q][0] + 1_000_000 + 10 * tags[q][1])
            Xs.append(torch.randn(o.M, Ns[q], dtype=torch.complex128, device="cuda", generator=g))
        torch.cuda.synchronize()
        return Xs

    def per_pass_ms(h):
        return float(np.median(np.diff(h["time_ms"])))

    modes, thetas = {}, {}
    for rep in range(2):   # the first round warms up (code objects, workspaces, the graph)
        Xs = fill()
        seq_ms, seq_filter_ms, seq_theta = 0.0, 0.0, []
        for q, o in enumerate(ops):
            th, r, st = o.solve(Xs[q], Ns[q], m, B, fixed_passes=K, filter_prec=lib.C128, b_upper=bs[q],
                                history=True)
            seq_ms += per_pass_ms(st["history"]) if K > 1 else st["t_total"]
            seq_filter_ms += st["t_filter"] / K
            seq_theta.append(th)
        modes["sequential_c128"] = {"pass_ms": seq_ms, "filter_ms_per_pass": seq_filter_ms}
        thetas["sequential_c128"] = seq_theta
        del Xs
        for name, graph in (("batched_c128", False), ("batched_graph_c128", True)):
            Xs = fill()
            th, rs, st = ctx.solve_batched(ops, Xs, Ns, m, B, lib.C128, fixed_passes=K, b_upper=bs,
                                           use_graph=graph, history=True)
            modes[name] = {"pass_ms": per_pass_ms(st[0]["history"]) if K > 1 else st[0]["t_total"],
                           "filter_ms_per_pass": st[0]["t_filter"] / K,
                           "max_resid": float(max(np.max(rs[q][:Ns[q]]) for q in range(len(ops))))}
            thetas[name] = th
            del Xs
        log(f"# round {rep}: " + ", ".join(f"{k} {v['pass_ms']:.1f} ms" for k, v in modes.items()))
    for v in modes.values():
        v["tflops"] = total / (v["pass_ms"] * 1e-3) / 1e12
    d_seq = max(float(np.max(np.abs(thetas["batched_graph_c128"][q] - thetas["sequential_c128"][q])))
                for q in range(len(ops)))
    pm = modes["batched_graph_c128"]["pass_ms"]
    out = {
        "metric": "batched ChFSI pass over 64 small complex problems", "value": pm, "unit": "ms",
        "n_gpus": 1, "steps": K, "warmup": K, "ms_per_step": pm, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": "16 periodic p=5 boxes (3^3..6^3 cells, 2..6 atoms with projectors, N=16..48) x 4 "
                               "Monkhorst-Pack k-points, m=20, one block per problem",
                   "problems": len(ops), "sum_M": int(sum(o.M for o in ops)), "degree": m, "block": B,
                   "pass_flops": total},
        "modes": modes,
        "speedup_batched_graph_vs_sequential": modes["sequential_c128"]["pass_ms"] / pm,
        "filter_speedup_batched_graph_vs_sequential": (modes["sequential_c128"]["filter_ms_per_pass"] /
                                                       modes["batched_graph_c128"]["filter_ms_per_pass"]),
        "max_dtheta_batched_vs_sequential": d_seq,
    }
    print(json.dumps(out), flush=True)


def run_c4(args):
    """Learned warm start: seeded 16-atom configurations in a 12^3-cell p = 5
    box solved by plain FP64 ChFSI from random starts to max r <= 1e-6; the
    network (32 -> 128 -> 128 -> 128, tanh, FP32) is trained on their Ritz
    blocks by the library's own kernels, then held-out configurations are
    solved from the network's block and from a random block.

    --c4-phase all runs everything in one process.  For the full
    configuration (1800 + 200), which does not fit one run, --c4-phase train
    --c4-range a:b solves and trains on one chunk of training configurations
    (kept on the device for the chunk's epochs), continuing from the network
    state in --c4-state (weights and the feature standardisation, fixed by
    the first chunk) and writing it back; --c4-phase eval then solves the
    held-out configurations from both starts."""
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    N, nb, B, m, tol = 128, 32, 128, 30, 1e-6
    torch.cuda.set_device(0)
    ctx = lib.Context(0)

    def random_block(op, j):
        g = torch.Generator(device="cuda")
        g.manual_seed(4000 + j + 1_000_000)
        return torch.randn(op.M, N + nb, dtype=torch.float64, device="cuda", generator=g)

    def solve(op, X, j):
        return op.solve(X, N, m, B, n_buf=nb, tol=tol, max_passes=80, seed=4000 + j + 2_000_000)

    def featurize(op):
        F = torch.empty(op.M, 32, dtype=torch.float32, device="cuda")
        lib.features(op, F)
        return F

    state = {}
    if args.c4_state and os.path.exists(args.c4_state):
        with np.load(args.c4_state) as z:
            state = {k: z[k] for k in z.files}
    net = lib.Network(ctx, 32, 128, N, seed=4242)
    if "params" in state:
        net.set_params(state["params"])
        net.set_norm(state["mean"], state["scale"])

    def train_chunk(lo, hi, epochs):
        # 1. training data: converged Ritz blocks of configurations lo .. hi - 1
        t0 = time.perf_counter()
        feats, targets, gen_passes = [], [], []
        for j in range(lo, hi):
            op = lib.Operator(ctx, workloads.config("c4", j))
            X = random_block(op, j)
            th, r, st = solve(op, X, j)
            feats.append(featurize(op))
            targets.append(X[:, :N].float().contiguous())
            gen_passes.append(st["passes"])
            del X
            op.close()
            if (j - lo) % 10 == 9:
                log(f"# c4 data: {j + 1 - lo}/{hi - lo} solved, mean passes {np.mean(gen_passes):.1f}, "
                    f"{time.perf_counter() - t0:.0f}s")
        t_gen = time.perf_counter() - t0
        # 2. standardisation from a host subsample of the first chunk's features
        if "mean" not in state:
            sample = np.concatenate([F[::64].cpu().numpy().astype(np.float64) for F in feats])
            state["mean"], state["scale"] = sample.mean(axis=0), sample.std(axis=0) + 1e-6
            net.set_norm(state["mean"], state["scale"])
        # 3. training (Adam, one configuration per step)
        t0 = time.perf_counter()
        rng = np.random.default_rng(7 + lo)
        curve = []
        for ep in range(epochs):
            losses = [net.train_step(feats[q], targets[q], lr=1e-3) for q in rng.permutation(hi - lo)]
            curve.append(float(np.mean(losses)))
            if ep % 5 == 4 or ep == epochs - 1:
                log(f"# c4 training epoch {ep + 1}: mean loss {curve[-1]:.4f} ({time.perf_counter() - t0:.0f}s)")
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        return t_gen, t_train, curve, gen_passes

    def save_state():
        if args.c4_state:
            os.makedirs(os.path.dirname(os.path.abspath(args.c4_state)), exist_ok=True)
            np.savez(args.c4_state, **state)

    if args.c4_phase == "train":
        lo, hi = (int(x) for x in args.c4_range.split(":"))
        t_gen, t_train, curve, gen_passes = train_chunk(lo, hi, args.c4_epochs)
        state["params"] = net.params()
        state["chunks"] = np.append(state.get("chunks", np.zeros((0, 2), dtype=np.int64)).reshape(-1, 2),
                                    [[lo, hi]], axis=0)
        state["loss_curve"] = np.append(state.get("loss_curve", np.zeros(0)), curve)
        state["gen_passes"] = np.append(state.get("gen_passes", np.zeros(0)), gen_passes)
        state["gen_s"] = float(state.get("gen_s", 0.0)) + t_gen
        state["train_s"] = float(state.get("train_s", 0.0)) + t_train
        save_state()
        print(json.dumps({"c4_train_chunk": [lo, hi], "epochs": args.c4_epochs, "data_generation_s": t_gen,
                          "training_s": t_train, "loss_first_last": [curve[0], curve[-1]],
                          "data_passes_mean": float(np.mean(gen_passes))}), flush=True)
        return
    if args.c4_phase == "all":
        t_gen, t_train, curve, gen_passes = train_chunk(0, args.c4_train, args.c4_epochs)
        state.update(params=net.params(), chunks=np.array([[0, args.c4_train]]), loss_curve=np.array(curve),
                     gen_passes=np.array(gen_passes, dtype=float), gen_s=t_gen, train_s=t_train)
        save_state()
    if "params" not in state:
        raise SystemExit("c4 eval: no trained network (run the train phase first, or --c4-phase all)")
    chunks = np.asarray(state["chunks"]).reshape(-1, 2)
    n_train = int(np.sum(chunks[:, 1] - chunks[:, 0]))
    curve = np.asarray(state["loss_curve"])
    n_test = args.c4_test
    # 4. held-out configurations: random start vs learned start
    rows, captures = [], []
    for i in range(n_test):
        j = 1800 + i
        op = lib.Operator(ctx, workloads.config("c4", j))
        X = random_block(op, j)
        _, _, st_r = solve(op, X, j)
        Q = X[:, :N].float().contiguous()
        Qbuf = X[:, N:].clone() if i < 8 else None   # Ritz vectors of states N+1 .. N+n_buf
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        F = featurize(op)
        Xl = torch.empty(op.M, N + nb, dtype=torch.float64, device="cuda")
        fallback = lib.initial_block(op, Xl, net, seed=4000 + j + 1_000_000)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t1
        _, _, st_l = solve(op, Xl, j)
        loss, _ = net.loss_grad(F, Q, want_grads=False)
        if i < 8:
            # diagnostic: how much of each converged state the network's span holds
            Y = torch.empty(op.M, N, dtype=torch.float32, device="cuda")
            net.forward(F, Y)
            Qy, _ = torch.linalg.qr(Y.double())
            Cq = Qy.T @ torch.cat([Q.double(), Qbuf], dim=1)
            captures.append((Cq * Cq).sum(dim=0).cpu().numpy())
            del Y, Qy, Cq, Qbuf
        rows.append({"passes_random": st_r["passes"], "passes_learned": st_l["passes"],
                     "ms_random": st_r["t_total"], "ms_learned": st_l["t_total"] + 1e3 * t_init,
                     "converged": bool(st_r["converged"] and st_l["converged"]), "fallback": fallback,
                     "heldout_loss": loss})
        del X, Xl, F, Q
        op.close()
        if i % 10 == 9 or i == n_test - 1:
            log(f"# c4 held-out {i + 1}/{n_test}: passes random {st_r['passes']} learned {st_l['passes']}"
                f"{' (fallback)' if fallback else ''}")
    pr = np.array([r_["passes_random"] for r_ in rows], dtype=float)
    pl = np.array([r_["passes_learned"] for r_ in rows], dtype=float)
    tr = np.array([r_["ms_random"] for r_ in rows])
    tl = np.array([r_["ms_learned"] for r_ in rows])
    epochs = int(curve.size // max(1, len(chunks)))
    out = {
        "metric": "filter passes saved by the learned warm start at max r <= 1e-6 (c4)",
        "value": float(np.mean(pr - pl)), "unit": "passes", "n_gpus": 1, "steps": n_test, "warmup": 0,
        "ms_per_step": float(np.mean(tl)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 solve, f32 network", "data": "synthetic",
        "config": {"workload": "c4: 16 Gaussian atoms with projectors in a 12^3-cell p=5 box (L=24, M=216000), "
                               f"N=128 + {nb} buffer, B=128, m=30, tol 1e-6; {n_train} training and {n_test} "
                               "held-out configurations (seeds 4000+j, held out from j=1800)",
                   "n_train": n_train, "n_test": n_test, "epochs_per_chunk": epochs,
                   "training_chunks": chunks.tolist()},
        "passes_random_mean": float(pr.mean()), "passes_random_sd": float(pr.std()),
        "passes_learned_mean": float(pl.mean()), "passes_learned_sd": float(pl.std()),
        "passes_saved_sd": float(np.std(pr - pl)),
        "time_to_tol_ms_random_mean": float(tr.mean()), "time_to_tol_ms_learned_mean": float(tl.mean()),
        "fallbacks": int(sum(r_["fallback"] for r_ in rows)),
        "all_converged": bool(all(r_["converged"] for r_ in rows)),
        "train_loss_first_last": [float(curve[0]), float(curve[-1])],
        "heldout_loss_mean": float(np.mean([r_["heldout_loss"] for r_ in rows])),
        "data_generation_s": float(state["gen_s"]), "training_s": float(state["train_s"]),
        "data_passes_mean": float(np.mean(state["gen_passes"])),
        "captured_fraction_by_state_quarter": [float(x) for x in
                                               np.mean(captures, axis=0)[:N].reshape(4, -1).mean(axis=1)],
        "captured_fraction_buffer_states": float(np.mean(np.mean(captures, axis=0)[N:])),
        "captured_fraction_random_block": N / 216000.0,
    }
    print(json.dumps(out), flush=True)


PEAKS_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "c128": 78.6, "c64": 157.3}


def run_kernels(args):
    """The cell kernel in every precision on its production operator: 128-column
    filter steps (the fused recurrence) on the c1 operator (real: F64, F32,
    BF16) and on the largest c3 operator at its first k-point (C128, C64)."""
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    B, steps = 128, max(2, args.steps * 4)
    c3 = workloads.config("c3", 7)
    c1, c3k = workloads.config("c1"), c3.with_k(workloads.kpoints_mp4(c3.L)[0])
    cases = [("f64", lib.F64, c1), ("f32", lib.F32, c1), ("bf16", lib.BF16, c1),
             ("c128", lib.C128, c3k), ("c64", lib.C64, c3k)]
    res, ops = {}, {}
    for name, prec, sys_ in cases:
        if id(sys_) not in ops:
            ops.clear()
            ops[id(sys_)] = lib.Operator(ctx, sys_)
        op = ops[id(sys_)]
        dt = torch.complex128 if op.is_complex else torch.float64
        X = torch.randn(op.M, B, dtype=dt, device="cuda")
        b, _ = op.bounds(20, seed=1)
        op.filter(X, 2, b * 0.1, b, -1.0, prec=prec, block=B)   # warm-up
        torch.cuda.synchronize()
        ctx.set_timing(True)
        ctx.kernel_time(reset=True)
        op.filter(X, steps, b * 0.1, b, -1.0, prec=prec, block=B)
        kms, n, kfl = ctx.kernel_time(reset=True)
        ctx.set_timing(False)
        ebytes = {"f64": 8, "f32": 4, "bf16": 4, "c128": 16, "c64": 8}[name]
        ms = kms / n
        tf = kfl / (kms * 1e-3) / 1e12
        hbm = 3.0 * op.M * B * ebytes / (ms * 1e-3) / 1e9
        res[name] = {"ms_per_step": ms, "tflops": tf, "frac_mfma_peak": tf / PEAKS_TFLOPS[name],
                     "algorithmic_GBps": hbm, "frac_hbm_peak": hbm / PEAK_HBM_GBS, "M": op.M, "E": op.E,
                     "mcell": op.mcell, "npairs": op.npairs, "launches": n}
        log(f"# {name}: {ms:.3f} ms per step, {tf:.2f} TFLOP/s, {hbm:.0f} GB/s algorithmic")
        del X
    # per-cell Gauss-quadrature potential on the c1 mesh: build time and the
    # FP64 filter step with one cell matrix per cell
    ops.clear()
    t0 = time.perf_counter()
    opq = lib.Operator(ctx, c1, potential="quadrature")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    X = torch.randn(opq.M, B, dtype=torch.float64, device="cuda")
    b, _ = opq.bounds(20, seed=1)
    opq.filter(X, 2, b * 0.1, b, -1.0, prec=lib.F64, block=B)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.kernel_time(reset=True)
    opq.filter(X, steps, b * 0.1, b, -1.0, prec=lib.F64, block=B)
    kms, n, kfl = ctx.kernel_time(reset=True)
    ctx.set_timing(False)
    ms = kms / n
    cellmat_gb = opq.E * ((opq.mcell + 15) // 16 * 16) ** 2 * 8 / 1e9
    res["f64_quadrature_potential"] = {
        "ms_per_step": ms, "tflops": kfl / (kms * 1e-3) / 1e12, "frac_mfma_peak": kfl / (kms * 1e-3) / 1e12 / 78.6,
        "build_s": build_s, "cell_matrices_GB": cellmat_gb, "launches": n}
    log(f"# f64 quadrature potential: {ms:.3f} ms per step (build {build_s:.1f} s, {cellmat_gb:.1f} GB of cell matrices)")
    del X, opq
    out = {"metric": "cell H·X filter step per precision", "value": res["f64"]["tflops"] * 1e3, "unit": "GFLOP/s",
           "n_gpus": 1, "steps": steps, "warmup": 2, "ms_per_step": res["f64"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "128-column filter steps: c1 operator (F64, F32, BF16); largest c3 operator "
                                  "at its first k-point (C128, C64); c1 with the per-cell quadrature potential "
                                  "(F64)"},
           "kernels": res}
    print(json.dumps(out), flush=True)


def run_density(args):
    """Electron density of a c2-sized block: the c1 operator (M = 2,985,984,
    p = 6) with 1024 + 128 FP64 columns, at the nodes and at the 343 Gauss
    points of each of the 13,824 cells, weights 2 f_i from the Fermi level of
    a synthetic spectrum (N_e = 2048, Fermi-Dirac smearing at 500 K)."""
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    s = workloads.config("c1")
    op = lib.Operator(ctx, s)
    ncols, steps = 1152, max(2, args.steps * 2)
    g = torch.Generator(device="cuda").manual_seed(61)
    X = torch.randn(op.M, ncols, dtype=torch.float64, device="cuda", generator=g)
    theta = np.sort(np.random.default_rng(62).uniform(-1.0, 1.5, ncols))
    kT = 500.0 * 3.166811563e-6     # Hartree per kelvin
    t0 = time.perf_counter()
    mu, f = lib.fermi_level(theta, 2048.0, kT)
    fermi_ms = (time.perf_counter() - t0) * 1e3
    w = 2.0 * f
    nq = (s.p + 1) ** 3
    outs = {"nodes": (lib.RHO_NODES, torch.empty(op.M, dtype=torch.float64, device="cuda")),
            "gauss": (lib.RHO_GAUSS, torch.empty(op.E * nq, dtype=torch.float64, device="cuda"))}
    res = {}
    for name, (points, out) in outs.items():
        for _ in range(max(1, args.warmup)):
            op.density(X, w, out, points=points)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(steps):
            op.density(X, w, out, points=points)
        e1.record(ctx.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / steps
        nbytes = op.M * ncols * 8 + op.M * 8 + out.numel() * 8   # X, M^-1/2, rho
        res[name] = {"ms": ms, "algorithmic_bytes": nbytes, "GBps": nbytes / (ms * 1e-3) / 1e9,
                     "frac_hbm_peak": nbytes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "outputs": out.numel()}
        log(f"# density {name}: {ms:.3f} ms, {res[name]['GBps']:.0f} GB/s algorithmic")
    gq = res["gauss"]
    out = {"metric": "electron density at the Gauss points of every cell (algorithmic HBM GB/s)",
           "value": gq["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": steps, "warmup": max(1, args.warmup),
           "ms_per_step": gq["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "density of a 1152-column FP64 block on the c1 operator (24^3 cells, p=6, "
                                  "M=2985984), 343 Gauss points per cell", "ncols": ncols, "M": op.M,
                      "E": op.E, "mu": mu, "kT": kT, "fermi_level_ms": fermi_ms},
           "roofline": {"bound": "hbm", "achieved": gq["GBps"], "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": gq["frac_hbm_peak"],
                        "traffic": profiled_traffic("density_c1_1152.md", "kernels_density.hip"),
                        "traffic_unit": "HBM bytes per Gauss-point launch"},
           "kernels": res}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = density_oracle_sample(s, X, w, op.E)
    print(json.dumps(out), flush=True)


def run_rrgep(args):
    """Spectrum-splitting Rayleigh-Ritz (Algorithm 2) in FP64 and in the
    paper's mixed precision.  Time: the c1 operator with a c2-sized filtered
    block (M = 2,985,984, N = 1152 FP64 columns, N_fr = 128 fractionally
    occupied states, about 11 % of N), beside the orthonormalise-then-project
    route (CholGS + Rayleigh-Ritz with all N Ritz vectors and residuals) the
    solver uses.  Accuracy: a c4 problem solved to max r <= 1e-6, filtered
    once more (m = 30), then the split step in both precisions: top-N_fr
    Ritz values and the spectrum-split density against FP64."""
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    steps = max(1, args.steps)

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        fn()
        e1.record(ctx.stream)
        e1.synchronize()
        return e0.elapsed_time(e1)

    # ---- accuracy on a converged c4 problem
    s4 = workloads.config("c4", 1800)
    op4 = lib.Operator(ctx, s4)
    N4, nb4, nfr4 = 128, 32, 16
    X4 = torch.from_numpy(workloads.start_block(op4.M, N4 + nb4, seed=7)).cuda()
    th4, r4, st4 = op4.solve(X4, N4, m=30, block=128, n_buf=nb4, tol=1e-6, max_passes=100)
    b4, _ = op4.bounds(20, seed=1)
    op4.filter(X4, 30, float(th4[-1]), b4, float(th4[0]))
    outs = {}
    for mode in (False, True):
        Xm = X4[:, :N4].clone()
        Pm = torch.empty(op4.M, nfr4, dtype=torch.float64, device="cuda")
        th = op4.rayleigh_ritz_split(Xm, nfr4, Pm, mixed=mode)
        mu, f = lib.fermi_level(th, 2.0 * (N4 - nfr4) + 8.0, 500.0 * 3.166811563e-6)
        f[:N4 - nfr4] = 1.0
        rho = torch.zeros(op4.M, dtype=torch.float64, device="cuda")
        op4.density(Xm, np.full(N4, 2.0), rho)
        op4.density(Pm, 2.0 * (f[N4 - nfr4:] - 1.0), rho, accumulate=True)
        outs[mode] = (th, rho.cpu().numpy())
    th64, rho64 = outs[False]
    thmx, rhomx = outs[True]
    acc = {"passes_to_converge": int(st4["passes"]), "N": N4, "nfr": nfr4,
           "max_dtheta_top_nfr_Ha": float(np.max(np.abs(thmx[N4 - nfr4:] - th64[N4 - nfr4:]))),
           "max_dtheta_all_Ha": float(np.max(np.abs(thmx - th64))),
           "density_rel_err": float(np.max(np.abs(rhomx - rho64)) / np.max(np.abs(rho64))),
           "final_max_resid": float(np.max(r4[:N4]))}
    log(f"# accuracy (c4): top-N_fr dtheta {acc['max_dtheta_top_nfr_Ha']:.2e} Ha, all {acc['max_dtheta_all_Ha']:.2e},"
        f" density {acc['density_rel_err']:.2e}")
    del X4, op4
    # ---- time at the c2 block size
    s1 = workloads.config("c1")
    op = lib.Operator(ctx, s1)
    N, nfr = 1152, 128
    g = torch.Generator(device="cuda").manual_seed(71)
    X0 = torch.randn(op.M, N, dtype=torch.float64, device="cuda", generator=g)
    X = torch.empty_like(X0)
    P = torch.empty(op.M, nfr, dtype=torch.float64, device="cuda")
    res = {}
    for name, fn in (("split_fp64", lambda: op.rayleigh_ritz_split(X, nfr, P, mixed=False)),
                     ("split_mixed", lambda: op.rayleigh_ritz_split(X, nfr, P, mixed=True)),
                     ("cholgs_rr_fp64", lambda: (op.orthonormalize(X), op.rayleigh_ritz(X)))):
        X.copy_(X0)
        fn()                                  # warm-up (workspace growth)
        ms = []
        for _ in range(steps):
            X.copy_(X0)
            ms.append(timed(fn))
        res[name] = {"ms": float(np.mean(ms))}
        log(f"# {name}: {res[name]['ms']:.1f} ms")
    out = {"metric": "spectrum-splitting Rayleigh-Ritz step, mixed precision vs FP64 (c2 block size)",
           "value": res["split_fp64"]["ms"] / res["split_mixed"]["ms"], "unit": "x speed-up",
           "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": res["split_mixed"]["ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64 / f32 blocks", "data": "synthetic",
           "config": {"workload": "rrgep: c1 operator (24^3 cells, p=6, M=2985984) with a 1152-column FP64 "
                                  "block, N_fr=128; accuracy on a converged c4 problem (N=128, N_fr=16)",
                      "N": N, "nfr": nfr, "M": op.M},
           "modes": res, "accuracy": acc}
    print(json.dumps(out), flush=True)


def run_scf_k(args):
    """The SCF loop of run_scf with k-point sampling: the same c4 system at
    the 2 x 2 x 2 Monkhorst-Pack k-points (offset grid, equal weights),
    eight complex Bloch operators through chfsi_scf_kpoints; the Gamma-point
    loop beside it.  Reports the steps and the time per step."""
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    s = workloads.config("c4", 1800)
    g = 2.0 * np.pi / s.L
    ks = [(g * (i - 0.5) / 2, g * (j - 0.5) / 2, g * (l - 0.5) / 2) for i in range(2) for j in range(2)
          for l in range(2)]
    ops = [lib.Operator(ctx, s.with_k(k)) for k in ks]
    N, nb, ne = 128, 32, 200.0
    kT = 500.0 * 3.166811563e-6
    Xs = [torch.from_numpy(workloads.start_block(o.M, N + nb, seed=11 + q, complex_=True)).cuda()
          for q, o in enumerate(ops)]
    tabs = ops[0].tables()
    mvol = float(np.sum(1.0 / tabs["dscale"] ** 2))
    rho = torch.full((ops[0].M,), ne / mvol, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.scf_kpoints(ops, Xs, rho, nwanted=N, n_buf=nb, n_electrons=ne, kT=kT, m=30, block=128, beta=0.3,
                          depth=4, tol=1e-6, maxit=80, rr_mode=2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = out["iters"]
    log(f"# scf_k: {len(ops)} k-points, {steps} steps, {dt:.2f} s, converged {out['converged']}")
    # the grid is closed under k -> -k (H(-k) = conj H(k), same density): one
    # k-point of each pair with twice the weight reaches the same density
    rho_full = rho.clone()
    half = [q for q, k in enumerate(ks) if k[0] < 0]
    Xh = [torch.from_numpy(workloads.start_block(ops[q].M, N + nb, seed=11 + q, complex_=True)).cuda()
          for q in half]
    rho.fill_(ne / mvol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outh = ctx.scf_kpoints([ops[q] for q in half], Xh, rho, weights=[2.0] * len(half), nwanted=N, n_buf=nb,
                           n_electrons=ne, kT=kT, m=30, block=128, beta=0.3, depth=4, tol=1e-6, maxit=80, rr_mode=2)
    torch.cuda.synchronize()
    dth = time.perf_counter() - t0
    drho = float(torch.max(torch.abs(rho - rho_full)) / torch.max(torch.abs(rho_full)))
    log(f"# scf_k, {len(half)} k-points of the pairs: {outh['iters']} steps, {dth:.2f} s, density {drho:.2e} apart")
    res = {"metric": "SCF step time with 2x2x2 k-point sampling, c4 system", "value": dt / max(1, steps) * 1e3,
           "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": dt / max(1, steps) * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "c128", "data": "synthetic",
           "config": {"workload": "scf_k: c4 held-out system (12^3 cells, p=5, M=216000, 16 atoms with "
                                  "projectors) at the 2x2x2 Monkhorst-Pack k-points (8 complex Bloch operators, "
                                  "equal weights), N=128+32, N_e=200, kT=500 K, m=30, Anderson beta 0.3 depth 4, "
                                  "tol 1e-6, spectrum-split mixed-precision Rayleigh-Ritz",
                      "M": ops[0].M, "kpoints": len(ops)},
           "converged": out["converged"], "scf_steps": steps, "total_s": dt, "mu": out["mu"],
           "residuals": [float(r) for r in out["residuals"]],
           "time_reversal_half": {"kpoints": len(half), "scf_steps": outh["iters"], "total_s": dth,
                                  "mu": outh["mu"], "converged": outh["converged"],
                                  "density_rel_diff_vs_full_grid": drho}}
    print(json.dumps(res), flush=True)


def run_scf(args):
    """Self-consistent field loop on the first held-out c4 system (12^3
    cells, p = 5, M = 216,000, 16 atoms with projectors): N = 128 states +
    32 buffer, N_e = 200, Fermi-Dirac smearing at 500 K, Anderson mixing
    (beta 0.3, depth 4), one ChFSI pass (m = 30) per step, to an M-norm
    density residual of 1e-6.  Reports the steps and the time per step."""
    import numpy as np
    import torch

    import paper_2203_07820_amd as lib
    import workloads

    torch.cuda.set_device(0)
    ctx = lib.Context(0)
    s = workloads.config("c4", 1800)
    op = lib.Operator(ctx, s)
    N, nb, ne = 128, 32, 200.0
    kT = 500.0 * 3.166811563e-6
    X = torch.from_numpy(workloads.start_block(op.M, N + nb, seed=11)).cuda()
    ones = torch.ones(op.M, dtype=torch.float64, device="cuda")
    tabs = op.tables()
    mvol = float(np.sum(1.0 / tabs["dscale"] ** 2))
    rho = ones * (ne / mvol)
    vh = torch.empty_like(rho)
    cg_it, cg_rr = op.hartree(rho, vh)
    torch.cuda.synchronize()
    X0, rho0 = X.clone(), rho.clone()
    # the full Rayleigh-Ritz route first, for comparison
    t0 = time.perf_counter()
    out0 = op.scf(X, rho, nwanted=N, n_buf=nb, n_electrons=ne, kT=kT, m=30, block=128, beta=0.3, depth=4,
                  tol=1e-6, maxit=80, rr_mode=0)
    torch.cuda.synchronize()
    dt0 = time.perf_counter() - t0
    rho_full = rho.clone()
    X.copy_(X0)
    rho.copy_(rho0)
    # the paper's route: spectrum splitting with the mixed-precision blocks
    t0 = time.perf_counter()
    out = op.scf(X, rho, nwanted=N, n_buf=nb, n_electrons=ne, kT=kT, m=30, block=128, beta=0.3, depth=4,
                 tol=1e-6, maxit=80, rr_mode=2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    drho = float(torch.max(torch.abs(rho - rho_full)) / torch.max(torch.abs(rho_full)))
    t1 = time.perf_counter()
    cg_it2, _ = op.hartree(rho, vh)
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t1
    steps = out["iters"]
    log(f"# scf: {steps} steps, {dt:.2f} s, converged {out['converged']}, residuals {out['residuals'][:3]} ..."
        f" {out['residuals'][-2:]}")
    res = {"metric": "SCF step time, c4 system (Hartree + LDA + one ChFSI pass with spectrum-split mixed "
                     "Rayleigh-Ritz + split density + Anderson)",
           "value": dt / max(1, steps) * 1e3, "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": 0,
           "ms_per_step": dt / max(1, steps) * 1e3, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "scf: c4 held-out system (12^3 cells, p=5, M=216000, 16 atoms with projectors), "
                                  "N=128+32, N_e=200, kT=500 K, m=30, Anderson beta 0.3 depth 4, tol 1e-6, "
                                  "spectrum-split mixed-precision Rayleigh-Ritz",
                      "M": op.M},
           "converged": out["converged"], "scf_steps": steps, "total_s": dt, "mu": out["mu"],
           "residuals": [float(r) for r in out["residuals"]],
           "hartree": {"cg_iterations": cg_it2, "seconds": t_h},
           "full_rr": {"ms_per_step": dt0 / max(1, out0["iters"]) * 1e3, "scf_steps": out0["iters"],
                       "total_s": dt0, "converged": out0["converged"], "mu": out0["mu"]},
           "density_rel_diff_split_vs_full": drho}
    print(json.dumps(res), flush=True)


def density_oracle_sample(s, X, w, E):
    """The oracle's Gauss-point density on a sample of cells, timed."""
    import numpy as np
    import torch

    from oracle import density as dens
    from oracle import fe
    cores = len(os.sched_getaffinity(0))
    Mdiag = fe.lumped_mass(s.ncell, s.p, s.L)
    cells = np.arange(0, E, max(1, E // 200))[:200]
    nodes = fe.cell_nodes(s.ncell, s.p)[cells]
    uniq, inv = np.unique(nodes.ravel(), return_inverse=True)
    Xu = X[torch.from_numpy(uniq).cuda()].cpu().numpy()
    Ph = ((1.0 / np.sqrt(Mdiag[uniq]))[:, None] * Xu)[inv.reshape(nodes.shape)]
    t0 = time.perf_counter()
    for i in range(cells.size):
        dens.density_gauss_cell(s.p, Ph[i], w)
    dt = time.perf_counter() - t0
    per_cell = (X.shape[0] // E) * X.shape[1] * 8     # unique nodes per cell x columns x 8 B
    return {"value": cells.size * per_cell / dt / 1e9, "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle.density.density_gauss_cell on {cells.size} of {E} cells with all "
                      f"{X.shape[1]} columns ({dt:.1f} s)", "seconds": dt}


def c2_oracle_sample(sys_, Xref, theta, ref_tol, nwanted=1024):
    """The oracle's cell-wise H~ applied to every wanted reference Ritz vector
    (full size, 64 columns at a time), timed: the residuals of all
    reference pairs in the oracle's own, independently built operator
    certify the FP64 reference that the mixed runs are measured against."""
    import numpy as np

    from oracle import fe
    cores = len(os.sched_getaffinity(0))
    op = fe.build_operator(sys_)
    res = np.empty(nwanted)
    t0 = time.perf_counter()
    for c0 in range(0, nwanted, 64):
        c1 = min(nwanted, c0 + 64)
        V = Xref[:, c0:c1].cpu().numpy()
        HV = fe.apply_cellwise(op, V, chunk=256)
        res[c0:c1] = np.linalg.norm(HV - V * theta[c0:c1][None, :], axis=0)
        log(f"# c2 oracle certification: {c1}/{nwanted} reference pairs, max residual so far "
            f"{res[:c1].max():.2e} ({time.perf_counter() - t0:.0f}s)")
    dt = time.perf_counter() - t0
    fl = 2.0 * op.cells.shape[1] ** 2 * op.E * nwanted
    q = np.quantile(res, [0.5, 0.9, 0.99, 1.0])
    return {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            "sample": f"oracle cell-wise H~X on all {nwanted} wanted reference Ritz vectors of the full c2 "
                      f"operator, 64 at a time ({dt:.0f} s); their residuals in the oracle's operator certify "
                      "the FP64 reference",
            "oracle_resid_max": float(res.max()), "oracle_resid_quantiles_50_90_99_100": [float(x) for x in q],
            "pairs_above_1e-9": int(np.sum(res > 1e-9)), "reference_tol": ref_tol}


if __name__ == "__main__":
    main()
