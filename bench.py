"""Benchmark of the RaNN overlapping-Schwarz hot path on one MI355X.

One step = one pass of the whole path on the 2D Poisson workload (8x8
subdomains, width-300 tanh RaNN per subdomain, 30x30 collocation points per
subdomain plus 64 per boundary edge, relative PCA threshold 1e-8, AS-CG with
the full stencil) with inputs resident in HBM:

  assemble (binning, window partition of unity, operator coefficients)
  -> PCA (value Gram, FP64 eigendecomposition, truncation)
  -> operator rows H, local Gram blocks, local inverses
  -> preconditioned CG to a relative normal residual of 1e-6
  -> probe evaluation u_h and misfit gradient (transpose evaluation)
  -> adjoint solve and dF = H z

The JSON line reports solves/s of that step (value), time-to-1e-6 end-to-end
and solve-only, the mixed-precision path on the same problem, fwd+bwd ms, the
roofline position of the dominant kernel, and the FP64 oracle timed on the
host cores on the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # dense FP64 (matrix cores and vector ALUs)
FP32_PEAK_TFLOPS = 157.3
KERNELS = ["k_eig", "k_factor", "k_pca_gram", "k_feat_rows", "k_local_gram", "k_normal", "k_Hx",
           "k_HTy_part", "k_tile_apply", "k_slot_reduce"]
# timers that cover several different kernels (not candidates for the roofline line)
GROUPS = {"k_eig", "k_factor", "k_Hx", "k_pca_gram"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter measurement
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when there is none or the kernel's source changed since it was taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh).get(kernel)
        with open(os.path.join(ROOT, rec["source"]), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError, KeyError, TypeError, AttributeError):
        return None
    if sha != rec.get("sha256"):
        return None
    return rec["fetch_bytes_per_launch"] * rec["fetch_scale"] + rec["write_bytes_per_launch"] * rec["write_scale"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--stencil", default="full")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 32-RHS mixed/FP64 comparison")
    ap.add_argument("--no-variants", action="store_true", help="skip the Krylov method x preconditioner grid")
    ap.add_argument("--no-nonlinear", action="store_true", help="skip the Newton iteration on the semilinear problem")
    ap.add_argument("--quick", action="store_true", help="skip the side measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB (counter calibration) and exit")
    return ap.parse_args()


class Inputs:
    """Problem arrays uploaded once; the step only passes device pointers."""

    def __init__(self, prob, torch, dev):
        from paper_2412_19207_amd import binding
        self.prob = prob
        self.F = torch.as_tensor(prob.F, device=dev)
        self.Xq = torch.as_tensor(prob.probes, device=dev)
        self.u_obs = torch.as_tensor(prob.u_probe[:, None], device=dev).repeat(1, prob.F.shape[1])
        self.binding = binding


def work_model(s, prob, k):
    """Algorithmic work per launch of each timed kernel (bytes the method must
    move, or flops it must do), from the handle's sizes."""
    row_off, _, p = s.layout()
    n = np.diff(row_off).astype(np.float64)
    m = np.asarray(prob.m, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    q = s.blocks().astype(np.float64)
    nnz, N, P = float(s.info.nnz), float(s.info.N), float(s.info.P)
    f_bytes = 4.0 if s.precision == "mixed" else 8.0
    ntile = np.ceil(q / 64.0)
    slots = float(np.sum(ntile * (ntile + 1) / 2.0 * 64.0))
    return {
        # nominal count of a dense symmetric eigendecomposition with vectors
        "k_eig": ("alu", float(np.sum(9.0 * m ** 3)), "flop", FP64_PEAK_TFLOPS),
        # Cholesky q^3/3 + triangular inverse q^3/3, FP64 on matrix cores
        "k_factor": ("mfma", float(np.sum(2.0 * q ** 3 / 3.0)), "flop", FP64_PEAK_TFLOPS),
        # symmetric rank-n update Psi^T Psi
        "k_pca_gram": ("mfma", float(np.sum(n * m * m)), "flop", FP64_PEAK_TFLOPS),
        "k_feat_rows": ("mfma", float(np.sum(2.0 * n * m * p)), "flop", FP64_PEAK_TFLOPS),
        # Gram blocks H_j^T H_k: counted for the diagonal blocks only (a lower bound)
        "k_local_gram": ("mfma", float(np.sum(2.0 * n * p * p)), "flop", FP64_PEAK_TFLOPS),
        # slabs of the normal matrix read once, x read, s written
        "k_normal": ("hbm", 8.0 * (float(s.info.normal_elems) + 2.0 * P * k), "byte", HBM_PEAK_GBS),
        # H read once, x read, y written
        "k_Hx": ("hbm", 8.0 * (nnz + P * k + N * k), "byte", HBM_PEAK_GBS),
        "k_HTy_part": ("hbm", 8.0 * (nnz + N * k + P * k), "byte", HBM_PEAK_GBS),
        # the stored local operators (q_i (q_i + 1) / 2 entries each: W_i in FP64,
        # the factor Y_i in FP32) read once, the gathered r, and the row/column
        # sum slots written (both kinds for W, the column sums for Y)
        "k_tile_apply": ("hbm", f_bytes * float(np.sum(q * (q + 1) / 2.0))
                         + 8.0 * (float(np.sum(q)) + (1.0 if s.precision == "mixed" else 2.0) * slots) * k,
                         "byte", HBM_PEAK_GBS),
        # the slots read, the local results written
        "k_slot_reduce": ("hbm", 8.0 * ((1.0 if s.precision == "mixed" else 2.0) * slots + float(np.sum(q))) * k,
                          "byte", HBM_PEAK_GBS),
    }


def run_step(inp, precision, stencil, tol, torch, timings=None, want_model=False):
    """One pass of the path; returns (solve info, adjoint info, work model or None)."""
    b = inp.binding
    sync = torch.cuda.synchronize
    t0 = time.perf_counter()
    s = b.Solver(inp.prob, precision=precision, stencil=stencil, precond="as")
    s.precision = precision
    if timings is not None:
        sync()
        timings["assemble_ms"] = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
    s.pca(inp.prob.meta["pca_tol"], "rel_eig")
    if timings is not None:
        sync()
        timings["pca_factor_ms"] = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
    W, info = s.solve(inp.F, tol=tol, maxiter=5000, check_every=10, stats=True)
    if timings is not None:
        sync()
        timings["solve_ms"] = (time.perf_counter() - t0) * 1e3
        t0 = time.perf_counter()
    U = s.eval(inp.Xq, W)
    dU = 2.0 * (U - inp.u_obs)
    dW = s.eval_T(inp.Xq, dU)
    dF, ainfo = s.solve_backward(dW, tol=tol, maxiter=5000, check_every=10)
    if timings is not None:
        sync()
        timings["eval_adjoint_ms"] = (time.perf_counter() - t0) * 1e3
    model = work_model(s, inp.prob, inp.prob.F.shape[1]) if want_model else None
    s.close()
    return info, ainfo, model


def solve_only(inp, precision, stencil, tol, torch, reps=3):
    """Time-to-tol of the solve with the preconditioner already built."""
    b = inp.binding
    s = b.Solver(inp.prob, precision=precision, stencil=stencil, precond="as")
    s.pca(inp.prob.meta["pca_tol"], "rel_eig")
    W, info = s.solve(inp.F, tol=tol, maxiter=5000, check_every=10)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        W, info = s.solve(inp.F, tol=tol, maxiter=5000, check_every=10)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    stats = dict(info=info, ms=float(np.median(times)), P=int(s.info.P), nnz=int(s.info.nnz),
                 factor_elems=int(s.info.factor_elems), N=int(s.info.N))
    s.close()
    return stats


def krylov_variants(inp, stencil, tol, torch):
    """The Krylov method x preconditioner grid of Table 1b on the benchmark
    workload (FP64, preconditioner built once per kind): iterations and the
    solve time to the tolerance (second of two solves), at most 1000
    iterations (status 1: not converged)."""
    b = inp.binding
    grid = {"as": ["cg", "cgs", "bicg", "gmres"], "sas": ["cgs", "bicg", "gmres"], "ras": ["cgs", "gmres"]}
    out = {}
    for kind, methods in grid.items():
        s = b.Solver(inp.prob, precision="fp64", stencil=stencil, precond=kind)
        s.pca(inp.prob.meta["pca_tol"], "rel_eig")
        for m in methods:
            s.solve(inp.F, tol=tol, maxiter=1000, method=m, restart=50, check_every=10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            W, info = s.solve(inp.F, tol=tol, maxiter=1000, method=m, restart=50, check_every=10)
            torch.cuda.synchronize()
            out[f"{m}/{kind}"] = {"iterations": int(info["iterations"]), "solve_ms": (time.perf_counter() - t0) * 1e3,
                                  "status": int(info["status"]),
                                  "max_rel_residual": float(info["max_rel_residual"])}
        s.close()
    return out


def nonlinear_newton(torch, wl, dev, steps=10):
    """Newton on the semilinear problem -lap u + u^3 = f with the benchmark's
    8x8, width-300 layout (FP64 AS-CG per step to 1e-10; the first step builds
    the PCA basis, later steps reuse it): time per step, increments, linear
    iterations, and the relative L2 error at the probes."""
    from paper_2412_19207_amd import nonlinear as gnl
    prob = wl.make("semilinear2d")
    gamma = prob.meta["gamma"]
    s, W, rec = gnl.solve_semilinear(prob, gamma, mode="newton", steps=steps, stop=1e-10,
                                     tol=prob.meta["tol"], device=str(dev))
    s.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s, W, rec = gnl.solve_semilinear(prob, gamma, mode="newton", steps=steps, stop=1e-10,
                                     tol=prob.meta["tol"], device=str(dev))
    torch.cuda.synchronize()
    total = (time.perf_counter() - t0) * 1e3
    U = s.eval(torch.as_tensor(prob.probes, device=dev), W)[:, 0].cpu().numpy()
    s.close()
    e = float(np.linalg.norm(U - prob.u_probe) / np.linalg.norm(prob.u_probe))
    return {"workload": prob.name, "g": "u^3", "steps": len(rec["inc"]), "total_ms": total,
            "step_ms": rec["step_ms"], "increments": rec["inc"], "linear_iterations": rec["iterations"],
            "e_L2_probes": e}


def cpu_baseline(prob, tol, stencil, min_seconds=10.0, max_reps=3):
    """The FP64 oracle on the same workload, on the host cores: assembly with PCA,
    then block-sparse AS-PCG to the same tolerance, repeated until about
    min_seconds of host work (at most max_reps solves)."""
    from oracle import assemble as oasm
    from oracle import solve as osolve
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(t.get("num_threads", 1)) for t in threadpool_info()] or [1])
    except Exception:  # threadpoolctl missing: report the interpreter's view
        threads = os.cpu_count()
    reps, t_all, iters = 0, 0.0, 0
    while reps < max_reps and (reps == 0 or t_all < min_seconds):
        t0 = time.perf_counter()
        sysm = oasm.assemble(prob, "rel_eig", prob.meta["pca_tol"])
        it = osolve.iterative(prob, sysm, stencil, "as", "cg", tol=tol, maxiter=5000)
        t_all += time.perf_counter() - t0
        iters = int(it["iters"].max())
        reps += 1
    return dict(total_s=t_all / reps, reps=reps, iters=iters, threads=threads)


def batched_comparison(torch, binding, wl, dev):
    """Many right-hand sides in one solve, mixed against FP64, on the
    multiscale workload with 32 batched right-hand sides (end-to-end time to
    the tolerance and the solve alone), and the same right-hand sides solved
    one at a time in FP64 for reference."""
    prob = wl.make("cfg3")
    meta = prob.meta
    F = torch.as_tensor(prob.F, device=dev)
    k = F.shape[1]
    out = {"workload": prob.name, "rhs": int(k), "subdomains": [int(x) for x in prob.l],
           "hidden_width": [int(prob.m.min()), int(prob.m.max())], "rows": int(prob.N),
           "tol": meta["tol"], "stencil": meta["stencil"], "precond": meta["precond"]}
    for precision in ["fp64", "mixed", "fp64", "mixed"]:  # first pair warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = binding.Solver(prob, precision=precision, stencil=meta["stencil"], precond=meta["precond"])
        s.pca(meta["pca_tol"], "rel_eig")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        W, info = s.solve(F, tol=meta["tol"], maxiter=5000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        W, info = s.solve(F, tol=meta["tol"], maxiter=5000)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        e2e = (t2 - t0) * 1e3
        out[precision] = {"time_to_tol_ms": {"end_to_end": e2e, "solve_only": (t3 - t2) * 1e3},
                          "solves_per_s": k / (e2e / 1e3), "iterations": int(info["iterations"]),
                          "max_rel_residual": float(info["max_rel_residual"])}
        s.close()
    # the same right-hand sides one at a time (FP64, preconditioner built once)
    s = binding.Solver(prob, precision="fp64", stencil=meta["stencil"], precond=meta["precond"])
    s.pca(meta["pca_tol"], "rel_eig")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q in range(k):
        s.solve(F[:, q:q + 1], tol=meta["tol"], maxiter=5000)
    torch.cuda.synchronize()
    out["fp64_one_at_a_time_solve_ms"] = (time.perf_counter() - t0) * 1e3
    s.close()
    out["mixed_over_fp64_speedup"] = {
        "end_to_end": out["fp64"]["time_to_tol_ms"]["end_to_end"] / out["mixed"]["time_to_tol_ms"]["end_to_end"],
        "solve_only": out["fp64"]["time_to_tol_ms"]["solve_only"] / out["mixed"]["time_to_tol_ms"]["solve_only"]}
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2412_19207_amd import binding
    from paper_2412_19207_amd import workloads as wl

    binding.load()
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        n = (512 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 5}))
        return
    prob = wl.make(args.workload)
    inp = Inputs(prob, torch, dev)
    k = prob.F.shape[1]

    for _ in range(args.warmup):
        run_step(inp, "fp64", args.stencil, args.tol, torch)
    torch.cuda.synchronize()
    binding.rann_dd_ktime_enable(True)
    t0 = time.perf_counter()
    last = None
    for _ in range(args.steps):
        last = run_step(inp, "fp64", args.stencil, args.tol, torch)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ktimes = {name: binding.rann_dd_ktime_query(name) for name in KERNELS}
    binding.rann_dd_ktime_enable(False)
    ms_step = elapsed / args.steps * 1e3
    info, ainfo, _ = last
    tm = {}
    _, _, model = run_step(inp, "fp64", args.stencil, args.tol, torch, timings=tm, want_model=True)
    # dominant kernel over the timed region and its roofline position
    dom = max((n for n in ktimes if n not in GROUPS), key=lambda n: ktimes[n][0])
    tot_ms, launches = ktimes[dom]
    avg_s = tot_ms / max(launches, 1) / 1e3
    bound, work, wunit, peak = model[dom]
    achieved = work / avg_s / (1e9 if wunit == "byte" else 1e12)
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak,
                "unit": "GB/s" if wunit == "byte" else "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(dom), "avg_launch_us": avg_s * 1e6, "launches": launches,
                "algorithmic_work_per_launch": work}
    kernel_table = {}
    for name, (ms, cnt) in ktimes.items():
        if cnt == 0:
            continue
        b_, w_, u_, pk_ = model[name]
        av = ms / cnt / 1e3
        ach = w_ / av / (1e9 if u_ == "byte" else 1e12)
        kernel_table[name] = {"ms_per_step": ms / args.steps, "avg_us": av * 1e6, "bound": b_,
                              "achieved": ach, "frac": ach / pk_, "launches_per_step": cnt / args.steps}
        if name in GROUPS:
            kernel_table[name]["group_of_kernels"] = True

    out = {
        "metric": "time-to-1e-6 residual & solves/s, mixed-batched vs FP64 AS-CG; fwd+bwd ms",
        "value": k / (ms_step / 1e3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob.name, "subdomains": [int(x) for x in prob.l],
                   "hidden_width": int(prob.m[0]), "rows": int(prob.N), "rhs": int(k),
                   "pca_tol": prob.meta["pca_tol"], "tol": args.tol, "stencil": args.stencil,
                   "precond": "as", "method": "cg"},
        "iterations": int(info["iterations"]),
        "adjoint_iterations": int(ainfo["iterations"]),
        "rel_residual": float(info["max_rel_residual"]),
        "roofline": roofline,
        "kernels": kernel_table,
    }
    if not args.quick:
        out["phases_ms"] = tm
        so = solve_only(inp, "fp64", args.stencil, args.tol, torch)
        out["time_to_1e-6_ms"] = {"end_to_end": tm["assemble_ms"] + tm["pca_factor_ms"] + tm["solve_ms"],
                                  "solve_only": so["ms"]}
        out["fwd_bwd_ms"] = tm["solve_ms"] + tm["eval_adjoint_ms"]
        out["sizes"] = {"P": so["P"], "N": so["N"], "nnz_H": so["nnz"], "factor_elems": so["factor_elems"]}
        if not args.no_mixed:
            tmm = {}
            mi, _, _ = run_step(inp, "mixed", args.stencil, args.tol, torch, timings=tmm)
            som = solve_only(inp, "mixed", args.stencil, args.tol, torch)
            out["mixed"] = {"time_to_1e-6_ms": {"end_to_end": tmm["assemble_ms"] + tmm["pca_factor_ms"] + tmm["solve_ms"],
                                                "solve_only": som["ms"]},
                            "iterations": int(mi["iterations"]), "phases_ms": tmm}
        if not args.no_batched:
            out["batched"] = batched_comparison(torch, binding, wl, dev)
        if not args.no_variants:
            out["krylov_variants"] = krylov_variants(inp, args.stencil, args.tol, torch)
        if not args.no_nonlinear:
            out["nonlinear_newton"] = nonlinear_newton(torch, wl, dev)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(prob, args.tol, args.stencil)
        out["cpu_baseline"] = {"value": k / cb["total_s"], "unit": "solves/s",
                               "cores": cb["threads"], "kind": "oracle",
                               "sample": f"{cb['reps']} full solve(s) of the same workload (assembly "
                                         f"with PCA + block-sparse AS-PCG to {args.tol:g}, "
                                         f"{cb['iters']} iterations), averaged",
                               "seconds": cb["total_s"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
