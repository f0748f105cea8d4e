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
           "k_HTy_part", "k_local_apply"]


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
    ap.add_argument("--quick", action="store_true", help="skip the side measurements")
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
        # the factor Y_i in FP32) read once; gathered r, the column-sum slots
        # (written and read) and the local results
        "k_local_apply": ("hbm", f_bytes * float(np.sum(q * (q + 1) / 2.0))
                          + 8.0 * (2.0 * float(np.sum(q)) + 2.0 * slots) * k, "byte", HBM_PEAK_GBS),
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


def cpu_baseline(prob, tol, stencil):
    """The FP64 oracle on the same workload, on the host cores: assembly with PCA,
    then block-sparse AS-PCG to the same tolerance."""
    from oracle import assemble as oasm
    from oracle import solve as osolve
    t0 = time.perf_counter()
    sysm = oasm.assemble(prob, "rel_eig", prob.meta["pca_tol"])
    t1 = time.perf_counter()
    it = osolve.iterative(prob, sysm, stencil, "as", "cg", tol=tol, maxiter=5000)
    t2 = time.perf_counter()
    return dict(total_s=t2 - t0, assemble_s=t1 - t0, solve_s=t2 - t1, iters=int(it["iters"].max()))


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
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
    dom = max(ktimes, key=lambda n: ktimes[n][0])
    tot_ms, launches = ktimes[dom]
    avg_s = tot_ms / max(launches, 1) / 1e3
    bound, work, wunit, peak = model[dom]
    achieved = work / avg_s / (1e9 if wunit == "byte" else 1e12)
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak,
                "unit": "GB/s" if wunit == "byte" else "TFLOP/s", "frac": achieved / peak,
                "traffic": None, "avg_launch_us": avg_s * 1e6, "launches": launches,
                "algorithmic_work_per_launch": work}
    kernel_table = {}
    for name, (ms, cnt) in ktimes.items():
        if cnt == 0:
            continue
        b_, w_, u_, pk_ = model[name]
        av = ms / cnt / 1e3
        ach = w_ / av / (1e9 if u_ == "byte" else 1e12)
        kernel_table[name] = {"ms_per_step": ms / args.steps, "avg_us": av * 1e6, "bound": b_,
                              "achieved": ach, "frac": ach / pk_}

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
    if not args.no_cpu_baseline:
        cb = cpu_baseline(prob, args.tol, args.stencil)
        out["cpu_baseline"] = {"value": k / cb["total_s"], "unit": "solves/s",
                               "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"one full solve of the same workload (assembly with PCA + "
                                         f"block-sparse AS-PCG to {args.tol:g}, {cb['iters']} iterations)",
                               "seconds": cb["total_s"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
