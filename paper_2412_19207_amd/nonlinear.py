"""Picard and Newton iterations for a semilinear problem A[u] + g(u) = f with a
polynomial reaction g(u) = sum_p gamma_p u^p (paper Sec. 2, the remark after
eq. (sum): each step of the nonlinear iteration solves one linear collocation
least-squares problem).

Each step runs on the library: the reaction and right-hand side of the step's
linear problem come from `rann_dd_linearize` (Newton or Picard) at the current
values u_k on the interior collocation points, a handle is assembled with that
reaction, its PCA basis is the first step's (the basis depends only on the
value matrix, not on the operator), the linear problem is solved by the chosen
Krylov method from the previous step's coefficients, and u_{k+1} at the
interior points comes from `rann_dd_eval`.
This module only sequences those calls and holds the device buffers.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding


def solve_semilinear(prob, gamma, mode="newton", steps=8, stop=0.0, tol=1e-10, maxiter=5000,
                     precision="fp64", stencil="full", precond="as", method="cg", pca_tol=None,
                     pca_mode=None, p_force=None, V_force=None, device="cuda:0", keep_iterates=False):
    """Run up to `steps` steps from u_0 = 0 on the first right-hand side column;
    stop early when the relative increment of u at the interior points drops to
    `stop`.  Returns the last handle (open; the caller closes it), its W, and a
    record of the increments, linear-solve iterations and per-step times."""
    import torch
    dev = torch.device(device)
    nI = int(prob.N_I)
    f = torch.as_tensor(np.ascontiguousarray(prob.F[:nI, 0], dtype=np.float64), device=dev)
    g_bnd = torch.as_tensor(np.ascontiguousarray(prob.F[nI:, :1], dtype=np.float64), device=dev)
    c0 = torch.as_tensor(np.ascontiguousarray(prob.c, dtype=np.float64), device=dev)
    Xi = torch.as_tensor(np.ascontiguousarray(prob.X_int, dtype=np.float64), device=dev)
    u = torch.zeros(nI, dtype=torch.float64, device=dev)
    c = torch.empty_like(u)
    fl = torch.empty_like(u)
    pca_tol = prob.meta["pca_tol"] if pca_tol is None else pca_tol
    pca_mode = prob.meta.get("pca_mode", "rel_eig") if pca_mode is None else pca_mode
    rec = dict(inc=[], iterations=[], step_ms=[], W=[])
    s_prev = None
    s = W = None
    for k in range(steps):
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        if k == 0:  # about u_0 = 0, on the default stream (no handle yet)
            binding.rann_dd_linearize(None, u.data_ptr(), c0.data_ptr(), f.data_ptr(), nI, gamma,
                                      binding.LINEARIZE[mode], c.data_ptr(), fl.data_ptr())
        s = binding.Solver(prob, precision=precision, stencil=stencil, precond=precond, device=device, c=c)
        if V_force is None:
            p_force = s.pca(pca_tol, pca_mode)
            V_force = s.arrays()[1].clone()
        else:
            s.pca(pca_tol, pca_mode, p_force=p_force, V_force=V_force)
        F = torch.cat([fl[:, None], g_bnd], 0)
        # warm start from the previous step's coefficients (same basis)
        W, info = s.solve(F, tol=tol, maxiter=maxiter, method=method, W0=W)
        u_new = s.eval(Xi, W)[:, 0].contiguous()
        # the next step's data, and the increment of this one
        inc = binding.rann_dd_linearize(s.handle, u_new.data_ptr(), c0.data_ptr(), f.data_ptr(), nI, gamma,
                                        binding.LINEARIZE[mode], c.data_ptr(), fl.data_ptr(), u.data_ptr())
        torch.cuda.synchronize(dev)
        rec["step_ms"].append((time.perf_counter() - t0) * 1e3)
        rec["inc"].append(inc)
        rec["iterations"].append(int(info["iterations"]))
        rec["status"] = int(info["status"])
        if keep_iterates:
            rec["W"].append(W.clone())
        u = u_new
        if s_prev is not None:
            s_prev.close()
        s_prev = s
        if inc <= stop:
            break
    rec["p"] = p_force
    rec["V"] = V_force
    return s, W, rec
