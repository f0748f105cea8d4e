"""Picard and Newton iterations for a semilinear problem (paper Sec. 2, the
remark after eq. (sum): for a nonlinear operator each step of a Picard or
Newton iteration solves one linear least-squares problem of the same form).

Test infrastructure only: used by tests/, the package's smoke check and the
benchmark's CPU baseline, never by the GPU library.

Problem: A[u] + g(u) = f in the box, u = g_D on the boundary, with A the linear
operator of the problem (its coefficients a, beta, c0) and the polynomial
reaction g(u) = sum_p gamma_p u^p.  Each step linearises g about the current
iterate u_k (values at the interior collocation points):

  Newton:  g(u) ~ g(u_k) + g'(u_k) (u - u_k)
           -> reaction c0 + g'(u_k),  interior right-hand side f - g(u_k) + g'(u_k) u_k
  Picard:  g(u) = u q(u) with q(u) = sum_{p>=1} gamma_p u^{p-1}, frozen at u_k
           -> reaction c0 + q(u_k),   interior right-hand side f - gamma_0

and solves the linear collocation least-squares problem with these data (the
Gauss-Newton step of the nonlinear least-squares problem for Newton).  The PCA
basis is that of the first step: it is built from the value matrix, which does
not depend on the operator.  Boundary rows are unchanged.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import assemble as asm
from . import lsq


def g_value(u, gamma):
    """g(u) = sum_p gamma_p u^p by Horner's rule."""
    out = np.zeros_like(u)
    for c in gamma[::-1]:
        out = out * u + c
    return out


def g_prime(u, gamma):
    """g'(u) = sum_{p>=1} p gamma_p u^{p-1}."""
    d = [p * gamma[p] for p in range(1, len(gamma))]
    return g_value(u, d) if d else np.zeros_like(u)


def linearize(u, c0, f, gamma, mode):
    """Reaction coefficient and interior right-hand side of one step."""
    gamma = list(gamma)
    if mode == "newton":
        gp = g_prime(u, gamma)
        return c0 + gp, f - g_value(u, gamma) + gp * u
    if mode == "picard":
        q = g_value(u, gamma[1:]) if len(gamma) > 1 else np.zeros_like(u)
        return c0 + q, f - gamma[0]
    raise ValueError(mode)


def step_problem(prob, c, f_int):
    """The linear problem of one step: reaction c, interior rows f_int."""
    F = np.array(prob.F, dtype=float, copy=True)
    F[:prob.N_I] = f_int.reshape(prob.N_I, -1)
    return dataclasses.replace(prob, c=np.asarray(c, dtype=float), F=F)


def nonlinear_residual(prob, sysm0, W, gamma):
    """r(W): interior rows A[u_W] + g(u_W) - f, boundary rows lambda_B (u_W - g_D),
    with the operator rows of the linear part (the problem's own c)."""
    H0 = sysm0.dense()
    Pm = asm.probe_matrix(prob, sysm0, prob.X_int)
    u = Pm @ W
    r = H0 @ W - sysm0.Fs[:, 0]
    r[:prob.N_I] += g_value(u, list(gamma))
    return r


def iterate(prob, gamma, mode="newton", steps=8, pca_mode="rel_eig", pca_tol=1e-8,
            V_force=None, p_force=None, stop=0.0):
    """Run `steps` Picard or Newton steps from u_0 = 0 (first right-hand side
    column only).  Returns the coefficient iterates W_1.., the interior values
    u_1.., the relative increments ||u_{k+1} - u_k|| / ||u_{k+1}|| at the
    interior points and the systems of the first and the last step."""
    f = np.asarray(prob.F[:prob.N_I, 0], dtype=float)
    c0 = np.asarray(prob.c, dtype=float)
    u = np.zeros(prob.N_I)
    V, p = V_force, p_force
    Ws, us, incs = [], [], []
    sys_first = sysm = None
    for _ in range(steps):
        c, fl = linearize(u, c0, f, gamma, mode)
        pk = step_problem(prob, c, fl[:, None])
        sysm = asm.assemble(pk, pca_mode, pca_tol, V_force=V, p_force=p)
        if V is None:
            V, p = sysm.V, sysm.p
        if sys_first is None:
            sys_first = sysm
        W = lsq.QRSolver(sysm.dense()).solve(sysm.Fs)[:, 0]
        u_new = asm.probe_matrix(pk, sysm, prob.X_int) @ W
        incs.append(float(np.linalg.norm(u_new - u) / max(np.linalg.norm(u_new), 1e-300)))
        u = u_new
        Ws.append(W)
        us.append(u)
        if incs[-1] <= stop:
            break
    return dict(W=Ws, u=us, inc=np.array(incs), V=V, p=p, sys_first=sys_first, sys_last=sysm)
