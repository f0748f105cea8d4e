"""Krylov solvers for the normal equations H^T H W = H^T F (paper Sec. 2-3).

* pcg  : preconditioned conjugate gradients (symmetric M, e.g. AS), one
         independent recurrence per right-hand side.
* gmres: left-preconditioned restarted GMRES (any M, e.g. RAS/SAS), modified
         Gram-Schmidt Arnoldi and Givens rotations.

Stopping rules (reading): the paper stops on the left-preconditioned residual
||M^{-1}(H^T H W - H^T F)|| / ||M^{-1} H^T F|| (Sec. 5, Example 1).  Here PCG
stops on the true normal residual ||H^T(F - H W)|| / ||H^T F|| recomputed from
scratch, checked when the recurrence residual passes the tolerance; GMRES stops
when its residual estimate passes and the recomputed preconditioned residual
confirms it.  Both return per-RHS iteration counts.
"""
from __future__ import annotations

import numpy as np


def pcg(A, M, B, X0=None, tol=1e-10, maxiter=1000, true_res=None):
    """A, M: callables on (P, k) arrays.  true_res(X) -> (k,) relative residuals."""
    B = B.reshape(B.shape[0], -1)
    P, k = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=float).reshape(P, k)
    R = B - A(X)
    Z = M(R)
    Pd = Z.copy()
    rho = np.einsum("ij,ij->j", R, Z)
    bnorm = np.linalg.norm(B, axis=0)
    bnorm[bnorm == 0] = 1.0
    active = np.ones(k, dtype=bool)
    iters = np.zeros(k, dtype=int)
    hist = []
    if true_res is not None:
        tr = true_res(X)
        active &= ~(tr <= tol)
    for it in range(maxiter):
        if not active.any():
            break
        S = A(Pd)
        pS = np.einsum("ij,ij->j", Pd, S)
        alpha = np.where(active, rho / np.where(pS == 0, 1.0, pS), 0.0)
        X += alpha[None, :] * Pd
        R -= alpha[None, :] * S
        iters += active
        rn = np.linalg.norm(R, axis=0) / bnorm
        hist.append(rn.copy())
        done = rn <= tol
        if true_res is not None and np.any(done & active):
            tr = true_res(X)
            done = tr <= tol
        active &= ~done
        Z = M(R)
        rho_new = np.einsum("ij,ij->j", R, Z)
        beta = np.where(active, rho_new / np.where(rho == 0, 1.0, rho), 0.0)
        Pd = Z + beta[None, :] * Pd
        rho = rho_new
    return X, iters, np.array(hist)


def gmres(A, M, b, x0=None, restart=50, tol=1e-5, maxiter=1000, side="left"):
    """GMRES(restart) for one right-hand side b (P,).

    side="left"  : Arnoldi on M A, residuals M (b - A x) (the paper's form);
    side="right" : Arnoldi on A M, x = x0 + M V y, residuals b - A x.
    """
    b = b.ravel()
    P = b.size
    A0, M0 = A, M
    A = lambda v: np.asarray(A0(v.reshape(P, 1))).ravel()
    M = lambda v: np.asarray(M0(v.reshape(P, 1))).ravel()
    x = np.zeros(P) if x0 is None else np.array(x0, dtype=float).ravel()
    right = (side == "right")
    pre = (lambda v: v) if right else M   # applied to residuals
    mb = np.linalg.norm(pre(b))
    if mb == 0:
        return x, 0, []
    it = 0
    hist = []
    while it < maxiter:
        r = pre(b - A(x))
        beta = np.linalg.norm(r)
        if beta / mb <= tol:
            break
        m = min(restart, maxiter - it)
        V = np.zeros((m + 1, P))
        Hh = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(m):
            w = A(M(V[j])) if right else M(A(V[j]))
            for i in range(j + 1):
                Hh[i, j] = V[i] @ w
                w = w - Hh[i, j] * V[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            if Hh[j + 1, j] > 0:
                V[j + 1] = w / Hh[j + 1, j]
            for i in range(j):
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j] = t
            den = np.hypot(Hh[j, j], Hh[j + 1, j])
            cs[j] = Hh[j, j] / den
            sn[j] = Hh[j + 1, j] / den
            Hh[j, j] = den
            Hh[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_used = j + 1
            hist.append(abs(g[j + 1]) / mb)
            if abs(g[j + 1]) / mb <= tol:
                break
        y = np.zeros(j_used)
        for i in range(j_used - 1, -1, -1):
            y[i] = (g[i] - Hh[i, i + 1:j_used] @ y[i + 1:]) / Hh[i, i]
        x = x + (M(V[:j_used].T @ y) if right else V[:j_used].T @ y)
        if hist and hist[-1] <= tol:
            r = pre(b - A(x))
            if np.linalg.norm(r) / mb <= tol:
                break
    return x, it, hist
