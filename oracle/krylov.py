"""Krylov solvers for the normal equations H^T H W = H^T F (paper Sec. 2-3).

* pcg  : preconditioned conjugate gradients (symmetric M, e.g. AS), one
         independent recurrence per right-hand side.
* gmres: left-preconditioned restarted GMRES (any M, e.g. RAS/SAS), modified
         Gram-Schmidt Arnoldi and Givens rotations.
* cgs  : conjugate gradients squared (Sonneveld), transpose-free, with the
         preconditioner applied to the search directions (any M).
* bicg : biconjugate gradients (Fletcher) with the shadow system driven by
         A^T and M^{-T} (any M).
The paper compares CG, CGS, BiCG and GMRES with the AS, SAS and RAS
preconditioners (Sec. 5, Example 1, Table 1b).  CGS and BiCG stop on the
recurrence residual b - A x (the normal residual in exact arithmetic),
confirmed by the recomputed one.

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


def cgs(A, M, b, x0=None, tol=1e-10, maxiter=1000, true_res=None, shadow="r"):
    """Conjugate gradients squared for one right-hand side b (P,).  In exact
    arithmetic the residual after i steps is phi_i(A M^{-1})^2 r_0, phi_i being
    the residual polynomial of BiCG on A M^{-1} with the shadow residual r~
    (shadow "r": r~ = r_0, the usual choice; "Mr": r~ = M^{-1} r_0, for which
    phi_i is the polynomial of preconditioned CG when A and M are symmetric)."""
    b = b.ravel()
    P = b.size
    A0, M0 = A, M
    A = lambda v: np.asarray(A0(v.reshape(P, 1))).ravel()
    M = lambda v: np.asarray(M0(v.reshape(P, 1))).ravel()
    x = np.zeros(P) if x0 is None else np.array(x0, dtype=float).ravel()
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0, []
    hist = []
    it = 0
    while it < maxiter:
        r = b - A(x)
        if true_res is None and np.linalg.norm(r) / bn <= tol:
            break
        rt = r.copy() if shadow == "r" else M(r)  # shadow residual
        rho_old = None
        q = np.zeros(P)
        pd = np.zeros(P)
        restart = False
        while it < maxiter:
            rho = rt @ r
            if rho == 0.0:
                restart = True
                break
            if rho_old is None:
                u = r.copy()
                pd = u.copy()
            else:
                beta = rho / rho_old
                u = r + beta * q
                pd = u + beta * (q + beta * pd)
            ph = M(pd)
            vh = A(ph)
            sigma = rt @ vh
            if sigma == 0.0:
                restart = True
                break
            alpha = rho / sigma
            q = u - alpha * vh
            uh = M(u + q)
            x = x + alpha * uh
            r = r - alpha * A(uh)
            rho_old = rho
            it += 1
            hist.append(np.linalg.norm(r) / bn)
            if hist[-1] <= tol:
                break
        tr = np.linalg.norm(b - A(x)) / bn if true_res is None else true_res(x)
        if tr <= tol or it >= maxiter:
            break
        if not restart and hist and hist[-1] > tol:
            break
        # the recurrence drifted from the true residual: restart from it
    return x, it, hist


def bicg(A, M, MT, b, x0=None, tol=1e-10, maxiter=1000, true_res=None, AT=None):
    """Biconjugate gradients for one right-hand side b (P,): the primal system
    preconditioned by M, the shadow system by M^T (MT) with A^T (AT, default A:
    the normal matrix is symmetric).  With symmetric A and M its iterates are
    those of preconditioned CG."""
    b = b.ravel()
    P = b.size
    A0, M0, MT0 = A, M, MT
    AT0 = AT if AT is not None else A
    A = lambda v: np.asarray(A0(v.reshape(P, 1))).ravel()
    M = lambda v: np.asarray(M0(v.reshape(P, 1))).ravel()
    MT = lambda v: np.asarray(MT0(v.reshape(P, 1))).ravel()
    AT = lambda v: np.asarray(AT0(v.reshape(P, 1))).ravel()
    x = np.zeros(P) if x0 is None else np.array(x0, dtype=float).ravel()
    bn = np.linalg.norm(b)
    if bn == 0:
        return x, 0, []
    hist = []
    it = 0
    while it < maxiter:
        r = b - A(x)
        if true_res is None and np.linalg.norm(r) / bn <= tol:
            break
        rt = r.copy()
        rho_old = None
        pd = np.zeros(P)
        pt = np.zeros(P)
        restart = False
        while it < maxiter:
            z = M(r)
            zt = MT(rt)
            rho = z @ rt
            if rho == 0.0:
                restart = True
                break
            if rho_old is None:
                pd = z.copy()
                pt = zt.copy()
            else:
                beta = rho / rho_old
                pd = z + beta * pd
                pt = zt + beta * pt
            q = A(pd)
            qt = AT(pt)
            sigma = pt @ q
            if sigma == 0.0:
                restart = True
                break
            alpha = rho / sigma
            x = x + alpha * pd
            r = r - alpha * q
            rt = rt - alpha * qt
            rho_old = rho
            it += 1
            hist.append(np.linalg.norm(r) / bn)
            if hist[-1] <= tol:
                break
        tr = np.linalg.norm(b - A(x)) / bn if true_res is None else true_res(x)
        if tr <= tol or it >= maxiter:
            break
        if not restart and hist and hist[-1] > tol:
            break
    return x, it, hist
