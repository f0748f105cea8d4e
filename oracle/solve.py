"""End-to-end oracle results (paper Algorithm 1, steps 1-7).

* reference(...)  : assemble, then the exact least-squares solution by the
                    oracle's own Householder QR (dense H; small and medium sizes)
* iterative(...)  : assemble, then CG (AS) or GMRES (RAS/SAS/AS) on the
                    block-sparse H with a Schwarz preconditioner
* refined(...)    : AS-PCG restarted from the recomputed normal residual, to
                    the FP64 floor (the full-size reference)
* normal_residual : ||H^T (F - H W)|| / ||H^T F|| per right-hand side
* adjoint         : dF = H (H^T H)^{-1} dW by QR; for the misfit
                    L = ||Pmat W - u_obs||^2 the seed is dW = 2 Pmat^T (Pmat W - u_obs)
"""
from __future__ import annotations

import numpy as np

from . import assemble as asm
from . import blocksparse as bs
from . import krylov as kr
from . import lsq
from . import schwarz as sw


def normal_residual(bh, W, Fs):
    W = W.reshape(bh.P, -1)
    g = bh.rmatvec(Fs)
    r = bh.rmatvec(Fs - bh.matvec(W))
    gn = np.linalg.norm(g, axis=0)
    gn[gn == 0] = 1.0
    return np.linalg.norm(r, axis=0) / gn


def reference(prob, pca_mode="rel_eig", tol=1e-8, V_force=None, p_force=None, sysm=None):
    if sysm is None:
        sysm = asm.assemble(prob, pca_mode, tol, V_force=V_force, p_force=p_force)
    H = sysm.dense()
    qr = lsq.QRSolver(H)
    W = qr.solve(sysm.Fs)
    return dict(sys=sysm, H=H, qr=qr, W=W, c=sysm.coeffs(W))


def iterative(prob, sysm, stencil="full", precond="as", method="cg", tol=1e-10,
              maxiter=2000, restart=50, local="chol"):
    bh = bs.BlockH(sysm)
    sten = sw.stencil(prob, stencil)
    M = sw.schwarz_blocks(bh, sten, kind=precond, local=local)
    rhs = bh.rmatvec(sysm.Fs)
    if method == "cg":
        W, iters, hist = kr.pcg(bh.normal, M.apply, rhs, tol=tol, maxiter=maxiter,
                                true_res=lambda X: normal_residual(bh, X, sysm.Fs))
    else:
        cols, iters, hist = [], [], []
        for q in range(rhs.shape[1]):
            if method == "cgs":
                x, it, h = kr.cgs(bh.normal, M.apply, rhs[:, q], tol=tol, maxiter=maxiter)
            elif method == "bicg":
                x, it, h = kr.bicg(bh.normal, M.apply, M.apply_T, rhs[:, q], tol=tol, maxiter=maxiter)
            else:
                x, it, h = kr.gmres(bh.normal, M.apply, rhs[:, q], restart=restart, tol=tol,
                                    maxiter=maxiter, side="right" if method == "gmres_right" else "left")
            cols.append(x)
            iters.append(it)
            hist.append(h)
        W = np.stack(cols, 1)
        iters = np.array(iters)
    return dict(W=W, iters=iters, hist=hist, M=M, bh=bh,
                res=normal_residual(bh, W, sysm.Fs))


def refined(prob, sysm, stencil="full", precond="as", tol=1e-10, inner=1e-4, cycles=30, maxiter=2000):
    """AS-PCG as iterative refinement: each cycle recomputes the normal residual
    r = H^T (F - H W) from the rows of H (the true residual of the stopping
    reading, which the recurrence residual drifts away from) and runs PCG on
    H^T H dW = r until the recurrence has reduced it by `inner`; W += dW.
    Stops when every right-hand side's true residual is at most tol, or when
    a cycle no longer reduces the largest one (the FP64 floor)."""
    bh = bs.BlockH(sysm)
    M = sw.schwarz_blocks(bh, sw.stencil(prob, stencil), kind=precond)
    k = sysm.Fs.shape[1]
    W = np.zeros((bh.P, k))
    res = normal_residual(bh, W, sysm.Fs)
    iters, hist = np.zeros(k, dtype=int), [res]
    for _ in range(cycles):
        todo = res > tol
        if not todo.any():
            break
        r = bh.rmatvec(sysm.Fs - bh.matvec(W))[:, todo]
        dW, it, _ = kr.pcg(bh.normal, M.apply, r, tol=inner, maxiter=maxiter)
        W[:, todo] += dW
        iters[todo] += it
        new = normal_residual(bh, W, sysm.Fs)
        if new.max() >= res.max():
            res = new
            break
        res = new
        hist.append(res)
    return dict(W=W, iters=iters, res=res, hist=hist)


def adjoint(qr, dW):
    return qr.adjoint(dW)


def misfit_seed(Pm, W, u_obs):
    """dL/dW for L = sum over RHS columns of ||Pmat W - u_obs||^2."""
    R = Pm @ W.reshape(Pm.shape[1], -1) - u_obs.reshape(Pm.shape[0], -1)
    return 2.0 * Pm.T @ R
