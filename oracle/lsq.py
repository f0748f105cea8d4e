"""Dense least squares by Householder QR, and its adjoint.

The paper solves min ||H W - F||_2 directly with a QR-based least-squares
routine as its comparison solver (Sec. 5, opening paragraph) and derives the
normal equations H^T H W = H^T F (Sec. 2, after eq. (sys)).  The preconditioned
iterative methods reach the same unique minimiser when H has full column rank,
so this dense solution is the parity reference.

Householder QR written out: for each column k a reflector I - beta v v^T maps
H[k:, k] onto a multiple of e_1; R is the resulting upper triangle.
Adjoint: W = R^{-1} Q^T F, so dL/dF = Q R^{-T} dL/dW (with Q the thin factor).
"""
from __future__ import annotations

import numpy as np

EPS = np.finfo(float).eps


def householder_qr(A):
    """Returns (reflectors [(v, beta)], R (p x p)) with A = Q [R; 0]."""
    A = np.array(A, dtype=float, copy=True)
    n, p = A.shape
    if n < p:
        raise ValueError("least squares needs at least as many rows as columns")
    refl = []
    for k in range(p):
        x = A[k:, k]
        nx = np.linalg.norm(x)
        if nx == 0.0:
            refl.append((np.zeros_like(x), 0.0))
            continue
        alpha = -nx if x[0] >= 0 else nx
        v = x.copy()
        v[0] -= alpha
        beta = 2.0 / (v @ v)
        A[k:, k:] -= beta * np.outer(v, v @ A[k:, k:])
        refl.append((v, beta))
    return refl, np.triu(A[:p, :p])


def apply_qt(refl, B):
    B = np.array(B, dtype=float, copy=True)
    for k, (v, beta) in enumerate(refl):
        if beta:
            B[k:] -= beta * np.outer(v, v @ B[k:])
    return B


def apply_q(refl, B):
    B = np.array(B, dtype=float, copy=True)
    for k in range(len(refl) - 1, -1, -1):
        v, beta = refl[k]
        if beta:
            B[k:] -= beta * np.outer(v, v @ B[k:])
    return B


def back_substitute(R, B):
    """Solve R X = B for upper-triangular R by back substitution."""
    p = R.shape[0]
    X = np.zeros((p,) + B.shape[1:])
    for i in range(p - 1, -1, -1):
        X[i] = (B[i] - R[i, i + 1:] @ X[i + 1:]) / R[i, i]
    return X


def forward_substitute_t(R, B):
    """Solve R^T X = B (R upper triangular) by forward substitution."""
    p = R.shape[0]
    X = np.zeros((p,) + B.shape[1:])
    for i in range(p):
        X[i] = (B[i] - R[:i, i] @ X[:i]) / R[i, i]
    return X


def numerical_rank(R, n_rows):
    d = np.abs(np.diag(R))
    if d.size == 0:
        return 0
    return int(np.count_nonzero(d > 10.0 * n_rows * EPS * d.max()))


class QRSolver:
    """Factor once, solve / adjoint many times."""

    def __init__(self, H):
        self.n, self.p = H.shape
        self.refl, self.R = householder_qr(H)
        self.rank = numerical_rank(self.R, self.n)

    def solve(self, F):
        F2 = F.reshape(self.n, -1)
        QtF = apply_qt(self.refl, F2)
        return back_substitute(self.R, QtF[:self.p]).reshape((self.p,) + F.shape[1:])

    def adjoint(self, dW):
        """dF = H (H^T H)^{-1} dW = Q [R^{-T} dW; 0]."""
        dW2 = dW.reshape(self.p, -1)
        Y = np.zeros((self.n, dW2.shape[1]))
        Y[:self.p] = forward_substitute_t(self.R, dW2)
        return apply_q(self.refl, Y).reshape((self.n,) + dW.shape[1:])

    def cond_estimate(self):
        s = np.linalg.svd(self.R, compute_uv=False)
        return float(s[0] / s[-1]) if s[-1] > 0 else np.inf
