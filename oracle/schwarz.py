"""Overlapping Schwarz preconditioners for H^T H (paper Sec. 3).

  AS : M^{-1} = sum_i R_i^T A_i^{-1} R_i,          A_i = R_i H^T H R_i^T
  RAS: M^{-1} = sum_i R_i^T D_i A_i^{-1} R_i,      D_i Boolean, sum_i R_i^T D_i R_i = I
  SAS: as RAS with (D_i)_cc = 1 / (number of blocks containing unknown c)
       (Sec. 5, Example 1)

R_i is a Boolean column selector.  Reading of which columns block i selects: the
basis functions of every subdomain in the stencil of subdomain i, in increasing
subdomain order:
  * "full": all subdomains whose open support box intersects the support of i
            (overlapping coefficient blocks; with at most two subdomains per
            dimension every block is the whole system)
  * "face": i and its neighbours that differ by one in exactly one tensor index
  * "self": i only (block Jacobi)
RAS ownership (the Boolean algebraic partition of unity D_i): the columns of
subdomain j belong to the first block, in increasing block order, whose
stencil contains j.  With the full stencil this assigns each subdomain to the
block of its lower-left neighbour (clamped at the domain edge), so the blocks
near the origin own several subdomains and some blocks own none.  Table 1a's
RAS spectrum (real parts in [0.1, 2.1]) and iteration counts are reproduced
under this reading; owning the centre subdomain of each block instead gives
real parts down to about -0.9 and GMRES counts ten times the paper's.

Local inverse (Sec. 3): either the QR factorisation A_i = Q_i P_i with
A_i^{-1} = P_i^{-1} Q_i^T and a pseudo-inverse when P_i is singular ("qr"), or an
equilibrated Cholesky factorisation with a diagonal shift on breakdown ("chol").
Both define the local inverse of the same block; they differ only in rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import geometry as geo

EPS = np.finfo(float).eps


def stencil(prob, kind):
    J = prob.J
    coords = [geo.subdomain_index(prob.l, j) for j in range(J)]
    cen = [geo.centre(prob, j) for j in range(J)]
    out = []
    for i in range(J):
        if kind == "self":
            out.append(np.array([i]))
            continue
        nb = []
        for j in range(J):
            diff = [abs(coords[i][q] - coords[j][q]) for q in range(prob.d)]
            if kind == "face":
                if sum(diff) <= 1:
                    nb.append(j)
            elif kind == "full":
                if all(abs(cen[i][q] - cen[j][q]) < 2.0 * prob.sigma[q] for q in range(prob.d)):
                    nb.append(j)
            else:
                raise ValueError(kind)
        out.append(np.array(nb))
    return out


def ras_owner(sten):
    """owner[j] = the first block (increasing index) whose stencil holds subdomain j."""
    J = len(sten)
    owner = np.full(J, -1, dtype=np.int64)
    for i in range(J):
        for j in sten[i]:
            if owner[j] < 0:
                owner[j] = i
    return owner


def block_columns(col_off, subs):
    return np.concatenate([np.arange(col_off[j], col_off[j + 1]) for j in subs])


def chol_local(A, shift_c=10.0, max_tries=12):
    """Equilibrated Cholesky D A D = L L^T with D = diag(A)^{-1/2}; on breakdown
    retry with D A D + eps I, eps = shift_c * u * q, growing by 10 each time.
    Returns a solve function and the number of shifts taken."""
    q = A.shape[0]
    dg = np.diag(A).copy()
    dg[dg <= 0] = 1.0
    Dv = 1.0 / np.sqrt(dg)
    B = Dv[:, None] * A * Dv[None, :]
    eps = 0.0
    for t in range(max_tries):
        try:
            L = np.linalg.cholesky(B + eps * np.eye(q))
            break
        except np.linalg.LinAlgError:
            eps = shift_c * EPS * q if eps == 0.0 else eps * 10.0
    else:
        raise np.linalg.LinAlgError("local block not positive definite after shifts")
    shifts = t

    def solve(r):
        y = sla.solve_triangular(L, Dv[:, None] * r.reshape(q, -1), lower=True)
        z = sla.solve_triangular(L.T, y, lower=False)
        return Dv[:, None] * z

    return solve, shifts


def qr_local(A):
    """A_i = Q P, A_i^{-1} = P^{-1} Q^T; pseudo-inverse of P when it is singular."""
    q = A.shape[0]
    Q, P = np.linalg.qr(A)
    d = np.abs(np.diag(P))
    singular = d.min() <= q * EPS * d.max()
    Pinv = np.linalg.pinv(P) if singular else None

    def solve(r):
        rhs = Q.T @ r.reshape(q, -1)
        if Pinv is not None:
            return Pinv @ rhs
        return sla.solve_triangular(P, rhs, lower=False)

    return solve, int(singular)


class Schwarz:
    """M^{-1} for H^T H given a function that returns the local block A_i."""

    def __init__(self, col_off, sten, local_block, kind="as", local="chol"):
        self.col_off = col_off
        self.sten = sten
        self.kind = kind
        self.P = int(col_off[-1])
        self.idx = [block_columns(col_off, s) for s in sten]
        self.solvers = []
        self.shifts = 0
        for i, s in enumerate(sten):
            A = local_block(i, self.idx[i])
            solve, sh = (chol_local(A) if local == "chol" else qr_local(A))
            self.solvers.append(solve)
            self.shifts += sh
        mult = np.zeros(self.P)
        for ix in self.idx:
            mult[ix] += 1.0
        self.mult = mult
        self.owner = ras_owner(sten)
        self.weights = []
        for i, s in enumerate(sten):
            ix = self.idx[i]
            if kind == "as":
                w = np.ones(ix.size)
            elif kind == "ras":
                w = np.concatenate([np.full(col_off[j + 1] - col_off[j], float(self.owner[j] == i))
                                    for j in s])
            elif kind == "sas":
                w = 1.0 / mult[ix]
            else:
                raise ValueError(kind)
            self.weights.append(w)

    def apply(self, R):
        R2 = R.reshape(self.P, -1)
        Z = np.zeros_like(R2)
        for ix, solve, w in zip(self.idx, self.solvers, self.weights):
            Z[ix] += w[:, None] * solve(R2[ix])
        return Z.reshape(R.shape)

    def apply_T(self, R):
        """The transpose M^{-T} = sum_i R_i^T A_i^{-1} D_i R_i (A_i^{-1} is
        symmetric): the weights act on the restricted input instead of the
        local result; equal to apply for AS."""
        R2 = R.reshape(self.P, -1)
        Z = np.zeros_like(R2)
        for ix, solve, w in zip(self.idx, self.solvers, self.weights):
            Z[ix] += solve(w[:, None] * R2[ix])
        return Z.reshape(R.shape)

    def dense(self):
        return self.apply(np.eye(self.P))


def schwarz_dense(HtH, col_off, sten, kind="as", local="chol"):
    return Schwarz(col_off, sten, lambda i, ix: HtH[np.ix_(ix, ix)], kind, local)


def schwarz_blocks(bh, sten, kind="as", local="chol"):
    """Local blocks from the block-sparse H: A_i = H_N(i)^T H_N(i) over the union of rows."""
    def local_block(i, ix):
        _, Hl = bh.local_matrix(sten[i])
        return Hl.T @ Hl
    return Schwarz(bh.col_off, sten, local_block, kind, local)
