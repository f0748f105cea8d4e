"""The block-sparse collocation matrix H = [H_1, ..., H_J] on per-subdomain blocks
(paper Sec. 3 remark: domain decomposition makes H block sparse).

Block j is dense over its row set S_j and its own p_j columns; products with H
and H^T touch only those blocks.  Used where a dense N x P matrix would not fit.
"""
from __future__ import annotations

import numpy as np


class BlockH:
    def __init__(self, sysm):
        self.S = sysm.S
        self.blocks = sysm.blocks
        self.col_off = sysm.col_off
        self.N = sysm.N
        self.P = sysm.P

    def matvec(self, X):
        """Y = H X for X (P, k)."""
        X = X.reshape(self.P, -1)
        Y = np.zeros((self.N, X.shape[1]))
        for j, (rows, B) in enumerate(zip(self.S, self.blocks)):
            Y[rows] += B @ X[self.col_off[j]:self.col_off[j + 1]]
        return Y

    def rmatvec(self, Y):
        """X = H^T Y for Y (N, k)."""
        Y = Y.reshape(self.N, -1)
        X = np.zeros((self.P, Y.shape[1]))
        for j, (rows, B) in enumerate(zip(self.S, self.blocks)):
            X[self.col_off[j]:self.col_off[j + 1]] = B.T @ Y[rows]
        return X

    def normal(self, X):
        return self.rmatvec(self.matvec(X))

    def local_matrix(self, subs):
        """Columns of the subdomains in `subs` restricted to the union of their rows:
        returns (rows, dense block)."""
        rows = np.unique(np.concatenate([self.S[j] for j in subs]))
        q = int(sum(self.col_off[j + 1] - self.col_off[j] for j in subs))
        Hl = np.zeros((rows.size, q))
        c0 = 0
        for j in subs:
            pj = int(self.col_off[j + 1] - self.col_off[j])
            loc = np.searchsorted(rows, self.S[j])
            Hl[loc, c0:c0 + pj] = self.blocks[j]
            c0 += pj
        return rows, Hl
