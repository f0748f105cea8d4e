"""Assembly of the collocation least-squares system (paper eqs. (sum), (system),
(system_new)) on per-subdomain blocks.

Global row order: interior collocation points, then boundary points.  Block j
holds the rows S_j (points strictly inside the support of subdomain j) and the
p_j columns of subdomain j after PCA:

  interior row x_i:  A[L w_j (V_{p_j}^T Phi_j)](x_i)
  boundary row x_b:  lambda_B (L w_j (V_{p_j}^T Phi_j))(x_b)

Boundary treatment (reading): one ansatz u = L sum_j w_j W_j . Phi_j + G.  In
"rows" mode L = 1, G = 0 and the Dirichlet data enter as boundary rows weighted
by lambda_B (the penalty rows of Sec. 5, Example 2); in "constrain" mode L and G
come from the constraining operator (eq. (operator)) and there are no boundary
rows.  The right-hand side handed in is f - A[G] (interior) and g - G
(boundary), unscaled; the boundary part is multiplied by lambda_B here.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import features as ft
from . import geometry as geo
from . import pca as pc


@dataclasses.dataclass
class System:
    N_I: int
    N: int
    S: List[np.ndarray]          # row sets
    p: np.ndarray                # post-PCA widths
    V: List[np.ndarray]          # (m_j, p_j)
    lam: List[Optional[np.ndarray]]
    ties: List[bool]
    col_off: np.ndarray          # (J+1,)
    blocks: List[np.ndarray]     # (n_j, p_j)
    raw: List[np.ndarray]        # (n_j, m_j) rows before the PCA layer
    Fs: np.ndarray               # (N, k) right-hand side with boundary rows scaled

    @property
    def J(self):
        return len(self.S)

    @property
    def P(self):
        return int(self.col_off[-1])

    def dense(self):
        H = np.zeros((self.N, self.P))
        for j in range(self.J):
            H[np.ix_(self.S[j], np.arange(self.col_off[j], self.col_off[j + 1]))] = self.blocks[j]
        return H

    def coeffs(self, W):
        """Raw-neuron coefficients c_j = V_{p_j} W_j, stacked over subdomains."""
        W = W.reshape(self.P, -1)
        return np.concatenate([self.V[j] @ W[self.col_off[j]:self.col_off[j + 1]]
                               for j in range(self.J)], axis=0)


def local_terms(prob, X, rows, j, sums, Lrows):
    """Window, multiplier and features of subdomain j at the points X[rows]."""
    Xr = X[rows]
    om, om_g, om_h = geo.partition_of_unity(prob, Xr, j, sums=tuple(s[rows] for s in sums))
    Lr = None if Lrows is None else Lrows[rows]
    M, Mg, Mh = ft.multiplier(Lr, om, om_g, om_h)
    phi, dphi, d2phi = ft.subdomain_features(prob, Xr, j)
    return om, M, Mg, Mh, phi, dphi, d2phi


def raw_rows(prob, rows, M, Mg, Mh, phi, dphi, d2phi):
    """Operator rows for interior points, lambda_B-weighted value rows for boundary points."""
    interior = rows < prob.N_I
    out = np.empty(phi.shape)
    ii = np.nonzero(interior)[0]
    if ii.size:
        gi = rows[ii]
        out[ii] = ft.operator_rows(prob.a[gi], prob.beta[gi], prob.c[gi], M[ii], Mg[ii], Mh[ii],
                                   phi[ii], dphi[:, ii], d2phi[:, ii])
    bb = np.nonzero(~interior)[0]
    if bb.size:
        out[bb] = prob.lambda_B * ft.value_rows(M[bb], phi[bb])
    return out


def assemble(prob, pca_mode="rel_eig", tol=1e-8, V_force=None, p_force=None):
    """Build the block system.  V_force (list of (m_j, p_j)) injects a PCA basis;
    p_force (J,) forces the truncation counts of the oracle's own PCA."""
    X = geo.all_points(prob)
    sums = geo.window_sum(prob, X)
    S = geo.support_rows(prob, X)
    V, lam, ties, blocks, raws = [], [], [], [], []
    for j in range(prob.J):
        rows = S[j]
        om, M, Mg, Mh, phi, dphi, d2phi = local_terms(prob, X, rows, j, sums, prob.Lfun)
        if V_force is not None:
            Vj, lj, tj = V_force[j], None, False
        else:
            Psi = om[:, None] * phi                       # value matrix, without L
            Vj, lj, tj = pc.pca_basis(Psi, pca_mode, tol)
            if p_force is not None and pca_mode != "off":
                _, s, Vt = np.linalg.svd(Psi, full_matrices=False)
                Vj = Vt[:int(p_force[j])].T.copy()
        A_raw = raw_rows(prob, rows, M, Mg, Mh, phi, dphi, d2phi)
        V.append(Vj)
        lam.append(lj)
        ties.append(tj)
        raws.append(A_raw)
        blocks.append(A_raw @ Vj)
    p = np.array([v.shape[1] for v in V], dtype=np.int64)
    col_off = np.concatenate([[0], np.cumsum(p)])
    Fs = np.array(prob.F, dtype=float, copy=True)
    Fs[prob.N_I:] *= prob.lambda_B
    return System(N_I=prob.N_I, N=prob.N, S=S, p=p, V=V, lam=lam, ties=ties,
                  col_off=col_off, blocks=blocks, raw=raws, Fs=Fs)


def probe_matrix(prob, sysm, Xq, Lq=None):
    """Value rows at probe points in the PCA basis: U = Pmat W evaluates
    sum_j L w_j (V_{p_j}^T Phi_j) . W_j (eq. (netdd) with eq. (pca_net)), without G."""
    sums = geo.window_sum(prob, Xq)
    Pm = np.zeros((Xq.shape[0], sysm.P))
    for j in range(prob.J):
        rows = np.nonzero(geo.member_mask(Xq, geo.centre(prob, j), prob.sigma))[0]
        if rows.size == 0:
            continue
        om, _, _ = geo.partition_of_unity(prob, Xq[rows], j, sums=tuple(s[rows] for s in sums))
        M = om if Lq is None else Lq[rows] * om
        phi, _, _ = ft.subdomain_features(prob, Xq[rows], j)
        Pm[np.ix_(rows, np.arange(sysm.col_off[j], sysm.col_off[j + 1]))] = (M[:, None] * phi) @ sysm.V[j]
    return Pm
