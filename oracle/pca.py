"""PCA of the local value matrix (paper Sec. 4).

Psi_j[i, k] = psi_j^k(x_i) = w_j(x_i) phi_k(x_i) over the rows of the subdomain
(eq. before (pca)).  A reduced SVD Psi_j = U S V^T (numpy's LAPACK SVD is the
primitive) gives singular values in descending order; the count p_j of values
above the threshold selects the leading p_j right singular vectors V_{p_j}
(eq. (pca)), and the reduced network is W_{p_j} . (V_{p_j}^T Phi_j) (eq. (pca_net)).

Threshold readings:
  * "abs_sigma": keep sigma_k > tau (the paper's constant threshold).
  * "rel_eig"  : keep lambda_k > tol * lambda_1 with lambda = sigma^2, i.e. the
                 eigenvalues of Psi^T Psi relative to the largest one.  The
                 configurations' "PCA tol" is read this way.
  * "off"      : no truncation, V = I.
A tie is reported when some lambda_k lies within relative 1e-6 of the threshold.
"""
from __future__ import annotations

import numpy as np

TIE_REL = 1e-6


def threshold_value(lam1, mode, tol):
    if mode == "rel_eig":
        return tol * lam1
    if mode == "abs_sigma":
        return tol * tol
    raise ValueError(mode)


def pca_basis(Psi, mode="rel_eig", tol=1e-8):
    """Returns (V_p (m, p), lam (min(n,m),) descending eigenvalues of Psi^T Psi, tie flag)."""
    m = Psi.shape[1]
    if mode == "off":
        return np.eye(m), None, False
    _, s, Vt = np.linalg.svd(Psi, full_matrices=False)
    lam = s * s
    thr = threshold_value(lam[0], mode, tol)
    p = int(np.count_nonzero(lam > thr))
    tie = bool(np.any(np.abs(lam - thr) <= TIE_REL * thr))
    return Vt[:p].T.copy(), lam, tie
