"""Random tanh features of one subdomain and the operator applied to them.

Paper eq. (rann) / (net): phi_k(x) = tanh(R_k . x~ + b_k) with R, b fixed.
Sec. 5 (Example 1): the input of each subdomain network is normalised to
[-1, 1]^d over the subdomain; read here as x~ = (x - mu_j) / sigma_j over the
support box.

Row entries (eqs. (sum), (system)): (H_j)_{ik} = A[L w_j phi_k](x_i) for a
collocation point, with A[u] = sum_i (-a_i d_ii u + beta_i d_i u) + c u, and
the Dirichlet trace (L w_j phi_k)(x_b) for a boundary point.  These are
computed here by writing u = M phi with M = L w_j and expanding the derivatives
of the product directly.
"""
from __future__ import annotations

import numpy as np


def features(X, mu_j, sigma, R, b):
    """tanh features and their first and pure second derivatives in x.

    Returns phi (n, m), dphi (d, n, m), d2phi (d, n, m)."""
    Xt = (X - mu_j[None, :]) / sigma[None, :]
    z = Xt @ R.T + b[None, :]
    t = np.tanh(z)
    sech2 = 1.0 - t * t
    d = X.shape[1]
    dphi = np.empty((d,) + t.shape)
    d2phi = np.empty((d,) + t.shape)
    for i in range(d):
        rho = R[:, i] / sigma[i]          # chain rule of the normalisation
        dphi[i] = sech2 * rho[None, :]
        d2phi[i] = -2.0 * t * sech2 * (rho * rho)[None, :]
    return t, dphi, d2phi


def multiplier(Lfun_rows, om, om_g, om_h):
    """M = L * w_j with derivatives (product rule).  Lfun_rows is (n, 1+2d)
    [L, dL/dx_i, d2L/dx_i^2] or None for L == 1."""
    if Lfun_rows is None:
        return om, om_g, om_h
    d = om_g.shape[1]
    L = Lfun_rows[:, 0]
    Lg = Lfun_rows[:, 1:1 + d]
    Lh = Lfun_rows[:, 1 + d:1 + 2 * d]
    M = L * om
    Mg = Lg * om[:, None] + L[:, None] * om_g
    Mh = Lh * om[:, None] + 2.0 * Lg * om_g + L[:, None] * om_h
    return M, Mg, Mh


def operator_rows(a, beta, c, M, Mg, Mh, phi, dphi, d2phi):
    """A[M phi_k] at interior points: u = M phi, d_i u = M_i phi + M phi_i,
    d_ii u = M_ii phi + 2 M_i phi_i + M phi_ii."""
    d = Mg.shape[1]
    out = c[:, None] * (M[:, None] * phi)
    for i in range(d):
        du = Mg[:, i:i + 1] * phi + M[:, None] * dphi[i]
        d2u = Mh[:, i:i + 1] * phi + 2.0 * Mg[:, i:i + 1] * dphi[i] + M[:, None] * d2phi[i]
        out += -a[:, i:i + 1] * d2u + beta[:, i:i + 1] * du
    return out


def value_rows(M, phi):
    """(M phi_k)(x): boundary (Dirichlet trace) and probe rows."""
    return M[:, None] * phi
