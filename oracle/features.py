"""Random tanh features of one subdomain and the operator applied to them.

Paper eq. (rann) / (net): phi_k(x) = tanh(R_k . x~ + b_k) with R, b fixed.
Sec. 5 (Example 1): the input of each subdomain network is normalised to
[-1, 1]^d over the subdomain; read here as x~ = (x - mu_j) / sigma_j over the
support box.

Several hidden layers (eq. (net)): Phi_j = f^{n-1} o ... o f^1 with
f^i(y) = tanh(R_i y + b_i), all R_i, b_i fixed.  Its derivatives in x are
carried layer by layer in forward mode (network_features): with a = R y + b,
d_q a = R d_q y and d_qq a = R d_qq y, the layer output t = tanh a has
d_q t = s d_q a and d_qq t = s d_qq a - 2 t s (d_q a)^2, s = 1 - t^2; the input
y = x~ has d_q y = e_q / sigma_q and d_qq y = 0.

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


def network_features(X, mu_j, sigma, layers):
    """Outputs of the last hidden layer of Phi_j (eq. (net)) and their first and
    pure second derivatives in x.  layers = [(R_1, b_1), ..., (R_{n-1}, b_{n-1})]
    with R_1 acting on the normalised input.  Returns phi (n, m), dphi (d, n, m),
    d2phi (d, n, m); one layer gives the same values as features()."""
    n, d = X.shape
    y = (X - mu_j[None, :]) / sigma[None, :]
    dy = np.zeros((d, n, d))
    for q in range(d):
        dy[q][:, q] = 1.0 / sigma[q]
    d2y = np.zeros((d, n, d))
    for R, b in layers:
        a = y @ R.T + b[None, :]
        da = dy @ R.T
        d2a = d2y @ R.T
        t = np.tanh(a)
        s = 1.0 - t * t
        y = t
        dy = s[None] * da
        d2y = s[None] * d2a - 2.0 * (t * s)[None] * da * da
    return y, dy, d2y


def subdomain_features(prob, X, j):
    """phi, dphi, d2phi of subdomain j's network at X: one hidden layer
    (features) or the inner layers of prob.inner[j] followed by R_j, b_j."""
    from .geometry import centre
    mu_j = centre(prob, j)
    inner = getattr(prob, "inner", None)
    if inner is None:
        return features(X, mu_j, prob.sigma, prob.R[j], prob.b[j])
    return network_features(X, mu_j, prob.sigma, list(inner[j]) + [(prob.R[j], prob.b[j])])


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
