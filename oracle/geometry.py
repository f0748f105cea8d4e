"""Subdomain supports and the window-function partition of unity.

Paper Sec. 2: the window functions w_j have support in the closure of the
subdomain and sum to one on the domain.  Sec. 5, Example 1: the unnormalised
window is a product over dimensions of [1 + cos(pi (x_i - mu_i)/sigma_i)]^2 and
w_j is that window divided by the sum of all windows; mu_i and sigma_i are the
centre and half-width of the subdomain in dimension i.

Reading used here: the product runs over all d dimensions, the window is zero
outside the open support box |x_i - mu_i| < sigma_i, and a point belongs to the
row set S_j of subdomain j iff it lies strictly inside the box, tested as
|x_i - mu_i| < sigma_i * (1 - 1e-12) in every dimension.
"""
from __future__ import annotations

import math

import numpy as np

EDGE = 1.0 - 1e-12


def subdomain_index(l, j):
    """Tensor coordinates of linear subdomain index j (dimension 0 fastest)."""
    out = []
    for li in l:
        out.append(j % int(li))
        j //= int(li)
    return tuple(out)


def centre(prob, j):
    cc = subdomain_index(prob.l, j)
    return np.array([prob.mu[i][cc[i]] for i in range(prob.d)], dtype=float)


def all_points(prob):
    """Interior collocation points followed by boundary points (global row order)."""
    return np.concatenate([prob.X_int, prob.X_bnd], axis=0)


def member_mask(X, mu_j, sigma):
    """Boolean mask of points strictly inside the support box of one subdomain."""
    inside = np.ones(X.shape[0], dtype=bool)
    for i in range(X.shape[1]):
        inside &= np.abs(X[:, i] - mu_j[i]) < sigma[i] * EDGE
    return inside


def support_rows(prob, X=None):
    """Row sets S_j (sorted global row indices) for every subdomain."""
    X = all_points(prob) if X is None else X
    return [np.nonzero(member_mask(X, centre(prob, j), prob.sigma))[0]
            for j in range(prob.J)]


def bump_1d(tau):
    """beta(tau) = (1 + cos(pi tau))^2 and its first two derivatives in tau."""
    c = np.cos(math.pi * tau)
    s = np.sin(math.pi * tau)
    val = (1.0 + c) ** 2
    d1 = -2.0 * math.pi * (1.0 + c) * s
    d2 = 2.0 * math.pi ** 2 * (s * s - (1.0 + c) * c)
    return val, d1, d2


def window_raw(X, mu_j, sigma):
    """Unnormalised window of one subdomain at points X (zero outside the support).

    Returns (w, grad (n,d), hess_diag (n,d)) as derivatives in x.
    """
    n, d = X.shape
    inside = member_mask(X, mu_j, sigma)
    vals, d1s, d2s = [], [], []
    for i in range(d):
        tau = (X[:, i] - mu_j[i]) / sigma[i]
        v, a1, a2 = bump_1d(tau)
        vals.append(v)
        d1s.append(a1 / sigma[i])
        d2s.append(a2 / sigma[i] ** 2)
    w = np.prod(vals, axis=0)
    grad = np.zeros((n, d))
    hess = np.zeros((n, d))
    for i in range(d):
        others = np.ones(n)
        for q in range(d):
            if q != i:
                others = others * vals[q]
        grad[:, i] = d1s[i] * others
        hess[:, i] = d2s[i] * others
    w = np.where(inside, w, 0.0)
    grad = np.where(inside[:, None], grad, 0.0)
    hess = np.where(inside[:, None], hess, 0.0)
    return w, grad, hess


def window_sum(prob, X):
    """S = sum over all subdomains of the unnormalised windows, with derivatives."""
    n, d = X.shape
    S = np.zeros(n)
    Sg = np.zeros((n, d))
    Sh = np.zeros((n, d))
    for j in range(prob.J):
        w, g, h = window_raw(X, centre(prob, j), prob.sigma)
        S += w
        Sg += g
        Sh += h
    return S, Sg, Sh


def partition_of_unity(prob, X, j, sums=None):
    """Normalised window w_j = w_hat_j / S at points X, with first and pure second
    derivatives by the quotient rule.  Points with S == 0 (outside every support)
    raise: the method needs every collocation point covered."""
    S, Sg, Sh = window_sum(prob, X) if sums is None else sums
    if np.any(S <= 0):
        raise ValueError("a point lies outside every subdomain support")
    w, g, h = window_raw(X, centre(prob, j), prob.sigma)
    om = w / S
    om_g = (g - om[:, None] * Sg) / S[:, None]
    om_h = (h - 2.0 * om_g * Sg - om[:, None] * Sh) / S[:, None]
    return om, om_g, om_h
