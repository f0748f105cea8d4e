"""Pins of the oracle's several-hidden-layer features (paper eq. (net)).

The network Phi_j = f^{n-1} o ... o f^1, f^i(y) = tanh(R_i y + b_i), is written
out below as a plain complex-safe composition (its definition); the oracle's
forward-mode derivatives are checked against complex-step derivatives of that
composition (exact to rounding for the first derivative) and against central
differences of the complex-step derivative (second derivative).  The rows,
probe values and the solve built on them are pinned through finite differences
of L w_j phi_k and a manufactured solution."""
import numpy as np
import pytest

from oracle import assemble as asm
from oracle import features as ft
from oracle import geometry as geo
from oracle import lsq
from paper_2412_19207_amd import workloads as wl


def _net_value(X, mu, sigma, layers):
    # eq. (net) on the normalised input, complex-safe
    y = (X - mu) / sigma
    for R, b in layers:
        y = np.tanh(y @ R.T + b)
    return y


def _random_net(rng, d, widths, m):
    layers, w_prev = [], d
    for i, w in enumerate(list(widths) + [m]):
        s = 2.0 if i == 0 else 3.0 / np.sqrt(w_prev)
        layers.append((s * rng.uniform(-1, 1, (w, w_prev)), rng.uniform(-1, 1, w)))
        w_prev = w
    return layers


def test_one_layer_network_is_the_closed_form():
    rng = np.random.default_rng(11)
    d, m = 3, 13
    mu = rng.uniform(0, 1, d)
    sigma = rng.uniform(0.1, 0.3, d)
    R = 2.0 * rng.uniform(-1, 1, (m, d))
    b = rng.uniform(-1, 1, m)
    X = mu + sigma * rng.uniform(-1, 1, (31, d))
    got = ft.network_features(X, mu, sigma, [(R, b)])
    ref = ft.features(X, mu, sigma, R, b)
    for g, r in zip(got, ref):
        assert np.max(np.abs(g - r)) <= 1e-14 * (1 + np.max(np.abs(r)))


@pytest.mark.parametrize("d,widths", [(1, (4,)), (2, (6, 9)), (3, (5, 7, 6))])
def test_network_values_and_derivatives_complex_step(d, widths):
    rng = np.random.default_rng(5 + d)
    m = 11
    mu = rng.uniform(0, 1, d)
    sigma = rng.uniform(0.1, 0.3, d)
    layers = _random_net(rng, d, widths, m)
    X = mu + sigma * rng.uniform(-1, 1, (27, d))
    phi, dphi, d2phi = ft.network_features(X, mu, sigma, layers)
    assert phi.shape == (27, m) and dphi.shape == (d, 27, m)
    assert np.max(np.abs(phi - _net_value(X, mu, sigma, layers))) < 1e-15
    h = 1e-30
    for q in range(d):
        e = np.zeros(d)
        e[q] = 1.0

        def cs1(Y):
            return np.imag(_net_value(Y + 1j * h * e, mu, sigma, layers)) / h

        assert np.max(np.abs(cs1(X) - dphi[q])) < 1e-13 * (1 + np.max(np.abs(dphi[q])))
        # second derivative: 6th-order central difference of the exact first derivative
        hh = 2e-3 * sigma[q]
        c1 = np.array([-1, 9, -45, 0, 45, -9, 1]) / 60.0
        fd = sum(c * cs1(X + s * hh * e) for c, s in zip(c1, range(-3, 4))) / hh
        assert np.max(np.abs(fd - d2phi[q])) < 1e-8 * (1 + np.max(np.abs(d2phi[q])))


def _L_closed_form(X, rho):
    out = np.ones(X.shape[0])
    for i in range(X.shape[1]):
        out *= np.tanh(X[:, i] / rho) * np.tanh((1 - X[:, i]) / rho)
    return out


@pytest.mark.parametrize("kind", ["rows", "constrain", "rows3d"])
def test_deep_operator_rows_match_finite_differences(kind):
    if kind == "rows":
        prob = wl.small2d(inner_widths=(6, 9))
        L_of = None
    elif kind == "rows3d":
        prob = wl.small3d(inner_widths=(7,))
        L_of = None
    else:
        prob = wl.ex1_replica(n=1, l=3, m=9, pts=21, inner_widths=(5, 8))
        L_of = lambda Y: _L_closed_form(Y, 0.5)  # ex1_replica with n = 1: rho = 1/2
    X = geo.all_points(prob)
    sums = geo.window_sum(prob, X)
    j = prob.J // 2
    rows = geo.support_rows(prob, X)[j]
    rows = rows[rows < prob.N_I][::5]
    om, M, Mg, Mh, phi, dphi, d2phi = asm.local_terms(prob, X, rows, j, sums, prob.Lfun)
    got = asm.raw_rows(prob, rows, M, Mg, Mh, phi, dphi, d2phi)
    mu = geo.centre(prob, j)
    layers = list(prob.inner[j]) + [(prob.R[j], prob.b[j])]

    def u(Y):
        om_y = geo.partition_of_unity(prob, Y, j)[0]
        L = np.ones(Y.shape[0]) if L_of is None else L_of(Y)
        return (L * om_y)[:, None] * _net_value(Y, mu, prob.sigma, layers)

    Xr = X[rows]
    h = 2e-3 * float(np.min(prob.sigma))
    c1 = np.array([-1, 9, -45, 0, 45, -9, 1]) / 60.0
    c2 = np.array([2, -27, 270, -490, 270, -27, 2]) / 180.0
    expect = prob.c[rows][:, None] * u(Xr)
    for i in range(prob.d):
        e = np.zeros(prob.d)
        e[i] = h
        vals = [u(Xr + s * e) for s in range(-3, 4)]
        d1 = sum(cc * v for cc, v in zip(c1, vals)) / h
        d2 = sum(cc * v for cc, v in zip(c2, vals)) / h ** 2
        expect += -prob.a[rows, i][:, None] * d2 + prob.beta[rows, i][:, None] * d1
    scale = np.max(np.abs(expect))
    assert np.max(np.abs(got - expect)) < 1e-6 * scale


def test_deep_probe_matrix_evaluates_the_network():
    """U = Pmat W equals sum_j w_j(x) Phi_j(x) . (V_j W_j) from the definition."""
    prob = wl.small2d(inner_widths=(6, 9))
    sysm = asm.assemble(prob, "rel_eig", 1e-10)
    rng = np.random.default_rng(2)
    W = rng.standard_normal((sysm.P, 2))
    Xq = prob.probes
    got = asm.probe_matrix(prob, sysm, Xq) @ W
    c = sysm.coeffs(W)
    moff = np.concatenate([[0], np.cumsum(prob.m)])
    expect = np.zeros((Xq.shape[0], 2))
    for j in range(prob.J):
        rows = np.nonzero(geo.member_mask(Xq, geo.centre(prob, j), prob.sigma))[0]
        om = geo.partition_of_unity(prob, Xq[rows], j)[0]
        layers = list(prob.inner[j]) + [(prob.R[j], prob.b[j])]
        expect[rows] += om[:, None] * (_net_value(Xq[rows], geo.centre(prob, j), prob.sigma, layers)
                                       @ c[moff[j]:moff[j + 1]])
    assert np.max(np.abs(got - expect)) < 1e-12 * (1 + np.max(np.abs(expect)))


def test_deep_network_recovers_a_manufactured_solution():
    """Two inner layers of width 24 on the small 2D problem: the least-squares
    solution approximates the exact solution (one hidden layer of the same
    widths gives 1.6e-2 relative probe error here; two inner layers 6.2e-3)."""
    prob = wl.small2d(inner_widths=(24, 24))
    sysm = asm.assemble(prob, "rel_eig", 1e-12)
    W = lsq.QRSolver(sysm.dense()).solve(sysm.Fs[:, :1])
    U = asm.probe_matrix(prob, sysm, prob.probes) @ W
    err = np.linalg.norm(U[:, 0] - prob.u_probe) / np.linalg.norm(prob.u_probe)
    assert err < 2e-2
