"""Pins of the oracle's features and row entries: complex-step derivatives of the
tanh features (tanh is analytic), and finite differences of the scalar function
L w_j phi_k for the operator rows (paper eqs. (rann), (sum), (system))."""
import numpy as np
import pytest

from oracle import assemble as asm
from oracle import features as ft
from oracle import geometry as geo
from paper_2412_19207_amd import workloads as wl


def _tanh_feature(X, mu, sigma, R, b):
    # the plain definition phi_k(x) = tanh(R_k . (x - mu)/sigma + b_k), complex-safe
    return np.tanh(((X - mu) / sigma) @ R.T + b)


def test_feature_derivatives_complex_step():
    rng = np.random.default_rng(3)
    d, m = 3, 17
    mu = rng.uniform(0, 1, d)
    sigma = rng.uniform(0.1, 0.3, d)
    R = 2.0 * rng.uniform(-1, 1, (m, d))
    b = rng.uniform(-1, 1, m)
    X = mu + sigma * rng.uniform(-1, 1, (25, d))
    phi, dphi, d2phi = ft.features(X, mu, sigma, R, b)
    assert np.allclose(phi, np.tanh(((X - mu) / sigma) @ R.T + b), rtol=0, atol=1e-15)
    h = 1e-30
    for i in range(d):
        e = np.zeros(d)
        e[i] = 1.0
        cs = np.imag(_tanh_feature(X + 1j * h * e, mu, sigma, R, b)) / h
        assert np.max(np.abs(cs - dphi[i])) < 1e-13 * (1 + np.max(np.abs(dphi[i])))

        # second derivative: 4th-order central difference of the exact complex-step first derivative
        def cs1(Y):
            return np.imag(_tanh_feature(Y + 1j * h * e, mu, sigma, R, b)) / h
        hh = 1e-3 * sigma[i]
        fd = (cs1(X - 2 * hh * e) - 8 * cs1(X - hh * e) + 8 * cs1(X + hh * e) - cs1(X + 2 * hh * e)) / (12 * hh)
        assert np.max(np.abs(fd - d2phi[i])) < 1e-7 * (1 + np.max(np.abs(d2phi[i])))


def _L_closed_form(X, rho):
    out = np.ones(X.shape[0])
    for i in range(X.shape[1]):
        out *= np.tanh(X[:, i] / rho) * np.tanh((1 - X[:, i]) / rho)
    return out


@pytest.mark.parametrize("kind", ["rows", "constrain"])
def test_operator_rows_match_finite_differences(kind):
    if kind == "rows":
        prob = wl.small2d()
    else:
        prob = wl.ex1_replica(n=1, l=3, m=9, pts=21)
    rho = 0.5  # ex1_replica with n=1 uses rho = (1/2)^1
    X = geo.all_points(prob)
    sums = geo.window_sum(prob, X)
    j = prob.J // 2
    rows = geo.support_rows(prob, X)[j]
    rows = rows[rows < prob.N_I][::7]
    om, M, Mg, Mh, phi, dphi, d2phi = asm.local_terms(prob, X, rows, j, sums, prob.Lfun)
    got = asm.raw_rows(prob, rows, M, Mg, Mh, phi, dphi, d2phi)

    mu = geo.centre(prob, j)

    def u(Y):
        om_y = geo.partition_of_unity(prob, Y, j)[0]
        L = np.ones(Y.shape[0]) if kind == "rows" else _L_closed_form(Y, rho)
        return (L * om_y)[:, None] * _tanh_feature(Y, mu, prob.sigma, prob.R[j], prob.b[j])

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


def test_boundary_rows_are_weighted_values():
    prob = wl.small2d()
    sysm = asm.assemble(prob, "off", 0.0)
    X = geo.all_points(prob)
    for j in [0, prob.J - 1]:
        rows = sysm.S[j]
        sel = np.nonzero(rows >= prob.N_I)[0]
        assert sel.size > 0
        Y = X[rows[sel]]
        om = geo.partition_of_unity(prob, Y, j)[0]
        expect = prob.lambda_B * om[:, None] * _tanh_feature(Y, geo.centre(prob, j), prob.sigma,
                                                            prob.R[j], prob.b[j])
        assert np.allclose(sysm.blocks[j][sel], expect, rtol=1e-13, atol=1e-13)
