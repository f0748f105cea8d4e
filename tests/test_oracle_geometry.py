"""Pins of the oracle's geometry and partition of unity against closed forms,
finite differences and brute force (paper Sec. 2 window functions; Sec. 5
Example 1 window formula)."""
import math

import numpy as np
import pytest

from oracle import geometry as geo
from paper_2412_19207_amd import workloads as wl


@pytest.fixture(scope="module", params=["small2d", "small3d", "ex1", "cfg1"])
def prob(request):
    if request.param == "ex1":
        return wl.ex1_replica(l=4, m=8, pts=20)
    return wl.make(request.param)


def random_points(prob, n=400, seed=0):
    rng = np.random.default_rng(seed)
    return prob.lo + (prob.hi - prob.lo) * rng.uniform(0.0, 1.0, size=(n, prob.d))


def test_partition_of_unity_sums(prob):
    X = random_points(prob)
    sums = geo.window_sum(prob, X)
    tot = np.zeros(X.shape[0])
    tg = np.zeros((X.shape[0], prob.d))
    th = np.zeros((X.shape[0], prob.d))
    scale_g = np.zeros_like(tg)
    scale_h = np.zeros_like(th)
    for j in range(prob.J):
        om, g, h = geo.partition_of_unity(prob, X, j, sums)
        tot += om
        tg += g
        th += h
        scale_g += np.abs(g)
        scale_h += np.abs(h)
    assert np.max(np.abs(tot - 1.0)) < 1e-14
    assert np.max(np.abs(tg) / (scale_g + 1.0)) < 1e-13
    assert np.max(np.abs(th) / (scale_h + 1.0)) < 1e-11


def test_window_peak_value(prob):
    for j in [0, prob.J - 1]:
        c = geo.centre(prob, j)[None, :]
        w, g, h = geo.window_raw(c, c[0], prob.sigma)
        assert abs(w[0] - 4.0 ** prob.d) < 1e-12
        assert np.max(np.abs(g)) < 1e-12


def test_window_fourth_order_zero_at_edge():
    # 1D: (1 + cos(pi (1 - e)))^2 = (1 - cos(pi e))^2 ~ pi^4 e^4 / 4
    sigma = np.array([0.3])
    for e in [1e-2, 3e-3, 1e-3]:
        x = np.array([[sigma[0] * (1.0 - e)]])
        w, _, _ = geo.window_raw(x, np.array([0.0]), sigma)
        assert abs(w[0] / (math.pi ** 4 * e ** 4 / 4.0) - 1.0) < 2.0 * e


def test_window_zero_outside_support():
    sigma = np.array([0.2, 0.1])
    X = np.array([[0.2, 0.0], [0.0, 0.1], [0.25, 0.05], [0.199999, 0.09999]])
    w, g, h = geo.window_raw(X, np.zeros(2), sigma)
    assert np.all(w[:3] == 0.0) and np.all(g[:3] == 0.0) and np.all(h[:3] == 0.0)
    assert w[3] > 0.0


def test_pu_derivatives_match_finite_differences(prob):
    X = random_points(prob, n=60, seed=1)
    hstep = 1e-4 * float(np.min(prob.sigma))
    for j in range(0, prob.J, max(1, prob.J // 4)):
        om, g, h = geo.partition_of_unity(prob, X, j)
        inside = geo.member_mask(X, geo.centre(prob, j), prob.sigma * (1 - 1e-3))
        for i in range(prob.d):
            e = np.zeros(prob.d)
            e[i] = hstep
            vals = [geo.partition_of_unity(prob, X + s * e, j)[0] for s in (-2, -1, 1, 2)]
            fd1 = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * hstep)
            fd2 = (-vals[0] + 16 * vals[1] - 30 * om + 16 * vals[2] - vals[3]) / (12 * hstep ** 2)
            sc1 = np.max(np.abs(g[inside, i])) + 1.0
            sc2 = np.max(np.abs(h[inside, i])) + 1.0
            assert np.max(np.abs(fd1 - g[:, i])[inside]) < 1e-6 * sc1
            assert np.max(np.abs(fd2 - h[:, i])[inside]) < 1e-4 * sc2


def test_support_rows_brute_force(prob):
    X = geo.all_points(prob)
    S = geo.support_rows(prob, X)
    for j in range(0, prob.J, max(1, prob.J // 5)):
        c = geo.centre(prob, j)
        brute = [r for r in range(X.shape[0])
                 if all(abs(X[r, i] - c[i]) < prob.sigma[i] * (1.0 - 1e-12) for i in range(prob.d))]
        assert list(S[j]) == brute


def test_every_point_covered(prob):
    X = geo.all_points(prob)
    S = geo.support_rows(prob, X)
    covered = np.zeros(X.shape[0], dtype=int)
    for rows in S:
        covered[rows] += 1
    assert covered.min() >= 1
