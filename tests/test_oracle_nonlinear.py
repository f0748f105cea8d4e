"""Pins of the oracle's Picard and Newton iterations (Sec. 2 remark: each step
of a nonlinear iteration solves one linear least-squares problem).

The nonlinear residual r(W) of the collocation problem is written here from its
definition (operator rows of the linear part, the reaction g on the values,
boundary rows); the oracle's steps are checked against it: a Newton step is the
Gauss-Newton step of ||r||^2 with a finite-difference Jacobian, the Newton
limit makes J^T r vanish, the Picard limit is a fixed point of its own
linearisation, and the operator rows are affine in the reaction coefficient
with the value rows as slope."""
import dataclasses

import numpy as np
import pytest

from oracle import assemble as asm
from oracle import lsq
from oracle import nonlinear as nl
from paper_2412_19207_amd import workloads as wl


@pytest.fixture(scope="module")
def semi():
    prob = wl.semilinear2d("small")
    gamma = prob.meta["gamma"]
    sys0 = asm.assemble(prob, "rel_eig", prob.meta["pca_tol"])
    H0 = sys0.dense()
    Pm = asm.probe_matrix(prob, sys0, prob.X_int)
    return prob, gamma, sys0, H0, Pm


def _residual(prob, H0, Pm, Fs, W, gamma):
    u = Pm @ W
    r = H0 @ W - Fs
    r[:prob.N_I] += sum(c * u ** p for p, c in enumerate(gamma))
    return r


def test_rows_are_affine_in_the_reaction_coefficient(semi):
    """H(c) - H(c0) = diag(c - c0) times the value rows on the interior rows and
    zero on the boundary rows: the reaction term enters an operator row as
    c times the basis function's value."""
    prob, gamma, sys0, H0, Pm = semi
    rng = np.random.default_rng(0)
    dc = rng.uniform(0.5, 3.0, prob.N_I)
    pk = dataclasses.replace(prob, c=prob.c + dc)
    H1 = asm.assemble(pk, V_force=sys0.V, p_force=sys0.p).dense()
    D = H1 - H0
    assert np.max(np.abs(D[:prob.N_I] - dc[:, None] * Pm)) <= 1e-12 * np.max(np.abs(H0))
    assert np.max(np.abs(D[prob.N_I:])) == 0.0


def test_g_and_its_derivative():
    u = np.linspace(-2, 3, 11)
    gamma = [0.5, -1.0, 0.25, 2.0]
    assert np.allclose(nl.g_value(u, gamma), 0.5 - u + 0.25 * u ** 2 + 2 * u ** 3, rtol=0, atol=1e-12)
    assert np.allclose(nl.g_prime(u, gamma), -1 + 0.5 * u + 6 * u ** 2, rtol=0, atol=1e-12)


def test_newton_step_is_the_gauss_newton_step_with_a_fd_jacobian(semi):
    """From the first iterate W_1, the oracle's next Newton step equals
    W_1 + argmin ||J d + r(W_1)|| with J from central differences of r."""
    prob, gamma, sys0, H0, Pm = semi
    out = nl.iterate(prob, gamma, "newton", steps=2, pca_tol=prob.meta["pca_tol"],
                     V_force=sys0.V, p_force=sys0.p)
    W1, W2 = out["W"]
    Fs = sys0.Fs[:, 0]
    r1 = _residual(prob, H0, Pm, Fs, W1, gamma)
    h = 1e-6 * max(1.0, np.abs(W1).max())
    J = np.empty((prob.N, W1.size))
    for q in range(W1.size):
        e = np.zeros(W1.size)
        e[q] = h
        J[:, q] = (_residual(prob, H0, Pm, Fs, W1 + e, gamma) - _residual(prob, H0, Pm, Fs, W1 - e, gamma)) / (2 * h)
    d = lsq.QRSolver(J).solve(-r1[:, None])[:, 0]
    err = np.linalg.norm(W1 + d - W2) / np.linalg.norm(W2)
    assert err <= 1e-6, err


def test_newton_limit_is_stationary_and_picard_limit_is_a_fixed_point(semi):
    """Newton (Gauss-Newton) converges to a stationary point of ||r(W)||^2:
    J^T r = 0 with J = H0 + diag(g'(u)) Pm.  Picard converges to a fixed point of
    its own step: H(c*)^T r = 0 with H(c*) = H0 + diag(q(u*)) Pm.  Both limits
    fit the collocation equations to the same order."""
    prob, gamma, sys0, H0, Pm = semi
    Fs = sys0.Fs[:, 0]
    kw = dict(pca_tol=prob.meta["pca_tol"], V_force=sys0.V, p_force=sys0.p)
    nw = nl.iterate(prob, gamma, "newton", steps=12, **kw)
    Wn = nw["W"][-1]
    assert nw["inc"][-1] < 1e-12
    r = _residual(prob, H0, Pm, Fs, Wn, gamma)
    un = Pm @ Wn
    Jn = H0.copy()
    Jn[:prob.N_I] += nl.g_prime(un, gamma)[:, None] * Pm
    scale = np.linalg.norm(Jn, 2) * np.linalg.norm(r)
    assert np.linalg.norm(Jn.T @ r) <= 1e-9 * scale
    pc = nl.iterate(prob, gamma, "picard", steps=60, stop=1e-13, **kw)
    Wp = pc["W"][-1]
    assert pc["inc"][-1] <= 1e-12
    rp = _residual(prob, H0, Pm, Fs, Wp, gamma)
    up = Pm @ Wp
    Hc = H0.copy()
    Hc[:prob.N_I] += nl.g_value(up, gamma[1:])[:, None] * Pm
    assert np.linalg.norm(Hc.T @ rp) <= 1e-9 * np.linalg.norm(Hc, 2) * np.linalg.norm(rp)
    # and Newton's limit is not a Picard fixed point (the two limits differ at
    # the order of the collocation residual), but both fit equally well
    assert abs(np.linalg.norm(rp) - np.linalg.norm(r)) <= 0.05 * np.linalg.norm(r)


@pytest.mark.parametrize("mode", ["newton", "picard"])
def test_affine_reaction_takes_one_step(semi, mode):
    """g(u) = 1.5 + 2u on a problem whose own reaction is c0 = 0.75: the first
    Newton or Picard step is the linear problem with reaction c0 + 2 and
    interior rows f - 1.5 (the oracle's QR solution of that problem), and the
    next increment vanishes."""
    prob, _, sys0, _, _ = semi
    prob = dataclasses.replace(prob, c=np.full(prob.N_I, 0.75))
    gamma = [1.5, 2.0]
    out = nl.iterate(prob, gamma, mode, steps=2, pca_tol=prob.meta["pca_tol"],
                     V_force=sys0.V, p_force=sys0.p)
    F = np.array(prob.F, dtype=float)
    F[:prob.N_I] -= 1.5
    pk = dataclasses.replace(prob, c=prob.c + 2.0, F=F)
    sk = asm.assemble(pk, V_force=sys0.V, p_force=sys0.p)
    Wref = lsq.QRSolver(sk.dense()).solve(sk.Fs)[:, 0]
    assert np.linalg.norm(out["W"][0] - Wref) <= 1e-10 * np.linalg.norm(Wref)
    assert out["inc"][1] <= 1e-10


def test_manufactured_solution_accuracy(semi):
    """Newton on -lap u + u^3 = f reaches the accuracy of the discretisation:
    relative L2 error at the probes below 5e-2 on this small layout."""
    prob, gamma, sys0, _, _ = semi
    out = nl.iterate(prob, gamma, "newton", steps=8, pca_tol=prob.meta["pca_tol"],
                     V_force=sys0.V, p_force=sys0.p)
    U = asm.probe_matrix(prob, out["sys_last"], prob.probes) @ out["W"][-1]
    e = np.linalg.norm(U - prob.u_probe) / np.linalg.norm(prob.u_probe)
    assert e < 5e-2, e
