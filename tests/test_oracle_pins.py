"""Pins of oracle functions that the other CPU tests do not reach: the raw-neuron
coefficients, the PCA tie flag, the Cholesky shift branch, the face stencil and
the pseudo-inverse branch of the QR local inverse.  Each pin is a closed form,
a brute-force count or a defining identity, chosen so that a plausible mistake
in the function (a transposed basis, a wrong threshold, a shift in the wrong
scaling, a missing neighbour, a transposed factor) fails it."""
import types

import numpy as np
import pytest

from oracle import assemble as asm
from oracle import blocksparse as bs
from oracle import krylov as kr
from oracle import pca as pc
from oracle import schwarz as sw
from oracle import solve
from paper_2412_19207_amd import workloads as wl


# ------------------------------------------------ raw-neuron coefficients
def _window_direct(prob, X):
    """omega_j(x) for all j, written out from the window of Sec. 5 (Ex. 1):
    prod_i (1 + cos(pi (x_i - mu_ji) / sigma_i))^2 inside the open support box,
    normalised by the sum over all subdomains."""
    J = prob.J
    W = np.zeros((X.shape[0], J))
    for j in range(J):
        mu = prob.centre(j)
        t = (X - mu[None, :]) / prob.sigma[None, :]
        inside = np.all(np.abs(t) < 1.0 - 1e-12, axis=1)
        W[:, j] = np.where(inside, np.prod((1.0 + np.cos(np.pi * t)) ** 2, axis=1), 0.0)
    return W / W.sum(axis=1, keepdims=True)


def test_coeffs_evaluate_the_raw_network():
    """u_h(x) = sum_j omega_j(x) sum_k c_jk tanh(R_jk . (x - mu_j)/sigma + b_jk)
    (eq. (netdd) with the raw network) must equal the probe rows in the PCA
    basis times W (eq. (pca_net)): pins c = blockdiag(V_{p_j}) W."""
    prob = wl.small2d(k=2)
    ref = solve.reference(prob, "rel_eig", 1e-10)
    sysm, W = ref["sys"], ref["W"]
    assert np.any(sysm.p < prob.m), "the truncation must be active for this pin"
    c = sysm.coeffs(W)
    X = prob.probes
    om = _window_direct(prob, X)
    u_direct = np.zeros((X.shape[0], W.shape[1]))
    off = 0
    for j in range(prob.J):
        mj = int(prob.m[j])
        z = ((X - prob.centre(j)[None, :]) / prob.sigma[None, :]) @ prob.R[j].T + prob.b[j][None, :]
        u_direct += om[:, j:j + 1] * (np.tanh(z) @ c[off:off + mj])
        off += mj
    assert off == c.shape[0]
    u_basis = asm.probe_matrix(prob, sysm, X) @ W
    scale = np.abs(u_direct).max()
    assert np.abs(u_direct - u_basis).max() <= 1e-11 * scale


def test_coeffs_are_invariant_to_a_rotation_of_the_basis():
    """Rotating each V_{p_j} by an orthogonal Q_j rotates W by Q_j^T and leaves
    c = V W unchanged (Sec. 4: only the span of V_{p_j} matters)."""
    prob = wl.small2d(k=1)
    ref = solve.reference(prob, "rel_eig", 1e-10)
    rng = np.random.default_rng(5)
    Vr = []
    for Vj in ref["sys"].V:
        Q, _ = np.linalg.qr(rng.standard_normal((Vj.shape[1], Vj.shape[1])))
        Vr.append(Vj @ Q)
    ref2 = solve.reference(prob, "rel_eig", 1e-10, V_force=Vr)
    c1, c2 = ref["c"], ref2["c"]
    assert np.linalg.norm(c1 - c2) <= 1e-8 * np.linalg.norm(c1)
    W1, W2 = ref["W"], ref2["W"]
    assert np.linalg.norm(W1 - W2) > 1e-3 * np.linalg.norm(W1), "the rotation must change W"


# ------------------------------------------------ PCA tie flag (Sec. 4)
def _psi_with_spectrum(s, n=40, seed=3):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, s.size)))
    V, _ = np.linalg.qr(rng.standard_normal((s.size, s.size)))
    return U @ np.diag(s) @ V.T


def test_pca_tie_flag_at_the_threshold():
    s = np.array([2.0, 1.0, 0.5, 1e-3, 1e-5, 1e-7])
    Psi = _psi_with_spectrum(s)
    # relative eigenvalue threshold exactly at lambda_4 = s_4^2
    tol = (s[3] / s[0]) ** 2
    V, lam, tie = pc.pca_basis(Psi, "rel_eig", tol)
    assert tie
    V, lam, tie = pc.pca_basis(Psi, "rel_eig", tol * (1.0 + 1e-3))
    assert not tie and V.shape[1] == 3
    V, lam, tie = pc.pca_basis(Psi, "rel_eig", tol * (1.0 - 1e-3))
    assert not tie and V.shape[1] == 4
    # the paper's absolute threshold on sigma, exactly at s_5
    V, lam, tie = pc.pca_basis(Psi, "abs_sigma", s[4])
    assert tie
    V, lam, tie = pc.pca_basis(Psi, "abs_sigma", s[4] * 1.01)
    assert not tie and V.shape[1] == 4
    V, lam, tie = pc.pca_basis(Psi, "abs_sigma", s[4] * 0.99)
    assert not tie and V.shape[1] == 5


# ------------------------------------------------ Cholesky shift branch (Sec. 3)
def test_cholesky_shift_on_an_exactly_singular_block():
    """A Gram block with a zero column (a dead neuron) is singular: the first
    factorisation hits an exact zero pivot, one shift eps = 10 u q is taken, and
    the solve is the closed form of the shifted equilibrated system."""
    rng = np.random.default_rng(11)
    B = rng.standard_normal((30, 7)) * np.array([1.0, 10.0, 0.1, 3.0, 1e2, 1.0, 0.5])
    B = np.concatenate([B[:, :3], np.zeros((30, 1)), B[:, 3:]], axis=1)   # column 3 is dead
    A = B.T @ B
    q = A.shape[0]
    solve_fn, shifts = sw.chol_local(A)
    assert shifts == 1
    eps = 10.0 * np.finfo(float).eps * q
    r = rng.standard_normal(q)
    z = solve_fn(r)[:, 0]
    # the dead column: D = 1 there and D A D + eps I is eps on the diagonal
    assert abs(z[3] - r[3] / eps) <= 1e-12 * abs(r[3] / eps)
    # the rest: D' (D' A' D' + eps I)^{-1} D' r' with D' = diag(A')^{-1/2}
    live = np.array([0, 1, 2, 4, 5, 6, 7])
    Al = A[np.ix_(live, live)]
    Dl = 1.0 / np.sqrt(np.diag(Al))
    zl = Dl * np.linalg.solve(Dl[:, None] * Al * Dl[None, :] + eps * np.eye(live.size), Dl * r[live])
    assert np.linalg.norm(z[live] - zl) <= 1e-10 * np.linalg.norm(zl)


def test_cholesky_shift_leaves_the_pcg_solution_unchanged():
    """A dead neuron (zero weights and bias: tanh 0 = 0) makes H and every local
    block containing it singular; PCA off keeps the zero column.  The shifted
    local factors only change the preconditioner: PCG still reaches the
    least-squares fit H W of the live columns."""
    prob = wl.small2d(k=1)
    prob.R[2][5] = 0.0
    prob.b[2][5] = 0.0
    sysm = asm.assemble(prob, "off", 0.0)
    bh = bs.BlockH(sysm)
    M = sw.schwarz_blocks(bh, sw.stencil(prob, "full"), kind="as")
    assert M.shifts >= 1
    rhs = bh.rmatvec(sysm.Fs)
    W, iters, _ = kr.pcg(bh.normal, M.apply, rhs, tol=1e-12, maxiter=4000,
                         true_res=lambda X: solve.normal_residual(bh, X, sysm.Fs))
    H = sysm.dense()
    live = np.abs(H).sum(axis=0) > 0
    assert np.count_nonzero(~live) == 1
    Wl, *_ = np.linalg.lstsq(H[:, live], sysm.Fs, rcond=None)
    fit_ref = H[:, live] @ Wl
    fit = H @ W
    assert np.linalg.norm(fit - fit_ref) <= 1e-7 * np.linalg.norm(fit_ref)


# ------------------------------------------------ face stencil
def _layout(l):
    d = len(l)
    mu = [(np.arange(n) + 0.5) / n for n in l]
    return types.SimpleNamespace(d=d, l=np.array(l), J=int(np.prod(l)), mu=mu,
                                 sigma=np.array([0.6 / n for n in l]))


@pytest.mark.parametrize("l", [(5, 4), (4, 3, 3), (1, 6)])
def test_face_stencil_brute_force(l):
    """face(i) = i plus the subdomains whose centre is one centre spacing away
    along exactly one axis, found here from the centres alone."""
    lay = _layout(l)
    sten = sw.stencil(lay, "face")
    cen = np.array([np.array([lay.mu[q][(j // int(np.prod(l[:q]))) % l[q]] for q in range(lay.d)])
                    for j in range(lay.J)])
    spacing = np.array([1.0 / n for n in l])
    for i in range(lay.J):
        steps = np.abs(cen - cen[i][None, :]) / spacing[None, :]
        one_step = np.isclose(steps, 1.0)
        same = np.isclose(steps, 0.0)
        nb = [j for j in range(lay.J)
              if j == i or (one_step[j].sum() == 1 and (one_step[j] | same[j]).all())]
        assert sorted(sten[i].tolist()) == nb
    # the counts: 1 + (number of axes with a neighbour on each side)
    interior = [i for i in range(lay.J) if all(0 < (i // int(np.prod(l[:q]))) % l[q] < l[q] - 1
                                               for q in range(lay.d) if l[q] > 1)]
    for i in interior:
        assert len(sten[i]) == 1 + 2 * sum(1 for n in l if n > 1)


# ------------------------------------------------ QR local inverse, singular branch
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_qr_local_pseudo_inverse_on_a_singular_block(seed):
    """A rank-deficient symmetric block: the branch must return the
    Moore-Penrose inverse, checked by its four defining conditions."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((9, 5)) * np.array([1.0, 3.0, 0.3, 2.0, 1.0])
    A = B @ B.T
    solve_fn, singular = sw.qr_local(A)
    assert singular == 1
    X = solve_fn(np.eye(9))
    nA = np.linalg.norm(A)
    nX = np.linalg.norm(X)
    assert np.linalg.norm(A @ X @ A - A) <= 1e-10 * nA
    assert np.linalg.norm(X @ A @ X - X) <= 1e-10 * nX
    assert np.linalg.norm(A @ X - (A @ X).T) <= 1e-10
    assert np.linalg.norm(X @ A - (X @ A).T) <= 1e-10


def test_qr_local_regular_block_is_the_inverse():
    rng = np.random.default_rng(4)
    B = rng.standard_normal((12, 6))
    A = B.T @ B
    solve_fn, singular = sw.qr_local(A)
    assert singular == 0
    assert np.linalg.norm(solve_fn(np.eye(6)) @ A - np.eye(6)) <= 1e-11
