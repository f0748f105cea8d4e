"""Pins of the oracle's PCA, least-squares, Schwarz and Krylov parts against
library routines, identities, special cases and the values the paper prints
(tests/golden/paper_values.json)."""
import json
import os

import numpy as np
import pytest

from oracle import assemble as asm
from oracle import blocksparse as bs
from oracle import geometry as geo
from oracle import krylov as kr
from oracle import lsq
from oracle import pca as pc
from oracle import schwarz as sw
from oracle import solve
from paper_2412_19207_amd import workloads as wl

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.fixture(scope="module")
def small2d():
    prob = wl.small2d()
    ref = solve.reference(prob, "rel_eig", 1e-10)
    return prob, ref


# ------------------------------------------------------------------ PCA (Sec. 4)

def test_pca_eigenvalues_match_gram_eigvalsh():
    prob = wl.small2d()
    X = geo.all_points(prob)
    S = geo.support_rows(prob, X)
    for j in range(prob.J):
        om = geo.partition_of_unity(prob, X[S[j]], j)[0]
        Psi = om[:, None] * np.tanh(((X[S[j]] - geo.centre(prob, j)) / prob.sigma) @ prob.R[j].T + prob.b[j])
        V, lam, tie = pc.pca_basis(Psi, "rel_eig", 1e-10)
        ev = np.sort(np.linalg.eigvalsh(Psi.T @ Psi))[::-1]
        assert np.max(np.abs(ev[:lam.size] - lam)) < 1e-12 * ev[0]
        assert np.allclose(V.T @ V, np.eye(V.shape[1]), atol=1e-13)
        p = V.shape[1]
        assert p == int(np.count_nonzero(ev > 1e-10 * ev[0]))
        # Eckart-Young: the truncation error equals the discarded spectrum
        resid = np.linalg.norm(Psi - Psi @ V @ V.T) ** 2
        assert abs(resid - lam[p:].sum()) <= 1e-10 * lam[0]


def test_pca_modes():
    rng = np.random.default_rng(0)
    Psi = rng.standard_normal((40, 12)) @ np.diag(10.0 ** -np.arange(12))
    V, lam, _ = pc.pca_basis(Psi, "abs_sigma", 1e-5)
    assert V.shape[1] == int(np.count_nonzero(np.sqrt(lam) > 1e-5))
    V, lam, _ = pc.pca_basis(Psi, "off", 0)
    assert np.array_equal(V, np.eye(12))


# ------------------------------------------------------------------ least squares

def test_householder_qr_matches_lstsq():
    rng = np.random.default_rng(1)
    for (n, p) in [(30, 30), (80, 23), (200, 61)]:
        A = rng.standard_normal((n, p)) @ np.diag(np.logspace(0, -6, p))
        B = rng.standard_normal((n, 3))
        qr = lsq.QRSolver(A)
        X = qr.solve(B)
        Xr = np.linalg.lstsq(A, B, rcond=None)[0]
        assert np.linalg.norm(X - Xr) / np.linalg.norm(Xr) < 1e-8
        # Q^T Q = I through the reflectors
        Q = lsq.apply_q(qr.refl, np.eye(n)[:, :p])
        assert np.allclose(Q.T @ Q, np.eye(p), atol=1e-13)
        assert np.allclose(Q @ qr.R, A, atol=1e-12 * np.abs(A).max())


def test_rank_detection():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((50, 10))
    A[:, 7] = A[:, 2]
    assert lsq.QRSolver(A).rank == 9


def test_in_span_manufactured_solution(small2d):
    prob, ref = small2d
    H = ref["H"]
    rng = np.random.default_rng(5)
    w_star = rng.standard_normal((H.shape[1], 2))
    W = ref["qr"].solve(H @ w_star)
    kappa = ref["qr"].cond_estimate()
    assert np.linalg.norm(W - w_star) / np.linalg.norm(w_star) < 100 * kappa * np.finfo(float).eps


def test_single_subdomain_is_plain_elm():
    """J = 1: the window is identically one, so H is the plain ELM matrix
    E_ik = A[phi_k](x_i) of eq. (ls1) and the solution is the ordinary least-squares one."""
    prob = wl.small2d(l=(1, 1), m=(37,), pts=(13, 11))
    sysm = asm.assemble(prob, "off", 0.0)
    X = geo.all_points(prob)
    mu, sig = geo.centre(prob, 0), prob.sigma
    R, b = prob.R[0], prob.b[0]
    t = np.tanh(((X - mu) / sig) @ R.T + b)
    s = 1 - t * t
    E = np.empty_like(t)
    I = slice(0, prob.N_I)
    lap = np.zeros((prob.N_I, R.shape[0]))
    grad = [np.zeros_like(lap) for _ in range(2)]
    for i in range(2):
        r = R[:, i] / sig[i]
        grad[i] = s[I] * r
        lap += -2 * t[I] * s[I] * r * r
    E[I] = (-(prob.a[:, 0:1] * lap) + prob.beta[:, 0:1] * grad[0] + prob.beta[:, 1:2] * grad[1]
            + prob.c[:, None] * t[I])
    E[prob.N_I:] = prob.lambda_B * t[prob.N_I:]
    assert np.allclose(sysm.blocks[0], E, rtol=1e-12, atol=1e-12 * np.abs(E).max())
    W = lsq.QRSolver(sysm.dense()).solve(sysm.Fs)
    Wr = np.linalg.lstsq(E, sysm.Fs, rcond=None)[0]
    assert np.linalg.norm(W - Wr) / np.linalg.norm(Wr) < 1e-7


def test_adjoint_matches_normal_equations_and_fd(small2d):
    prob, ref = small2d
    H, qr = ref["H"], ref["qr"]
    rng = np.random.default_rng(7)
    dW = rng.standard_normal((H.shape[1], 1))
    dF = qr.adjoint(dW)
    expect = H @ np.linalg.solve(H.T @ H, dW)
    assert np.linalg.norm(dF - expect) / np.linalg.norm(expect) < 1e-6
    # misfit L(F) = ||Pm W(F) - u||^2 is quadratic in F: central differences are exact up to rounding
    Pm = asm.probe_matrix(prob, ref["sys"], prob.probes)
    F0 = ref["sys"].Fs[:, :1]
    u = prob.u_probe[:, None]

    def loss(F):
        return float(np.sum((Pm @ qr.solve(F) - u) ** 2))

    grad = qr.adjoint(solve.misfit_seed(Pm, qr.solve(F0), u))
    for q in range(3):
        dirn = rng.standard_normal(F0.shape)
        h = 1e-3
        fd = (loss(F0 + h * dirn) - loss(F0 - h * dirn)) / (2 * h)
        ad = float(np.sum(grad * dirn))
        assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_block_sparse_transpose_dot_product(small2d):
    prob, ref = small2d
    bh = bs.BlockH(ref["sys"])
    rng = np.random.default_rng(11)
    x = rng.standard_normal((bh.P, 3))
    y = rng.standard_normal((bh.N, 3))
    lhs = np.sum(bh.matvec(x) * y)
    rhs = np.sum(x * bh.rmatvec(y))
    assert abs(lhs - rhs) <= 1e-14 * np.linalg.norm(bh.matvec(x)) * np.linalg.norm(y) * 10
    assert np.allclose(bh.matvec(x), ref["H"] @ x, atol=1e-12 * np.abs(ref["H"]).max())


# ------------------------------------------------------------------ Schwarz (Sec. 3)

@pytest.fixture(scope="module")
def dense_small2d(small2d):
    prob, ref = small2d
    H = ref["H"]
    return prob, ref, H.T @ H


@pytest.mark.parametrize("stencil", ["self", "face", "full"])
def test_as_symmetric_positive_definite_and_trace(dense_small2d, stencil):
    prob, ref, HtH = dense_small2d
    sten = sw.stencil(prob, stencil)
    M = sw.schwarz_dense(HtH, ref["sys"].col_off, sten, "as").dense()
    assert np.allclose(M, M.T, atol=1e-9 * np.abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0
    T = M @ HtH
    q_sum = sum(len(sw.block_columns(ref["sys"].col_off, s)) for s in sten)
    assert abs(np.trace(T) - q_sum) < 1e-6 * q_sum
    # self-adjoint in the H^T H inner product: H^T H M H^T H symmetric
    S = HtH @ T
    assert np.allclose(S, S.T, atol=1e-6 * np.abs(S).max())


@pytest.mark.parametrize("kind", ["ras", "sas"])
def test_restricted_weights_partition_identity(dense_small2d, kind):
    prob, ref, HtH = dense_small2d
    sten = sw.stencil(prob, "full")
    M = sw.schwarz_dense(HtH, ref["sys"].col_off, sten, kind)
    P = ref["sys"].P
    acc = np.zeros(P)
    for ix, w in zip(M.idx, M.weights):
        acc[ix] += w
    assert np.allclose(acc, 1.0, atol=1e-15)


def test_self_stencil_ras_equals_as(dense_small2d):
    prob, ref, HtH = dense_small2d
    sten = sw.stencil(prob, "self")
    Ma = sw.schwarz_dense(HtH, ref["sys"].col_off, sten, "as").dense()
    Mr = sw.schwarz_dense(HtH, ref["sys"].col_off, sten, "ras").dense()
    assert np.allclose(Ma, Mr, atol=1e-12 * np.abs(Ma).max())


def test_local_cholesky_and_qr_agree(dense_small2d):
    prob, ref, HtH = dense_small2d
    sten = sw.stencil(prob, "self")
    Mc = sw.schwarz_dense(HtH, ref["sys"].col_off, sten, "as", "chol").dense()
    Mq = sw.schwarz_dense(HtH, ref["sys"].col_off, sten, "as", "qr").dense()
    assert np.linalg.norm(Mc - Mq) / np.linalg.norm(Mq) < 1e-5


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_two_subdomains_per_dim_full_stencil_is_exact(which):
    """Every block is the whole system: M^{-1} H^T H = J I and one CG iteration."""
    if which == "2d":
        prob = wl.small2d(l=(2, 2), m=(30, 25, 28, 33), pts=(8, 7))
    else:
        prob = wl.small3d(pts=(4, 4, 3))
    ref = solve.reference(prob, "rel_eig", 1e-10)
    H = ref["H"]
    HtH = H.T @ H
    sten = sw.stencil(prob, "full")
    assert all(len(s) == prob.J for s in sten)
    M = sw.schwarz_dense(HtH, ref["sys"].col_off, sten, "as")
    T = M.dense() @ HtH
    ev = np.linalg.eigvals(T).real
    kappa = ev.max() / ev.min()
    assert abs(kappa - GOLDEN["as_full_stencil_two_per_dim_kappa"]["value"]) < 1e-4
    assert np.allclose(T, prob.J * np.eye(T.shape[0]), atol=1e-4 * prob.J)
    it = solve.iterative(prob, ref["sys"], "full", "as", "cg", tol=1e-8)
    assert int(it["iters"].max()) == GOLDEN["as_full_stencil_two_per_dim_iterations"]["value"]


def test_as_lambda_max_bound_2d_paper_layout():
    prob = wl.ex1_replica(l=4, m=16, pts=40, delta=2.0)
    sysm = asm.assemble(prob, "off", 0.0)
    H = sysm.dense()
    HtH = H.T @ H
    M = sw.schwarz_dense(HtH, sysm.col_off, sw.stencil(prob, "full"), "as").dense()
    ev = np.linalg.eigvals(M @ HtH).real
    assert ev.max() <= GOLDEN["as_lambda_max_bound_2d"]["value"] * (1 + 1e-6)
    # mean eigenvalue = mean block multiplicity (trace identity)
    assert abs(ev.mean() - 6.25) < 1e-3


def test_as_lambda_max_bound_3d():
    prob = wl.small3d(l=(3, 3, 3), m=12, pts=(4, 4, 4), overlap_frac=0.3)
    sysm = asm.assemble(prob, "rel_eig", 1e-12)
    H = sysm.dense()
    HtH = H.T @ H
    M = sw.schwarz_dense(HtH, sysm.col_off, sw.stencil(prob, "full"), "as").dense()
    ev = np.linalg.eigvals(M @ HtH).real
    assert ev.max() <= GOLDEN["as_lambda_max_bound_3d"]["value"] * (1 + 1e-6)


# ------------------------------------------------------------------ Krylov

@pytest.mark.parametrize("stencil", ["face", "full"])
def test_pcg_reaches_qr_solution(small2d, stencil):
    prob, ref = small2d
    it = solve.iterative(prob, ref["sys"], stencil, "as", "cg", tol=1e-12, maxiter=3000)
    assert np.all(it["res"] <= 1e-12)
    err = np.linalg.norm(it["W"] - ref["W"]) / np.linalg.norm(ref["W"])
    assert err < 1e-8


@pytest.mark.parametrize("kind", ["ras", "sas", "as"])
def test_gmres_reaches_qr_solution(small2d, kind):
    prob, ref = small2d
    it = solve.iterative(prob, ref["sys"], "full", kind, "gmres", tol=1e-12, maxiter=2000)
    err = np.linalg.norm(it["W"] - ref["W"]) / np.linalg.norm(ref["W"])
    assert err < 1e-5
    assert np.all(it["res"] < 1e-8)


@pytest.mark.parametrize("kind", ["ras", "sas", "as"])
def test_right_preconditioned_gmres_reaches_qr_solution(small2d, kind):
    prob, ref = small2d
    it = solve.iterative(prob, ref["sys"], "full", kind, "gmres_right", tol=1e-12, maxiter=2000)
    err = np.linalg.norm(it["W"] - ref["W"]) / np.linalg.norm(ref["W"])
    assert err < 1e-5
    assert np.all(it["res"] < 1e-8)


def test_right_preconditioned_gmres_residual_is_the_true_one_and_monotone(small2d):
    """Right preconditioning minimises ||b - A x|| over the Krylov space of A M:
    within one cycle the recorded residuals never increase, and the last one
    equals the recomputed true residual of the returned x."""
    prob, ref = small2d
    from oracle import blocksparse as bs, krylov as kr, schwarz as sw
    bh = bs.BlockH(ref["sys"])
    M = sw.schwarz_blocks(bh, sw.stencil(prob, "face"), kind="ras", local="chol")
    b = bh.rmatvec(ref["sys"].Fs)[:, 0]
    x, its, hist = kr.gmres(bh.normal, M.apply, b, restart=400, tol=1e-6, maxiter=400, side="right")
    assert 1 < its < 400                    # one cycle, stopped by the tolerance
    assert np.all(np.diff(hist) <= 0.0)
    true = np.linalg.norm(b - bh.normal(x.reshape(-1, 1)).ravel()) / np.linalg.norm(b)
    assert true <= 1e-6
    assert abs(true - hist[-1]) <= 1e-3 * hist[-1]


def test_ex1_replica_statistics_match_paper_order_of_magnitude():
    """Paper Table 1a/1b (4x4 subdomains, m=16, delta=2, 40x40 points, no PCA):
    AS-CG 8 iterations, AS-GMRES 13 iterations, e_L2 6.44e-3, averaged over 10 draws.
    The replica uses 3 draws; it must land within a factor of 4 of the iteration
    counts and a factor of 10 of the error."""
    its_cg, its_gm, errs = [], [], []
    for seed in range(3):
        prob = wl.ex1_replica(seed=seed)
        sysm = asm.assemble(prob, "off", 0.0)
        cg = solve.iterative(prob, sysm, "full", "as", "cg", tol=1e-5)
        gm = solve.iterative(prob, sysm, "full", "as", "gmres", tol=1e-5)
        Pm = asm.probe_matrix(prob, sysm, prob.probes, Lq=prob.L_probe)
        u = (Pm @ gm["W"])[:, 0]
        its_cg.append(cg["iters"][0])
        its_gm.append(gm["iters"][0])
        errs.append(np.linalg.norm(u - prob.u_probe) / np.linalg.norm(prob.u_probe))
    g = GOLDEN
    assert g["ex1_replica_as_cg_iterations"]["value"] / 4 <= np.mean(its_cg) <= 4 * g["ex1_replica_as_cg_iterations"]["value"]
    assert g["ex1_replica_as_gmres_iterations"]["value"] / 4 <= np.mean(its_gm) <= 4 * g["ex1_replica_as_gmres_iterations"]["value"]
    assert g["ex1_replica_as_gmres_eL2"]["value"] / 10 <= np.mean(errs) <= 10 * g["ex1_replica_as_gmres_eL2"]["value"]


def test_ex1_replica_restricted_and_scaled_schwarz_match_paper_order_of_magnitude():
    """Tables 1a/1b with the SAS and RAS preconditioners (GMRES, CGS, BiCG):
    the mean iteration counts over 3 draws land within a factor of 4 of the
    paper's, and the real parts of the RAS-preconditioned spectrum stay below
    twice the paper's largest (2.1).  Pins the RAS ownership reading: owning the
    centre subdomain of each block instead needs 300 to 2000 GMRES iterations
    here (Table 1a: 31)."""
    g = GOLDEN
    its = {}
    re_max = []
    for seed in range(3):
        prob = wl.ex1_replica(seed=seed)
        sysm = asm.assemble(prob, "off", 0.0)
        for kind in ["sas", "ras"]:
            for method in ["gmres", "cgs", "bicg"]:
                r = solve.iterative(prob, sysm, "full", kind, method, tol=1e-5, maxiter=2000)
                its.setdefault(f"{kind}_{method}", []).append(int(r["iters"][0]))
        if seed == 0:
            H = sysm.dense()
            HtH = H.T @ H
            M = sw.schwarz_dense(HtH, sysm.col_off, sw.stencil(prob, "full"), "ras").dense()
            re_max.append(np.linalg.eigvals(M @ HtH).real.max())
    for key, vals in its.items():
        paper = g[f"ex1_replica_{key}_iterations"]["value"]
        assert paper / 4 <= np.mean(vals) <= 4 * paper, (key, vals, paper)
    assert max(re_max) <= 2 * g["ex1_replica_ras_real_part_range"]["value"][1]


@pytest.mark.parametrize("tol,bound", [(1e-10, 3e-2), (1e-14, 1e-4)])
def test_manufactured_accuracy_1d(tol, bound):
    """-u'' = f with u = sin(2 pi x) + 0.1 sin(20 pi x): the least-squares solution
    must reproduce u on a fine grid (a sign error or dropped term in any row
    gives an O(1) error)."""
    prob = wl.cfg1()
    ref = solve.reference(prob, "rel_eig", tol)
    u = asm.probe_matrix(prob, ref["sys"], prob.probes) @ ref["W"]
    err = np.linalg.norm(u[:, 0] - prob.u_probe) / np.linalg.norm(prob.u_probe)
    assert err < bound


# ---------------------------------------------------------------- CGS and BiCG
def _small_normal_system(kind):
    prob = wl.small2d(k=1)
    sysm = asm.assemble(prob, "rel_eig", 1e-10)
    bh = bs.BlockH(sysm)
    M = sw.schwarz_blocks(bh, sw.stencil(prob, "full"), kind=kind)
    b = bh.rmatvec(sysm.Fs)[:, 0]
    return prob, sysm, bh, M, b


@pytest.mark.parametrize("kind", ["as", "sas", "ras"])
@pytest.mark.parametrize("method", ["cgs", "bicg"])
def test_cgs_and_bicg_reach_the_qr_solution(kind, method):
    """Table 1b's CG variants with the AS, SAS and RAS preconditioners reach the
    exact least-squares solution (the QR solution of the oracle)."""
    prob, sysm, bh, M, b = _small_normal_system(kind)
    ref = solve.reference(prob, "rel_eig", 1e-10, sysm=sysm)
    if method == "cgs":
        x, it, _ = kr.cgs(bh.normal, M.apply, b, tol=1e-13, maxiter=3000)
    else:
        x, it, _ = kr.bicg(bh.normal, M.apply, M.apply_T, b, tol=1e-13, maxiter=3000)
    err = np.linalg.norm(x - ref["W"][:, 0]) / np.linalg.norm(ref["W"][:, 0])
    assert err <= 1e-7, (method, kind, it, err)


def test_transposed_schwarz_apply_is_the_transpose():
    """<M^{-1} u, v> = <u, M^{-T} v> for SAS and RAS (and M^{-T} = M^{-1} for AS)."""
    rng = np.random.default_rng(3)
    for kind in ["as", "sas", "ras"]:
        _, _, _, M, b = _small_normal_system(kind)
        u, v = rng.standard_normal(b.size), rng.standard_normal(b.size)
        lhs = M.apply(u[:, None])[:, 0] @ v
        rhs = u @ M.apply_T(v[:, None])[:, 0]
        assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + 1.0), kind
    _, _, _, M, b = _small_normal_system("as")
    u = rng.standard_normal((b.size, 2))
    assert np.allclose(M.apply(u), M.apply_T(u), rtol=0, atol=1e-12 * np.abs(M.apply(u)).max())


def test_bicg_with_symmetric_operator_and_preconditioner_is_pcg():
    """With A = H^T H and the symmetric AS preconditioner, BiCG's shadow sequence
    equals its primal one and its iterates are those of preconditioned CG."""
    _, _, bh, M, b = _small_normal_system("as")
    for k in range(1, 6):
        xb, itb, _ = kr.bicg(bh.normal, M.apply, M.apply_T, b, tol=1e-300, maxiter=k)
        xc, itc, _ = kr.pcg(bh.normal, M.apply, b, tol=1e-300, maxiter=k)
        assert itb == k and int(itc[0]) == k
        assert np.linalg.norm(xb - xc[:, 0]) <= 1e-9 * np.linalg.norm(xc[:, 0]), k


def test_cgs_residual_is_the_squared_cg_polynomial():
    """Sonneveld's identity: with the shadow M^{-1} r_0 and symmetric A, M, the
    CGS residual after k steps is phi_k(A M^{-1})^2 r_0, where phi_k is the
    residual polynomial of preconditioned CG (its coefficients from a plain CG
    run, the polynomial built with numpy.polynomial)."""
    from numpy.polynomial import polynomial as npoly
    _, _, bh, M, b = _small_normal_system("as")
    A = lambda v: bh.normal(v[:, None])[:, 0]
    Mi = lambda v: M.apply(v[:, None])[:, 0]
    B = lambda v: A(Mi(v))
    # plain PCG from x0 = 0: r_{j+1} = r_j - a_j A p_j, p_{j+1} = z_{j+1} + c_j p_j
    r = b.copy()
    z = Mi(r)
    pdir = z.copy()
    phi = np.array([1.0])      # r_j = phi_j(B) r_0
    psi = np.array([0.0, 1.0])  # A p_j = psi_j(B) r_0
    for k in range(1, 5):
        Ap = A(pdir)
        a = (r @ z) / (pdir @ Ap)
        r_new = r - a * Ap
        z_new = Mi(r_new)
        c = (r_new @ z_new) / (r @ z)
        phi = npoly.polysub(phi, a * psi)
        psi = npoly.polyadd(npoly.polymulx(phi), c * psi)
        pdir = z_new + c * pdir
        r, z = r_new, z_new
        # phi_k(B)^2 r_0 by Horner's rule in B
        coef = npoly.polymul(phi, phi)
        v = coef[-1] * b
        for cf in coef[-2::-1]:
            v = B(v) + cf * b
        x, it, _ = kr.cgs(bh.normal, M.apply, b, tol=1e-300, maxiter=k, shadow="Mr")
        r_cgs = b - A(x)
        assert it == k
        assert np.linalg.norm(r_cgs - v) <= 1e-6 * np.linalg.norm(b), (k, np.linalg.norm(r_cgs - v))


def _moment_polynomial(B, r0, s0, k):
    """Residual polynomial of BiCG on the operator B after k steps, from its
    Petrov-Galerkin definition alone: r_k = phi_k(B) r_0 with phi_k(0) = 1 and
    r_k orthogonal to span{s0, B^T s0, ..., (B^T)^{k-1} s0}.  In the monomial
    basis this is the k x k moment system sum_j c_j s0.B^{i+j+1} r0 = s0.B^i r0."""
    K = [r0]
    for _ in range(2 * k):
        K.append(B(K[-1]))
    mom = np.array([s0 @ v for v in K])
    G = np.array([[mom[i + j + 1] for j in range(k)] for i in range(k)])
    c = np.linalg.solve(G, mom[:k])
    return np.concatenate([[1.0], -c])


def _poly_apply(B, coef, v):
    out = coef[-1] * v
    for cf in coef[-2::-1]:
        out = B(out) + cf * v
    return out


@pytest.mark.parametrize("kind", ["sas", "ras"])
def test_bicg_and_cgs_residuals_match_the_petrov_galerkin_polynomial(kind):
    """With a non-symmetric preconditioner (SAS, RAS): BiCG's residual after k
    steps is phi_k(A M^{-1}) r_0, where phi_k is fixed by the Petrov-Galerkin
    condition against the shadow Krylov space K_k((A M^{-1})^T, M^{-T} r_0)
    (the shadow search directions are M^{-T} applied to the shadow residuals);
    CGS with the shadow r_0 has the residual phi_k(A M^{-1})^2 r_0 with the
    polynomial of BiCG on A M^{-1} tested against K_k((A M^{-1})^T, r_0)."""
    prob, sysm, bh, M, b = _small_normal_system(kind)
    A = lambda v: bh.normal(v[:, None])[:, 0]
    Mi = lambda v: M.apply(v[:, None])[:, 0]
    MiT = lambda v: M.apply_T(v[:, None])[:, 0]
    B = lambda v: A(Mi(v))
    nb = np.linalg.norm(b)
    # k <= 3: the monomial moment system loses about three digits per degree
    for k in range(1, 4):
        phi = _moment_polynomial(B, b, MiT(b), k)
        out = solve.iterative(prob, sysm, "full", kind, "bicg", tol=1e-300, maxiter=k)
        assert out["iters"][0] == k
        rb = b - A(out["W"][:, 0])
        assert np.linalg.norm(rb - _poly_apply(B, phi, b)) <= 1e-6 * nb, (kind, k)
        chi = _moment_polynomial(B, b, b, k)
        out = solve.iterative(prob, sysm, "full", kind, "cgs", tol=1e-300, maxiter=k)
        assert out["iters"][0] == k
        rc = b - A(out["W"][:, 0])
        want = _poly_apply(B, np.polynomial.polynomial.polymul(chi, chi), b)
        # CGS may amplify the residual (squared polynomial): relative to it
        scale = max(nb, np.linalg.norm(want))
        assert np.linalg.norm(rc - want) <= 1e-6 * scale, (kind, k, np.linalg.norm(rc - want) / scale)


def test_refined_pcg_reaches_the_qr_solution():
    """AS-PCG restarted from the recomputed normal residual (the full-size
    reference) lands on the QR least-squares solution, and with tol 0 stops at
    the FP64 floor instead of iterating on."""
    prob = wl.small2d(k=2)
    ref = solve.reference(prob, "rel_eig", 1e-10)
    r = solve.refined(prob, ref["sys"], tol=1e-13)
    assert np.all(r["res"] <= 1e-13)
    assert np.linalg.norm(r["W"] - ref["W"]) <= 1e-9 * np.linalg.norm(ref["W"])
    r0 = solve.refined(prob, ref["sys"], tol=0.0, cycles=50)
    assert len(r0["hist"]) < 50 and np.all(r0["res"] <= 1e-12)
