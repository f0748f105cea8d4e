"""GPU parity of the HIP path against the FP64 oracle, through the C interface.

Sizes span several 64-wide kernel tiles with ragged tails (uneven widths, point
counts that are not multiples of the tile).  Tolerances:
  * integer work (binning, truncation counts): bit-exact
  * entries of H, products, local inverses: 1e-11 relative to the largest entry
    (same FP64 formulas, different summation order)
  * FP64 solve: coefficient error <= 1e-8 relative, mixed <= 1e-6
"""
import numpy as np
import pytest
import torch

from oracle import assemble as oasm
from oracle import blocksparse as obs
from oracle import geometry as ogeo
from oracle import schwarz as osw
from oracle import solve as osolve
from paper_2412_19207_amd import binding
from paper_2412_19207_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    binding.load()


def make(name):
    if name == "ex1":
        return wl.ex1_replica(l=4, m=16, pts=40)
    if name == "small2d_k3":
        return wl.small2d(k=3)
    return wl.make(name)


def vforce(sysm):
    return torch.as_tensor(np.concatenate([v.ravel() for v in sysm.V]), device=DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def case_small2d():
    _need_gpu()
    prob = wl.small2d(k=2)
    ref = osolve.reference(prob, "rel_eig", 1e-10)
    return prob, ref


# ------------------------------------------------------------------ a1 binning
@pytest.mark.parametrize("name", ["small2d", "small3d", "cfg1", "ex1"])
def test_binning_bit_exact(name):
    _need_gpu()
    prob = make(name)
    s = binding.Solver(prob, device=DEV)
    row_off, rows, _ = s.layout()
    S = ogeo.support_rows(prob)
    assert np.array_equal(row_off, np.concatenate([[0], np.cumsum([len(x) for x in S])]))
    assert np.array_equal(rows, np.concatenate(S).astype(np.int32))


# ------------------------------------------------------------------ a3/a4 PCA
@pytest.mark.parametrize("name", ["small2d", "small3d", "cfg1"])
def test_pca_counts_and_spectrum(name):
    _need_gpu()
    prob = make(name)
    tol = prob.meta.get("pca_tol") or 1e-10
    sysm = oasm.assemble(prob, "rel_eig", tol)
    s = binding.Solver(prob, device=DEV)
    p = s.pca(tol, "rel_eig")
    assert np.array_equal(p, sysm.p)
    _, V, eig = s.arrays()
    eig = eig.cpu().numpy()
    V = V.cpu().numpy()
    off = 0
    voff = 0
    for j in range(prob.J):
        m = int(prob.m[j])
        lam = sysm.lam[j]
        lg = eig[off:off + m]
        n = min(lam.size, m)
        # eigenvalues of the FP64 Gram agree within its rounding level
        assert np.max(np.abs(lg[:n] - lam[:n])) <= 10 * m * np.finfo(float).eps * lam[0]
        Vg = V[voff:voff + m * p[j]].reshape(m, p[j])
        assert np.allclose(Vg.T @ Vg, np.eye(p[j]), atol=1e-10)
        # subspace: sin(theta) bounded by u * lambda_1 / gap
        Vo = sysm.V[j]
        gap = lam[p[j] - 1] - (lam[p[j]] if p[j] < lam.size else 0.0)
        bound = 100 * m * np.finfo(float).eps * lam[0] / max(gap, 1e-300)
        sin_t = np.linalg.norm(Vo - Vg @ (Vg.T @ Vo), 2)
        assert sin_t <= max(bound, 1e-10), (j, sin_t, bound)
        off += m
        voff += m * p[j]


# ------------------------------------------------------------------ a2/a5 rows
@pytest.mark.parametrize("name", ["small2d", "small3d", "cfg1", "ex1"])
def test_rows_match_oracle_with_forced_basis(name):
    _need_gpu()
    prob = make(name)
    tol = prob.meta.get("pca_tol") or 1e-10
    sysm = oasm.assemble(prob, "rel_eig", tol)
    s = binding.Solver(prob, device=DEV)
    s.pca(tol, "rel_eig", p_force=sysm.p, V_force=vforce(sysm))
    blocks, _, _ = s.arrays()
    blocks = blocks.cpu().numpy()
    o = 0
    scale = max(np.abs(b).max() for b in sysm.blocks)
    for j in range(prob.J):
        B = sysm.blocks[j]
        G = blocks[o:o + B.size].reshape(B.shape)
        o += B.size
        assert np.max(np.abs(G - B)) <= 1e-11 * scale, j


@pytest.mark.parametrize("name", ["small2d", "small3d"])
def test_rows_with_own_pca_match_oracle_in_gpu_basis(name):
    """Rows built after the library's own PCA (from the tanh values its value
    matrices kept) against the oracle's rows in the library's basis."""
    _need_gpu()
    prob = make(name)
    tol = prob.meta.get("pca_tol") or 1e-10
    s = binding.Solver(prob, device=DEV)
    p = s.pca(tol, "rel_eig")
    blocks, V, _ = s.arrays()
    blocks, V = blocks.cpu().numpy(), V.cpu().numpy()
    Vg, off = [], 0
    for j in range(prob.J):
        m = int(prob.m[j])
        Vg.append(V[off:off + m * p[j]].reshape(m, p[j]))
        off += m * p[j]
    sysg = oasm.assemble(prob, "rel_eig", tol, V_force=Vg)
    scale = max(np.abs(b).max() for b in sysg.blocks)
    o = 0
    for j in range(prob.J):
        B = sysg.blocks[j]
        G = blocks[o:o + B.size].reshape(B.shape)
        o += B.size
        assert np.max(np.abs(G - B)) <= 1e-11 * scale, j


def test_rows_raw_features_without_pca():
    _need_gpu()
    prob = wl.small2d()
    sysm = oasm.assemble(prob, "off", 0.0)
    s = binding.Solver(prob, device=DEV)
    p = s.pca(0.0, "off")
    assert np.array_equal(p, prob.m)
    blocks = s.arrays()[0].cpu().numpy()
    flat = np.concatenate([b.ravel() for b in sysm.blocks])
    assert np.max(np.abs(blocks - flat)) <= 1e-11 * np.abs(flat).max()


# ------------------------------------------------------------------ products
def test_products_match_dense(case_small2d):
    prob, ref = case_small2d
    sysm, H = ref["sys"], ref["H"]
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(0)
    for k in [1, 3, 16, 37]:
        x = rng.standard_normal((sysm.P, k))
        y = rng.standard_normal((sysm.N, k))
        xg, yg = torch.as_tensor(x, device=DEV), torch.as_tensor(y, device=DEV)
        Hx = s.matvec(xg).cpu().numpy()
        HTy = s.rmatvec(yg).cpu().numpy()
        Nx = s.apply_normal(xg).cpu().numpy()
        assert rel(Hx, H @ x) < 1e-13
        assert rel(HTy, H.T @ y) < 1e-13
        assert rel(Nx, H.T @ (H @ x)) < 1e-12


@pytest.mark.parametrize("stencil", ["self", "face", "full"])
@pytest.mark.parametrize("kind", ["as", "ras", "sas"])
def test_preconditioner_matches_oracle(case_small2d, stencil, kind):
    prob, ref = case_small2d
    sysm, H = ref["sys"], ref["H"]
    HtH = H.T @ H
    M = osw.schwarz_dense(HtH, sysm.col_off, osw.stencil(prob, stencil), kind).dense()
    s = binding.Solver(prob, device=DEV, stencil=stencil, precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(1)
    r = rng.standard_normal((sysm.P, 2))
    z = s.apply_precond(torch.as_tensor(r, device=DEV)).cpu().numpy()
    kappa = np.linalg.cond(HtH)
    assert rel(z, M @ r) < max(1e-9, 1e-15 * kappa), (rel(z, M @ r), kappa)


@pytest.fixture(scope="module")
def case_small2d_k37():
    _need_gpu()
    prob = wl.small2d(k=37)
    ref = osolve.reference(prob, "rel_eig", 1e-10)
    return prob, ref


@pytest.mark.parametrize("stencil", ["face", "full"])
@pytest.mark.parametrize("kind", ["as", "ras", "sas"])
@pytest.mark.parametrize("k", [16, 37])
def test_preconditioner_batched_matches_oracle(case_small2d, stencil, kind, k):
    """16 or more right-hand sides run the local solves on the matrix cores
    (chunks of 32 and 16, the rest on the vector path): FP64 to the same bar."""
    prob, ref = case_small2d
    sysm, H = ref["sys"], ref["H"]
    HtH = H.T @ H
    M = osw.schwarz_dense(HtH, sysm.col_off, osw.stencil(prob, stencil), kind).dense()
    s = binding.Solver(prob, device=DEV, stencil=stencil, precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(7)
    r = rng.standard_normal((sysm.P, k))
    z = s.apply_precond(torch.as_tensor(r, device=DEV)).cpu().numpy()
    kappa = np.linalg.cond(HtH)
    ref_z = M @ r
    for t in range(k):
        e = rel(z[:, t], ref_z[:, t])
        assert e < max(1e-9, 1e-15 * kappa), (t, e, kappa)


@pytest.fixture(scope="module")
def case_wide_blocks():
    _need_gpu()
    prob = wl.small2d(l=(4, 3), m=(150, 171, 133, 164, 148, 177), k=2)
    ref = osolve.reference(prob, "rel_eig", 1e-10)
    return prob, ref


@pytest.mark.parametrize("kind", ["as", "ras", "sas"])
@pytest.mark.parametrize("k", [16, 32, 37])
def test_preconditioner_large_blocks_matches_oracle(case_wide_blocks, kind, k):
    """Schwarz blocks of up to 9 tiles per edge (4x3 subdomains, full stencil,
    q up to 563): the FP64 matrix-core local solves that stream the tiles of a
    block one output tile per workgroup (k_rowcol_mfma64), against the
    oracle's dense M^-1 column by column."""
    prob, ref = case_wide_blocks
    sysm, H = ref["sys"], ref["H"]
    HtH = H.T @ H
    M = osw.schwarz_dense(HtH, sysm.col_off, osw.stencil(prob, "full"), kind).dense()
    s = binding.Solver(prob, device=DEV, stencil="full", precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    assert s.info.max_q > 6 * 64
    rng = np.random.default_rng(9)
    r = rng.standard_normal((sysm.P, k))
    z = s.apply_precond(torch.as_tensor(r, device=DEV)).cpu().numpy()
    kappa = np.linalg.cond(HtH)
    ref_z = M @ r
    for t in range(k):
        e = rel(z[:, t], ref_z[:, t])
        assert e < max(1e-9, 1e-15 * kappa), (t, e, kappa)


@pytest.mark.parametrize("k", [16, 32])
def test_solve_wide_block_rows_matches_qr(k):
    """Block rows of about 60 columns and slabs of up to 563 (4x3 subdomains,
    full stencil): the matrix-core normal-matrix product over several column
    sweeps and the local solves of large blocks inside CG, against QR per
    right-hand side."""
    _need_gpu()
    prob = wl.small2d(l=(4, 3), m=(150, 171, 133, 164, 148, 177), k=k)
    ref = osolve.reference(prob, "rel_eig", 1e-10)
    sysm = ref["sys"]
    assert sysm.P / prob.J >= 48
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    # the normal residual's FP64 floor here is about 5e-13 (any k)
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, maxiter=5000)
    assert info["status"] == 0
    Wn = W.cpu().numpy()
    for t in range(k):
        assert rel(Wn[:, t], ref["W"][:, t]) <= 1e-8, t


@pytest.mark.parametrize("kb", [16, 32])
def test_mixed_batched_apply_close_to_fp64(case_small2d, kb):
    """Mixed path against the FP64 oracle apply: one right-hand side at a time
    (FP64 arithmetic on the FP32 factor) and kb at once (FP32 operands and
    accumulation on the matrix cores, one pass with A_i^-1 in FP32).  Both stay
    within 1e-5 relative, about 170 units of FP32 rounding (measured: 2e-8 and
    2.4e-7 to 3.3e-7)."""
    prob, ref = case_small2d
    sysm, H = ref["sys"], ref["H"]
    HtH = H.T @ H
    M = osw.schwarz_dense(HtH, sysm.col_off, osw.stencil(prob, "full"), "as").dense()
    s = binding.Solver(prob, device=DEV, precision="mixed")
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(8)
    r = rng.standard_normal((sysm.P, kb))
    zb = s.apply_precond(torch.as_tensor(r, device=DEV)).cpu().numpy()
    z1 = np.stack([s.apply_precond(torch.as_tensor(r[:, t:t + 1], device=DEV)).cpu().numpy()[:, 0]
                   for t in range(4)], 1)
    ref_z = M @ r
    e1 = max(rel(z1[:, t], ref_z[:, t]) for t in range(4))
    eb = max(rel(zb[:, t], ref_z[:, t]) for t in range(kb))
    print(f"mixed apply vs FP64: one at a time {e1:.2e}, batched FP32 {eb:.2e}")
    assert e1 < 1e-5 and eb < 1e-5, (e1, eb)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_batched_solve_matches_qr(case_small2d_k37, precision, bar):
    """37 right-hand sides in one solve (matrix-core chunks of 32, then 4 + 1)."""
    prob, ref = case_small2d_k37
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precision=precision)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=5000)
    assert info["status"] == 0
    assert info["max_rel_residual"] <= 1e-13
    Wn = W.cpu().numpy()
    for t in range(Wn.shape[1]):
        e = rel(Wn[:, t], ref["W"][:, t])
        assert e <= bar, (t, e)


# ------------------------------------------------------------------ a8/a9 solves
@pytest.mark.parametrize("stencil", ["face", "full"])
def test_fp64_solve_matches_qr(case_small2d, stencil):
    prob, ref = case_small2d
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, stencil=stencil)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, maxiter=3000)
    assert info["status"] == 0
    assert info["max_rel_residual"] <= 1e-12
    err = rel(W.cpu().numpy(), ref["W"])
    assert err <= 1e-8, err
    # iteration counts: the oracle PCG with the same stencil needs about as many
    it = osolve.iterative(prob, sysm, stencil, "as", "cg", tol=1e-12, maxiter=3000)
    assert abs(int(info["iterations"]) - int(it["iters"].max())) <= max(3, 0.2 * it["iters"].max())


def _pca_bound(s, sysm, kappa):
    """Predicted coefficient error of an end-to-end solve with an independent PCA:
    the GPU and oracle bases span subspaces that differ by sin(theta) (eigenvector
    rounding, ~ u lambda_1 / gap), amplified at most by kappa(H)."""
    _, V, _ = s.arrays()
    V = V.cpu().numpy()
    o, worst = 0, 0.0
    for j, Vo in enumerate(sysm.V):
        m, p = Vo.shape
        Vg = V[o:o + m * p].reshape(m, p)
        o += m * p
        worst = max(worst, np.linalg.norm(Vo - Vg @ (Vg.T @ Vo), 2))
    return max(1e-8, 10.0 * kappa * worst), worst


def test_fp64_end_to_end_independent_pca(case_small2d):
    prob, ref = case_small2d
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10)
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=3000)
    c = s.coeffs(W).cpu().numpy()
    U = s.eval(torch.as_tensor(prob.probes, device=DEV), W).cpu().numpy()
    Uref = oasm.probe_matrix(prob, ref["sys"], prob.probes) @ ref["W"]
    bound, sin_t = _pca_bound(s, ref["sys"], ref["qr"].cond_estimate())
    err_c = rel(c, ref["c"])
    print(f"end-to-end: coef err {err_c:.2e} (bound {bound:.2e}, sin theta {sin_t:.2e}), "
          f"u err {rel(U, Uref):.2e}")
    assert err_c <= bound
    assert rel(U, Uref) <= 1e-8


@pytest.mark.parametrize("kind", ["ras", "sas", "as"])
@pytest.mark.parametrize("method", ["gmres", "gmres_right"])
def test_gmres_matches_qr(case_small2d, kind, method):
    prob, ref = case_small2d
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    # 1e-12: the FP64 floor of the true normal residual here is 3e-14 to 1e-13
    # (left-preconditioned SAS stalls at 1e-13); the coefficient error at 1e-12 is
    # about 1e-12 to 4e-10, so the FP64 bar holds with room
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, method=method, restart=50,
                      maxiter=5000)
    assert info["status"] == 0
    assert info["max_rel_residual"] <= 1e-12
    err = rel(W.cpu().numpy(), ref["W"])
    print(f"gmres {method}/{kind}: iterations {info['iterations']}, coefficient error {err:.2e}")
    assert err <= 1e-8, err


# ------------------------------------------------------------------ CGS and BiCG (Table 1b)
@pytest.mark.parametrize("stencil", ["face", "full"])
@pytest.mark.parametrize("kind", ["as", "sas", "ras"])
@pytest.mark.parametrize("k", [1, 16, 37])
def test_transposed_preconditioner_matches_oracle(case_small2d, stencil, kind, k):
    """M^{-T} r against the transpose of the oracle's dense M^{-1} (the vector,
    the matrix-core and the mixed chunking of the local solves)."""
    prob, ref = case_small2d
    sysm, H = ref["sys"], ref["H"]
    HtH = H.T @ H
    s = binding.Solver(prob, device=DEV, stencil=stencil, precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(9)
    r = rng.standard_normal((sysm.P, k))
    M = osw.schwarz_dense(HtH, sysm.col_off, osw.stencil(prob, stencil), kind).dense()
    z = s.apply_precond_T(torch.as_tensor(r, device=DEV)).cpu().numpy()
    kappa = np.linalg.cond(HtH)
    ref_z = M.T @ r
    for t in range(k):
        e = rel(z[:, t], ref_z[:, t])
        assert e < max(1e-9, 1e-15 * kappa), (t, e, kappa)


@pytest.mark.parametrize("method,kind", [("cgs", "as"), ("cgs", "sas"), ("cgs", "ras"),
                                         ("bicg", "as"), ("bicg", "sas"), ("bicg", "ras")])
def test_cgs_bicg_match_qr_and_oracle_iterations(case_small2d, method, kind):
    """FP64 CGS and BiCG reach the QR solution to the FP64 bar, with per-RHS
    iteration counts close to the oracle's (same recurrences, summation order
    and the assembled normal matrix aside)."""
    prob, ref = case_small2d
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, method=method, maxiter=5000)
    assert info["status"] == 0
    assert info["max_rel_residual"] <= 1e-12
    err = rel(W.cpu().numpy(), ref["W"])
    it = osolve.iterative(prob, sysm, "full", kind, method, tol=1e-12, maxiter=5000)
    print(f"{method}/{kind}: GPU iterations {info['rhs_iterations']}, oracle {it['iters']}, err {err:.2e}")
    assert err <= 1e-8, err
    for t in range(prob.F.shape[1]):
        g, o = int(info["rhs_iterations"][t]), int(it["iters"][t])
        assert abs(g - o) <= max(3, 0.25 * o), (t, g, o)


@pytest.mark.parametrize("method", ["cgs", "bicg"])
def test_cgs_bicg_batched_mixed_and_adjoint(case_small2d_k37, method):
    """37 right-hand sides (matrix-core chunks of the preconditioner) with the
    SAS preconditioner: mixed precision to 1e-6; then the adjoint through the
    same method against the QR adjoint.  The tolerance is 1e-12: without CG's
    symmetric recurrence these methods stall near 1e-13 in FP64 (the oracle
    leaves 5 (CGS) and 12 (BiCG) of these 37 right-hand sides above 1e-13)."""
    prob, ref = case_small2d_k37
    sysm, qr = ref["sys"], ref["qr"]
    s = binding.Solver(prob, device=DEV, precision="mixed", precond="sas")
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, method=method, maxiter=5000)
    assert info["status"] == 0
    assert info["max_rel_residual"] <= 1e-12
    Wn = W.cpu().numpy()
    for t in range(Wn.shape[1]):
        assert rel(Wn[:, t], ref["W"][:, t]) <= 1e-6, t
    s64 = binding.Solver(prob, device=DEV, precond="sas")
    s64.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(5)
    dW = rng.standard_normal((sysm.P, 3))
    # the adjoint confirms on ||dW - H^T H z|| / ||dW||, whose FP64 floor for a
    # random dW is near u kappa(H^T H) (about 6e-10 here, even for a direct solve)
    dF, st = s64.solve_backward(torch.as_tensor(dW, device=DEV), tol=1e-9, maxiter=5000, method=method)
    assert st["status"] == 0
    expect = qr.adjoint(dW)
    expect[prob.N_I:] *= prob.lambda_B
    assert rel(dF.cpu().numpy(), expect) <= 1e-8


def test_mixed_precision_solution(case_small2d):
    prob, ref = case_small2d
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precision="mixed")
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=5000)
    assert info["max_rel_residual"] <= 1e-13
    assert rel(W.cpu().numpy(), ref["W"]) <= 1e-6


def test_cfg1_full_size_fp64():
    _need_gpu()
    prob = wl.cfg1()
    ref = osolve.reference(prob, "rel_eig", 1e-10)
    s = binding.Solver(prob, device=DEV)
    p = s.pca(1e-10)
    assert np.array_equal(p, ref["sys"].p)
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, maxiter=2000)
    c = s.coeffs(W).cpu().numpy()
    U = s.eval(torch.as_tensor(prob.probes, device=DEV), W).cpu().numpy()
    Uref = oasm.probe_matrix(prob, ref["sys"], prob.probes) @ ref["W"]
    bound, _ = _pca_bound(s, ref["sys"], ref["qr"].cond_estimate())
    assert rel(c, ref["c"]) <= bound
    assert rel(U, Uref) <= 1e-8
    # with the oracle's basis the solve itself matches at the FP64 bar
    s2 = binding.Solver(prob, device=DEV)
    s2.pca(1e-10, p_force=ref["sys"].p, V_force=vforce(ref["sys"]))
    W2, _ = s2.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=2000)
    assert rel(W2.cpu().numpy(), ref["W"]) <= 1e-8


# ------------------------------------------------------------------ a10 adjoint, a11 eval
@pytest.mark.parametrize("k", [3, 16])
def test_eval_and_transpose(case_small2d, k):
    """Probe values and their transpose against the oracle's probe matrix: per
    pair (k = 3) and through the explicit probe values and batched products
    (k = 16)."""
    prob, ref = case_small2d
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    Pm = oasm.probe_matrix(prob, sysm, prob.probes)
    rng = np.random.default_rng(2)
    W = rng.standard_normal((sysm.P, k))
    dU = rng.standard_normal((prob.probes.shape[0], k))
    Xq = torch.as_tensor(prob.probes, device=DEV)
    U = s.eval(Xq, torch.as_tensor(W, device=DEV)).cpu().numpy()
    dW = s.eval_T(Xq, torch.as_tensor(dU, device=DEV)).cpu().numpy()
    assert rel(U, Pm @ W) < 1e-12
    assert rel(dW, Pm.T @ dU) < 1e-12


def test_adjoint_matches_qr_and_fd(case_small2d):
    prob, ref = case_small2d
    sysm, qr = ref["sys"], ref["qr"]
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(3)
    dW = rng.standard_normal((sysm.P, 2))
    dF, _ = s.solve_backward(torch.as_tensor(dW, device=DEV), tol=1e-13, maxiter=3000)
    expect = qr.adjoint(dW)
    expect[prob.N_I:] *= prob.lambda_B
    assert rel(dF.cpu().numpy(), expect) <= 1e-8
    # autograd function against central differences of the (quadratic) misfit
    Xq = torch.as_tensor(prob.probes, device=DEV)
    fn = binding.RannDDSolve.make(s, Xq, tol=1e-13)
    f = torch.as_tensor(prob.F[:prob.N_I, :1], device=DEV).clone().requires_grad_(True)
    g = torch.as_tensor(prob.F[prob.N_I:, :1], device=DEV).clone().requires_grad_(True)
    u_obs = torch.as_tensor(prob.u_probe[:, None], device=DEV)
    loss = ((fn(f, g) - u_obs) ** 2).sum()
    loss.backward()
    for q in range(3):
        df = torch.as_tensor(rng.standard_normal(f.shape), device=DEV)
        dg = torch.as_tensor(rng.standard_normal(g.shape), device=DEV)
        ad = float((f.grad * df).sum() + (g.grad * dg).sum())
        h = 1e-3
        with torch.no_grad():
            lp = float(((fn(f + h * df, g + h * dg) - u_obs) ** 2).sum())
            lm = float(((fn(f - h * df, g - h * dg) - u_obs) ** 2).sum())
        fd = (lp - lm) / (2 * h)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


# ------------------------------------------------------------------ status codes, determinism
def test_not_converged_and_nan_status(case_small2d):
    prob, ref = case_small2d
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10)
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-14, maxiter=1, check_every=1)
    assert info["status"] == binding.RANN_ENOTCONV
    assert np.all(np.isfinite(W.cpu().numpy()))
    F = prob.F.copy()
    F[3, 0] = np.nan
    with pytest.raises(binding.RannError) as e:
        s.solve(torch.as_tensor(F, device=DEV), tol=1e-10, maxiter=50)
    assert e.value.code == binding.RANN_ENAN


def test_bitwise_repeatable(case_small2d):
    prob, ref = case_small2d
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10)
    F = torch.as_tensor(prob.F, device=DEV)
    W1, _ = s.solve(F, tol=1e-12)
    W2, _ = s.solve(F, tol=1e-12)
    assert torch.equal(W1, W2)


@pytest.mark.parametrize("k", [2, 32])
def test_check_windows_do_not_change_the_iterates(k):
    """The host's check cadence, and the windows it shortens near convergence,
    decide only when the host looks at the recurrence: every cadence gives the
    same iterates bit for bit and the same per-right-hand-side counts."""
    _need_gpu()
    prob = wl.small2d(k=k)
    s = binding.Solver(prob, device=DEV)
    s.pca(1e-10)
    F = torch.as_tensor(prob.F, device=DEV)
    runs = [s.solve(F, tol=1e-10, check_every=c) for c in (1, 7, 10)]
    for _, info in runs:
        assert info["status"] == 0
    W0, i0 = runs[0]
    for W, info in runs[1:]:
        assert torch.equal(W, W0)
        assert np.array_equal(info["rhs_iterations"], i0["rhs_iterations"])


@pytest.mark.parametrize("method", ["cg", "bicg", "gmres"])
@pytest.mark.parametrize("k", [4, 8, 64])
def test_power_of_two_rhs_reductions(method, k):
    """Right-hand-side counts whose dot products and partial sums take the
    wave-butterfly reductions (k a power of two up to 64): solutions against
    the QR solution column by column, FP64."""
    _need_gpu()
    prob = wl.small2d(k=k)
    ref = osolve.reference(prob, "rel_eig", 1e-10)
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precond="as")
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, method=method, maxiter=5000)
    assert info["status"] == 0
    assert info["max_rel_residual"] <= 1e-12
    Wn = W.cpu().numpy()
    for t in range(k):
        e = rel(Wn[:, t], ref["W"][:, t])
        assert e <= 1e-8, (t, e)


# ------------------------------------------------------------------ 3D: 27-block stencils
@pytest.fixture(scope="module")
def case_small3d():
    """3x3x3 subdomains of uneven width: the full stencil of the centre block
    holds all 27 subdomains, the face stencil 7."""
    _need_gpu()
    prob = wl.small3d(l=(3, 3, 3), k=2)
    ref = osolve.reference(prob, "rel_eig", 1e-10)
    return prob, ref


@pytest.mark.parametrize("stencil", ["face", "full"])
@pytest.mark.parametrize("kind", ["as", "ras", "sas"])
@pytest.mark.parametrize("k", [1, 16])
def test_preconditioner_3d_matches_oracle(case_small3d, stencil, kind, k):
    prob, ref = case_small3d
    sysm, H = ref["sys"], ref["H"]
    HtH = H.T @ H
    sten = osw.stencil(prob, stencil)
    if stencil == "full":
        assert max(len(s) for s in sten) == 27
    M = osw.schwarz_dense(HtH, sysm.col_off, sten, kind).dense()
    s = binding.Solver(prob, device=DEV, stencil=stencil, precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    rng = np.random.default_rng(21)
    r = rng.standard_normal((sysm.P, k))
    kappa = np.linalg.cond(HtH)
    z = s.apply_precond(torch.as_tensor(r, device=DEV)).cpu().numpy()
    zt = s.apply_precond_T(torch.as_tensor(r, device=DEV)).cpu().numpy()
    for t in range(k):
        e = rel(z[:, t], (M @ r)[:, t])
        et = rel(zt[:, t], (M.T @ r)[:, t])
        assert e < max(1e-9, 1e-15 * kappa), (t, e, kappa)
        assert et < max(1e-9, 1e-15 * kappa), (t, et, kappa)


@pytest.mark.parametrize("method,kind,stencil", [("cg", "as", "full"), ("cg", "as", "face"),
                                                 ("gmres", "ras", "full"), ("gmres_right", "sas", "full"),
                                                 ("bicg", "ras", "face"), ("cgs", "sas", "full")])
def test_solve_3d_matches_qr(case_small3d, method, kind, stencil):
    prob, ref = case_small3d
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, stencil=stencil, precond=kind)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-12, method=method, restart=50,
                      maxiter=5000)
    assert info["status"] == 0
    assert info["max_rel_residual"] <= 1e-12
    Wn = W.cpu().numpy()
    errs = [rel(Wn[:, t], ref["W"][:, t]) for t in range(Wn.shape[1])]
    print(f"3D {method}/{kind}/{stencil}: iterations {info['rhs_iterations']}, errors {errs}")
    assert max(errs) <= 1e-8, errs


# ------------------------------------------------------------------ local shift, rank tie
def test_local_shift_counted_and_fit_unchanged():
    """A dead neuron (zero weights and bias) with the PCA off makes H and every
    local block holding it singular: the equilibrated Cholesky takes a
    diagonal shift (counted in the stats), and CG still reaches the
    least-squares fit H W of the live columns (Sec. 3, local inverse)."""
    _need_gpu()
    prob = wl.small2d(k=1)
    prob.R[2][5] = 0.0
    prob.b[2][5] = 0.0
    sysm = oasm.assemble(prob, "off", 0.0)
    H = sysm.dense()
    live = np.abs(H).sum(axis=0) > 0
    assert np.count_nonzero(~live) == 1
    Wl, *_ = np.linalg.lstsq(H[:, live], sysm.Fs, rcond=None)
    s = binding.Solver(prob, device=DEV)
    s.pca(0.0, "off")
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-10, maxiter=5000)
    print(f"dead neuron: status {info['status']} shifts {info['shifts']} residual {info['max_rel_residual']:.2e}")
    assert info["status"] == 0
    assert info["shifts"] >= 1
    fit = s.matvec(W).cpu().numpy()
    # the fit is unique; at a normal residual of 1e-10 it is pinned to about
    # kappa(H) 1e-10 (the raw features without PCA are ill-conditioned)
    kappa = np.linalg.cond(H[:, live])
    assert rel(fit, H[:, live] @ Wl) <= 10 * kappa * 1e-10, (rel(fit, H[:, live] @ Wl), kappa)


def test_pca_rank_tie_status():
    """A relative threshold placed on an eigenvalue of one subdomain's value
    Gram returns RANN_WRANKTIE (outputs valid); moved by 0.1 % either way the
    count changes by one and the status is 0 (Sec. 4 threshold)."""
    _need_gpu()
    prob = wl.small2d(k=1)
    sysm = oasm.assemble(prob, "rel_eig", 1e-10)
    j, kk = 3, 6
    lam = sysm.lam[j]
    tol = lam[kk] / lam[0]
    s = binding.Solver(prob, device=DEV)
    s.pca(tol, "rel_eig")
    assert s.pca_status == binding.RANN_WRANKTIE
    s2 = binding.Solver(prob, device=DEV)
    p_hi = s2.pca(tol * (1 + 1e-3), "rel_eig")
    assert s2.pca_status == 0 and p_hi[j] == kk
    s3 = binding.Solver(prob, device=DEV)
    p_lo = s3.pca(tol * (1 - 1e-3), "rel_eig")
    assert s3.pca_status == 0 and p_lo[j] == kk + 1


def test_mixed_fp32_gram_blocks(case_small2d_k37):
    """Mixed precision with the Schwarz blocks formed from FP32 operator rows on
    the FP32 matrix cores (FP32 accumulation): the solve still reaches the QR
    solution to the mixed bar, column by column (the preconditioner only shapes
    the iteration; residuals use the FP64 rows)."""
    prob, ref = case_small2d_k37
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precision="mixed")
    s.set_tuning(gram32=1)
    s.pca(1e-10, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=5000)
    assert info["status"] == 0
    Wn = W.cpu().numpy()
    for t in range(Wn.shape[1]):
        assert rel(Wn[:, t], ref["W"][:, t]) <= 1e-6, t
