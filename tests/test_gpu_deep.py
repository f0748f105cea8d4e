"""GPU parity of subdomain networks with several fixed hidden layers (paper
eq. (net)) against the FP64 oracle, through the C interface.

Cases: 2D with two inner layers (12, 20) and uneven last widths; 3D with one
inner layer; the Example 1 replica in constrain mode with three inner layers;
a wide case with two inner layers of the largest width (64) and last widths up
to 200 (several 64-wide feature tiles, ragged tails).  Bars as for one hidden
layer: H entries within 1e-11 of the largest entry with the oracle's basis
forced; eigenvalues within 10 m u lambda_1 and the subspace within
100 m u lambda_1 / gap; probe values and their transpose within 1e-12; FP64
solves within 1e-8 of the QR solution, mixed within 1e-6."""
import numpy as np
import pytest
import torch

from oracle import assemble as oasm
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
    if name == "small2d_deep":
        return wl.small2d(inner_widths=(12, 20))
    if name == "small3d_deep":
        return wl.small3d(inner_widths=(9,))
    if name == "ex1_deep":
        return wl.ex1_replica(l=4, m=16, pts=40, inner_widths=(6, 10, 7))
    if name == "wide_deep":
        return wl.small2d(m=(130, 70, 200, 97, 160, 64), inner_widths=(64, 64), k=1)
    raise KeyError(name)


def vforce(sysm):
    return torch.as_tensor(np.concatenate([v.ravel() for v in sysm.V]), device=DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


_REF = {}


def reference(name):
    if name not in _REF:
        prob = make(name)
        tol = prob.meta.get("pca_tol") or 1e-10
        _REF[name] = (prob, tol, osolve.reference(prob, "rel_eig", tol))
    return _REF[name]


@pytest.mark.parametrize("name", ["small2d_deep", "small3d_deep", "ex1_deep", "wide_deep"])
def test_deep_rows_match_oracle_with_forced_basis(name):
    _need_gpu()
    prob, tol, ref = reference(name)
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV)
    s.pca(tol, "rel_eig", p_force=sysm.p, V_force=vforce(sysm))
    blocks = s.arrays()[0].cpu().numpy()
    o = 0
    scale = max(np.abs(b).max() for b in sysm.blocks)
    for j in range(prob.J):
        B = sysm.blocks[j]
        G = blocks[o:o + B.size].reshape(B.shape)
        o += B.size
        assert np.max(np.abs(G - B)) <= 1e-11 * scale, j


def test_deep_rows_without_pca():
    """Raw rows (identity basis) of the wide case: every feature tile."""
    _need_gpu()
    prob = make("wide_deep")
    sysm = oasm.assemble(prob, "off", 0.0)
    s = binding.Solver(prob, device=DEV)
    p = s.pca(0.0, "off")
    assert np.array_equal(p, prob.m)
    blocks = s.arrays()[0].cpu().numpy()
    flat = np.concatenate([b.ravel() for b in sysm.blocks])
    assert np.max(np.abs(blocks - flat)) <= 1e-11 * np.abs(flat).max()


@pytest.mark.parametrize("name", ["small2d_deep", "small3d_deep", "wide_deep"])
def test_deep_pca_counts_and_spectrum(name):
    _need_gpu()
    prob, tol, ref = reference(name)
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV)
    p = s.pca(tol, "rel_eig")
    assert np.array_equal(p, sysm.p)
    _, V, eig = s.arrays()
    eig, V = eig.cpu().numpy(), V.cpu().numpy()
    off = voff = 0
    for j in range(prob.J):
        m = int(prob.m[j])
        lam = sysm.lam[j]
        n = min(lam.size, m)
        assert np.max(np.abs(eig[off:off + n] - lam[:n])) <= 10 * m * np.finfo(float).eps * lam[0]
        Vg = V[voff:voff + m * p[j]].reshape(m, p[j])
        Vo = sysm.V[j]
        gap = lam[p[j] - 1] - (lam[p[j]] if p[j] < lam.size else 0.0)
        bound = 100 * m * np.finfo(float).eps * lam[0] / max(gap, 1e-300)
        assert np.linalg.norm(Vo - Vg @ (Vg.T @ Vo), 2) <= max(bound, 1e-10), j
        off += m
        voff += m * p[j]


@pytest.mark.parametrize("name", ["small2d_deep", "small3d_deep", "ex1_deep"])
def test_deep_eval_and_transpose(name):
    _need_gpu()
    prob, tol, ref = reference(name)
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV)
    s.pca(tol, p_force=sysm.p, V_force=vforce(sysm))
    Lq = None if prob.L_probe is None else torch.as_tensor(prob.L_probe, device=DEV)
    Pm = oasm.probe_matrix(prob, sysm, prob.probes, prob.L_probe)
    rng = np.random.default_rng(2)
    W = rng.standard_normal((sysm.P, 3))
    dU = rng.standard_normal((prob.probes.shape[0], 3))
    Xq = torch.as_tensor(prob.probes, device=DEV)
    U = s.eval(Xq, torch.as_tensor(W, device=DEV), Lq).cpu().numpy()
    dW = s.eval_T(Xq, torch.as_tensor(dU, device=DEV), Lq).cpu().numpy()
    assert rel(U, Pm @ W) < 1e-12
    assert rel(dW, Pm.T @ dU) < 1e-12


@pytest.mark.parametrize("name,precision,bar", [("small2d_deep", "fp64", 1e-8), ("small2d_deep", "mixed", 1e-6),
                                                ("small3d_deep", "fp64", 1e-8), ("ex1_deep", "fp64", 1e-8)])
def test_deep_solve_matches_qr(name, precision, bar):
    _need_gpu()
    prob, tol, ref = reference(name)
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precision=precision)
    s.pca(tol, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=5000)
    assert info["status"] == 0
    Wn = W.cpu().numpy()
    for t in range(Wn.shape[1]):
        assert rel(Wn[:, t], ref["W"][:, t]) <= bar, t


def test_deep_end_to_end_independent_pca():
    """Own PCA, solve and probe evaluation: u_h within 1e-8 of the oracle's."""
    _need_gpu()
    prob, tol, ref = reference("small2d_deep")
    s = binding.Solver(prob, device=DEV)
    s.pca(tol)
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=5000)
    assert info["status"] == 0
    U = s.eval(torch.as_tensor(prob.probes, device=DEV), W).cpu().numpy()
    Uref = oasm.probe_matrix(prob, ref["sys"], prob.probes) @ ref["W"]
    err = rel(U, Uref)
    print(f"deep end-to-end: u err {err:.2e}")
    assert err <= 1e-8


def test_deep_mixed_fp32_gram_blocks():
    """The FP32 copy of the rows (Schwarz blocks from FP32 rows) on the layered path."""
    _need_gpu()
    prob, tol, ref = reference("small2d_deep")
    sysm = ref["sys"]
    s = binding.Solver(prob, device=DEV, precision="mixed")
    s.set_tuning(gram32=1)
    s.pca(tol, p_force=sysm.p, V_force=vforce(sysm))
    W, info = s.solve(torch.as_tensor(prob.F, device=DEV), tol=1e-13, maxiter=5000)
    assert info["status"] == 0
    Wn = W.cpu().numpy()
    for t in range(Wn.shape[1]):
        assert rel(Wn[:, t], ref["W"][:, t]) <= 1e-6, t
