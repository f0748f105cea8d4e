"""ctypes binding of librann_dd.so (include/rann_dd.h), with the same entry-point
names, plus a small handle wrapper that marshals torch device tensors.

Every numerical step runs inside the HIP library; this module only builds the
descriptor, passes device pointers and the current torch stream, and checks
status codes.  There is no fallback: if the library is missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librann_dd.so")

RANN_OK, RANN_EINVAL, RANN_ENOMEM, RANN_EDEVICE, RANN_ENAN, RANN_EBREAKDOWN = 0, -1, -2, -3, -4, -5
RANN_ENOTCONV, RANN_WRANKTIE = 1, 2
FP64, MIXED = 0, 1
STENCIL = {"self": 0, "face": 1, "full": 2}
PRECOND = {"none": 0, "as": 1, "ras": 2, "sas": 3}
PCA_MODE = {"rel_eig": 0, "abs_sigma": 1, "off": 2}
METHOD = {"cg": 0, "gmres": 1, "gmres_right": 2, "cgs": 3, "bicg": 4}
LINEARIZE = {"newton": 0, "picard": 1}

c_dp = ctypes.POINTER(ctypes.c_double)
c_ip = ctypes.POINTER(ctypes.c_int32)
c_lp = ctypes.POINTER(ctypes.c_int64)


class Desc(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("l", ctypes.c_int32 * 4), ("mu", c_dp), ("sigma", ctypes.c_double * 4),
        ("m", c_ip), ("R", ctypes.c_void_p), ("b", ctypes.c_void_p), ("n_int", ctypes.c_int64),
        ("X_int", ctypes.c_void_p), ("a", ctypes.c_void_p), ("beta", ctypes.c_void_p),
        ("c", ctypes.c_void_p), ("n_bnd", ctypes.c_int64), ("X_bnd", ctypes.c_void_p),
        ("lambda_B", ctypes.c_double), ("Lfun", ctypes.c_void_p), ("precision", ctypes.c_int32),
        ("stencil", ctypes.c_int32), ("precond", ctypes.c_int32),
        ("n_inner", ctypes.c_int32), ("inner_w", ctypes.c_int32 * 3), ("R_inner", ctypes.c_void_p),
        ("b_inner", ctypes.c_void_p),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int32), ("method", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("check_every", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("max_rel_residual", ctypes.c_double), ("rel_residual", c_dp),
                ("rhs_iterations", c_ip), ("shifts", ctypes.c_int32),
                ("setup_ms", ctypes.c_double * 4)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_grid", ctypes.c_int32), ("red_cap", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("pca_subspace", ctypes.c_int32), ("gram32", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"tile_grid": self.tile_grid, "red_cap": self.red_cap, "use_graph": self.use_graph}


class Info(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("J", ctypes.c_int32), ("N_int", ctypes.c_int64),
                ("N_bnd", ctypes.c_int64), ("N", ctypes.c_int64), ("P", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("nnz", ctypes.c_int64), ("sum_m", ctypes.c_int64),
                ("factor_elems", ctypes.c_int64), ("max_q", ctypes.c_int32),
                ("pca_done", ctypes.c_int32), ("normal_elems", ctypes.c_int64),
                ("cg_graphs", ctypes.c_int32), ("graph_failed", ctypes.c_int32)]


_SIGS = {
    "rann_dd_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "rann_dd_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "rann_dd_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(Tuning),
                                        ctypes.POINTER(ctypes.c_double)]),
    "rann_dd_assemble": (ctypes.c_int, [ctypes.POINTER(Desc), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "rann_dd_pca": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int32, c_ip, ctypes.c_void_p, c_ip]),
    "rann_dd_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                     ctypes.POINTER(SolveOpts), ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "rann_dd_solve_backward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.POINTER(SolveOpts), ctypes.c_void_p, ctypes.POINTER(Stats)]),
    "rann_dd_eval": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_eval_T": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_coeffs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_matvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_rmatvec": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_apply_normal": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_apply_precond": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_apply_precond_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                                     ctypes.c_void_p]),
    "rann_dd_apply_precond_T": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "rann_dd_linearize": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, c_dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, c_dp]),
    "rann_dd_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "rann_dd_get_layout": (ctypes.c_int, [ctypes.c_void_p, c_lp, c_ip, c_ip]),
    "rann_dd_get_arrays": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rann_dd_get_blocks": (ctypes.c_int, [ctypes.c_void_p, c_lp]),
    "rann_dd_ktime_enable": (ctypes.c_int, [ctypes.c_int32]),
    "rann_dd_ktime_query": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "rann_dd_destroy": (None, [ctypes.c_void_p]),
    "rann_dd_trim_cache": (ctypes.c_size_t, []),
    "rann_dd_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the library first (paper_2412_19207_amd.build.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RannError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rann_dd error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc < 0:
        raise RannError(rc, load().rann_dd_last_error().decode())
    return rc


# thin wrappers with the C names ---------------------------------------------------

def rann_dd_assemble(desc: Desc, stream: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(load().rann_dd_assemble(ctypes.byref(desc), ctypes.c_void_p(stream), ctypes.byref(h)))
    return h


def rann_dd_pca(h, tol, mode, p_force=None, V_force_ptr=0, J=None):
    lib = load()
    pf = None
    if p_force is not None:
        pf = np.ascontiguousarray(p_force, dtype=np.int32)
    pout = np.zeros(J, dtype=np.int32)
    rc = _check(lib.rann_dd_pca(h, float(tol), int(mode),
                                pf.ctypes.data_as(c_ip) if pf is not None else None,
                                ctypes.c_void_p(V_force_ptr) if V_force_ptr else None,
                                pout.ctypes.data_as(c_ip)))
    return rc, pout


def rann_dd_solve(h, F_ptr, k, W0_ptr, opts: SolveOpts, W_ptr, stats: Optional[Stats]):
    return _check(load().rann_dd_solve(h, ctypes.c_void_p(F_ptr), int(k),
                                       ctypes.c_void_p(W0_ptr) if W0_ptr else None,
                                       ctypes.byref(opts), ctypes.c_void_p(W_ptr),
                                       ctypes.byref(stats) if stats is not None else None))


def rann_dd_solve_backward(h, dW_ptr, k, opts: SolveOpts, dF_ptr, stats: Optional[Stats]):
    return _check(load().rann_dd_solve_backward(h, ctypes.c_void_p(dW_ptr), int(k), ctypes.byref(opts),
                                                ctypes.c_void_p(dF_ptr),
                                                ctypes.byref(stats) if stats is not None else None))


def rann_dd_eval(h, Xq_ptr, M, Lq_ptr, W_ptr, k, U_ptr):
    return _check(load().rann_dd_eval(h, ctypes.c_void_p(Xq_ptr), int(M),
                                      ctypes.c_void_p(Lq_ptr) if Lq_ptr else None,
                                      ctypes.c_void_p(W_ptr), int(k), ctypes.c_void_p(U_ptr)))


def rann_dd_eval_T(h, Xq_ptr, M, Lq_ptr, dU_ptr, k, dW_ptr):
    return _check(load().rann_dd_eval_T(h, ctypes.c_void_p(Xq_ptr), int(M),
                                        ctypes.c_void_p(Lq_ptr) if Lq_ptr else None,
                                        ctypes.c_void_p(dU_ptr), int(k), ctypes.c_void_p(dW_ptr)))


def rann_dd_coeffs(h, W_ptr, k, c_ptr):
    return _check(load().rann_dd_coeffs(h, ctypes.c_void_p(W_ptr), int(k), ctypes.c_void_p(c_ptr)))


def rann_dd_matvec(h, x_ptr, k, y_ptr):
    return _check(load().rann_dd_matvec(h, ctypes.c_void_p(x_ptr), int(k), ctypes.c_void_p(y_ptr)))


def rann_dd_rmatvec(h, y_ptr, k, x_ptr):
    return _check(load().rann_dd_rmatvec(h, ctypes.c_void_p(y_ptr), int(k), ctypes.c_void_p(x_ptr)))


def rann_dd_apply_normal(h, x_ptr, k, s_ptr):
    return _check(load().rann_dd_apply_normal(h, ctypes.c_void_p(x_ptr), int(k), ctypes.c_void_p(s_ptr)))


def rann_dd_apply_precond(h, r_ptr, k, z_ptr):
    return _check(load().rann_dd_apply_precond(h, ctypes.c_void_p(r_ptr), int(k), ctypes.c_void_p(z_ptr)))


def rann_dd_get_tuning(h) -> Tuning:
    t = Tuning()
    _check(load().rann_dd_get_tuning(h, ctypes.byref(t)))
    return t


def rann_dd_set_tuning(h, t: Tuning):
    return _check(load().rann_dd_set_tuning(h, ctypes.byref(t)))


def rann_dd_autotune(h, k, iters):
    t = Tuning()
    us = ctypes.c_double(0.0)
    _check(load().rann_dd_autotune(h, int(k), int(iters), ctypes.byref(t), ctypes.byref(us)))
    return t, us.value


def rann_dd_apply_precond_noalloc(h, r_ptr, k, z_ptr):
    return _check(load().rann_dd_apply_precond_noalloc(h, ctypes.c_void_p(r_ptr), int(k), ctypes.c_void_p(z_ptr)))


def rann_dd_apply_precond_T(h, r_ptr, k, z_ptr):
    return _check(load().rann_dd_apply_precond_T(h, ctypes.c_void_p(r_ptr), int(k), ctypes.c_void_p(z_ptr)))


def rann_dd_linearize(h, u_ptr, c0_ptr, f_ptr, n, gamma, mode, c_out_ptr, f_out_ptr, u_prev_ptr=0):
    """Returns the relative increment ||u - u_prev|| / ||u|| (0.0 without u_prev)."""
    g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    inc = ctypes.c_double(0.0)
    _check(load().rann_dd_linearize(h, ctypes.c_void_p(u_ptr), ctypes.c_void_p(c0_ptr), ctypes.c_void_p(f_ptr),
                                    int(n), g.ctypes.data_as(c_dp), int(g.size), int(mode),
                                    ctypes.c_void_p(c_out_ptr), ctypes.c_void_p(f_out_ptr),
                                    ctypes.c_void_p(u_prev_ptr or None), ctypes.byref(inc)))
    return float(inc.value)


def rann_dd_get_info(h) -> Info:
    info = Info()
    _check(load().rann_dd_get_info(h, ctypes.byref(info)))
    return info


def rann_dd_get_layout(h, J, pairs, with_p=True):
    row_off = np.zeros(J + 1, dtype=np.int64)
    rows = np.zeros(max(pairs, 1), dtype=np.int32)
    p = np.zeros(J, dtype=np.int32)
    _check(load().rann_dd_get_layout(h, row_off.ctypes.data_as(c_lp), rows.ctypes.data_as(c_ip),
                                     p.ctypes.data_as(c_ip) if with_p else None))
    return row_off, rows[:pairs], (p if with_p else None)


def rann_dd_get_arrays(h, blocks_ptr=0, V_ptr=0, eig_ptr=0):
    return _check(load().rann_dd_get_arrays(h, ctypes.c_void_p(blocks_ptr) if blocks_ptr else None,
                                            ctypes.c_void_p(V_ptr) if V_ptr else None,
                                            ctypes.c_void_p(eig_ptr) if eig_ptr else None))


def rann_dd_get_blocks(h, J):
    q = np.zeros(J, dtype=np.int64)
    _check(load().rann_dd_get_blocks(h, q.ctypes.data_as(c_lp)))
    return q


def rann_dd_ktime_enable(on: bool):
    return _check(load().rann_dd_ktime_enable(1 if on else 0))


def rann_dd_ktime_query(name: str):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().rann_dd_ktime_query(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def rann_dd_destroy(h):
    load().rann_dd_destroy(h)


def rann_dd_trim_cache():
    return int(load().rann_dd_trim_cache())


def rann_dd_last_error() -> str:
    return load().rann_dd_last_error().decode()


# handle wrapper over torch device tensors -------------------------------------------

class Solver:
    """One assembled problem on the current CUDA (HIP) device.

    `prob` is a workloads.Problem (or any object with the same fields).  Every
    array is uploaded once as an FP64 device tensor; the library copies what it
    keeps, so the uploads are released after assembly.  `c` (an FP64 device
    tensor of n_int entries) replaces the problem's reaction coefficient."""

    def __init__(self, prob, precision="fp64", stencil="full", precond="as", device="cuda:0",
                 stream=None, c=None):
        import torch
        self.torch = torch
        self.precision, self.stencil, self.precond = precision, stencil, precond
        self.dev = torch.device(device)
        self.prob = prob
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        d = prob.d
        self.d = d
        self.J = int(np.prod(prob.l))
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.dev)
        inner = getattr(prob, "inner", None)
        w_in = d if not inner else int(np.asarray(inner[0][-1][0]).shape[0])
        R = t(np.concatenate([np.asarray(r).reshape(-1, w_in) for r in prob.R], axis=0))
        b = t(np.concatenate([np.asarray(x).ravel() for x in prob.b]))
        Xi, a, be = t(prob.X_int), t(prob.a), t(prob.beta)
        c = t(prob.c) if c is None else c.to(self.dev, torch.float64).contiguous()
        Xb = t(prob.X_bnd) if prob.X_bnd.shape[0] else None
        Lf = t(prob.Lfun) if prob.Lfun is not None else None
        self._mu = np.ascontiguousarray(np.concatenate([np.asarray(m, float) for m in prob.mu]))
        self._m = np.ascontiguousarray(np.asarray(prob.m, dtype=np.int32))
        desc = Desc()
        desc.d = d
        for i in range(4):
            desc.l[i] = int(prob.l[i]) if i < d else 1
            desc.sigma[i] = float(prob.sigma[i]) if i < d else 1.0
        desc.mu = self._mu.ctypes.data_as(c_dp)
        desc.m = self._m.ctypes.data_as(c_ip)
        desc.R, desc.b = R.data_ptr(), b.data_ptr()
        desc.n_int = prob.X_int.shape[0]
        desc.X_int, desc.a, desc.beta, desc.c = Xi.data_ptr(), a.data_ptr(), be.data_ptr(), c.data_ptr()
        desc.n_bnd = prob.X_bnd.shape[0]
        desc.X_bnd = Xb.data_ptr() if Xb is not None else None
        desc.lambda_B = float(prob.lambda_B)
        desc.Lfun = Lf.data_ptr() if Lf is not None else None
        desc.precision = FP64 if precision == "fp64" else MIXED
        desc.stencil = STENCIL[stencil]
        desc.precond = PRECOND[precond]
        if inner:
            # several hidden layers: every subdomain's inner layers, in order
            widths = [int(np.asarray(Ri).shape[0]) for Ri, _ in inner[0]]
            desc.n_inner = len(widths)
            for i, w in enumerate(widths):
                desc.inner_w[i] = w
            Rin = t(np.concatenate([np.asarray(Ri, float).ravel() for layers in inner for Ri, _ in layers]))
            bin_ = t(np.concatenate([np.asarray(bi, float).ravel() for layers in inner for _, bi in layers]))
            desc.R_inner, desc.b_inner = Rin.data_ptr(), bin_.data_ptr()
        self.handle = rann_dd_assemble(desc, self.stream.cuda_stream)
        self.info = rann_dd_get_info(self.handle)
        self.p = None

    def close(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.rann_dd_destroy(h)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up
    def pca(self, tol=1e-8, mode="rel_eig", p_force=None, V_force=None):
        vptr = V_force.data_ptr() if V_force is not None else 0
        rc, p = rann_dd_pca(self.handle, tol, PCA_MODE[mode], p_force, vptr, self.J)
        self.p = p
        self.info = rann_dd_get_info(self.handle)
        self.pca_status = rc
        return p

    # -- solves
    def _opts(self, tol, maxiter, method, restart, check_every):
        return SolveOpts(tol=float(tol), maxiter=int(maxiter), method=METHOD[method],
                         restart=int(restart), check_every=int(check_every))

    def solve(self, F, tol=1e-10, maxiter=2000, method="cg", restart=50, check_every=10, W0=None,
              stats=True):
        torch = self.torch
        F = F.to(self.dev, torch.float64).contiguous()
        k = F.shape[1]
        W = torch.empty((self.info.P, k), dtype=torch.float64, device=self.dev)
        st = None
        rel = np.zeros(k)
        its = np.zeros(k, dtype=np.int32)
        if stats:
            st = Stats()
            st.rel_residual = rel.ctypes.data_as(c_dp)
            st.rhs_iterations = its.ctypes.data_as(c_ip)
        rc = rann_dd_solve(self.handle, F.data_ptr(), k, W0.data_ptr() if W0 is not None else 0,
                           self._opts(tol, maxiter, method, restart, check_every), W.data_ptr(), st)
        info = dict(status=rc)
        if st is not None:
            info.update(iterations=st.iterations, converged=st.converged,
                        max_rel_residual=st.max_rel_residual, rel_residual=rel.copy(),
                        rhs_iterations=its.copy(), shifts=st.shifts)
        return W, info

    def solve_backward(self, dW, tol=1e-12, maxiter=2000, method="cg", restart=50, check_every=10):
        torch = self.torch
        dW = dW.to(self.dev, torch.float64).contiguous()
        k = dW.shape[1]
        dF = torch.empty((self.info.N, k), dtype=torch.float64, device=self.dev)
        st = Stats()
        rc = rann_dd_solve_backward(self.handle, dW.data_ptr(), k,
                                    self._opts(tol, maxiter, method, restart, check_every),
                                    dF.data_ptr(), st)
        return dF, dict(status=rc, iterations=st.iterations)

    # -- launch parameters
    def graph_state(self):
        """(captured CG window graphs held, 1 if a capture failed)."""
        i = rann_dd_get_info(self.handle)
        return int(i.cg_graphs), int(i.graph_failed)

    def tuning(self):
        return rann_dd_get_tuning(self.handle).as_dict()

    def set_tuning(self, tile_grid=None, red_cap=None, use_graph=None, pca_subspace=None, gram32=None):
        t = rann_dd_get_tuning(self.handle)
        if gram32 is not None:
            t.gram32 = int(bool(gram32))
        if pca_subspace is not None:
            t.pca_subspace = int(bool(pca_subspace))
        if tile_grid is not None:
            t.tile_grid = int(tile_grid)
        if red_cap is not None:
            t.red_cap = int(red_cap)
        if use_graph is not None:
            t.use_graph = int(bool(use_graph))
        rann_dd_set_tuning(self.handle, t)

    def autotune(self, k, iters=20, cache=True):
        """Launch parameters of the Krylov step for k right-hand sides: from the
        tuning cache when it holds this case, else timed by rann_dd_autotune and
        stored there (paper_2412_19207_amd.autotune)."""
        from . import autotune as at
        return at.tune(self, k, iters=iters, use_cache=cache)

    # -- products and probes
    def matvec(self, x):
        y = self.torch.empty((self.info.N, x.shape[1]), dtype=self.torch.float64, device=self.dev)
        rann_dd_matvec(self.handle, x.contiguous().data_ptr(), x.shape[1], y.data_ptr())
        return y

    def rmatvec(self, y):
        x = self.torch.empty((self.info.P, y.shape[1]), dtype=self.torch.float64, device=self.dev)
        rann_dd_rmatvec(self.handle, y.contiguous().data_ptr(), y.shape[1], x.data_ptr())
        return x

    def apply_normal(self, x):
        s = self.torch.empty((self.info.P, x.shape[1]), dtype=self.torch.float64, device=self.dev)
        rann_dd_apply_normal(self.handle, x.contiguous().data_ptr(), x.shape[1], s.data_ptr())
        return s

    def apply_precond(self, r):
        z = self.torch.empty((self.info.P, r.shape[1]), dtype=self.torch.float64, device=self.dev)
        rann_dd_apply_precond(self.handle, r.contiguous().data_ptr(), r.shape[1], z.data_ptr())
        return z

    def apply_precond_T(self, r):
        z = self.torch.empty((self.info.P, r.shape[1]), dtype=self.torch.float64, device=self.dev)
        rann_dd_apply_precond_T(self.handle, r.contiguous().data_ptr(), r.shape[1], z.data_ptr())
        return z

    def eval(self, Xq, W, Lq=None):
        torch = self.torch
        Xq = Xq.to(self.dev, torch.float64).contiguous()
        U = torch.empty((Xq.shape[0], W.shape[1]), dtype=torch.float64, device=self.dev)
        rann_dd_eval(self.handle, Xq.data_ptr(), Xq.shape[0], Lq.data_ptr() if Lq is not None else 0,
                     W.contiguous().data_ptr(), W.shape[1], U.data_ptr())
        return U

    def eval_T(self, Xq, dU, Lq=None):
        torch = self.torch
        Xq = Xq.to(self.dev, torch.float64).contiguous()
        dW = torch.empty((self.info.P, dU.shape[1]), dtype=torch.float64, device=self.dev)
        rann_dd_eval_T(self.handle, Xq.data_ptr(), Xq.shape[0], Lq.data_ptr() if Lq is not None else 0,
                       dU.contiguous().data_ptr(), dU.shape[1], dW.data_ptr())
        return dW

    def coeffs(self, W):
        c = self.torch.empty((self.info.sum_m, W.shape[1]), dtype=self.torch.float64, device=self.dev)
        rann_dd_coeffs(self.handle, W.contiguous().data_ptr(), W.shape[1], c.data_ptr())
        return c

    # -- internal arrays (verification)
    def layout(self):
        return rann_dd_get_layout(self.handle, self.J, self.info.pairs, with_p=self.info.pca_done == 1)

    def blocks(self):
        return rann_dd_get_blocks(self.handle, self.J)

    def arrays(self):
        torch = self.torch
        blocks = torch.empty(max(self.info.nnz, 1), dtype=torch.float64, device=self.dev)
        vlen = int(sum(int(m) * int(p) for m, p in zip(self.prob.m, self.p)))
        V = torch.empty(max(vlen, 1), dtype=torch.float64, device=self.dev)
        eig = torch.empty(max(self.info.sum_m, 1), dtype=torch.float64, device=self.dev)
        rann_dd_get_arrays(self.handle, blocks.data_ptr(), V.data_ptr(), eig.data_ptr())
        return blocks, V, eig


def _split_blocks(flat, sizes):
    out, o = [], 0
    for (n, p) in sizes:
        out.append(flat[o:o + n * p].reshape(n, p))
        o += n * p
    return out


class RannDDSolve:
    """torch.autograd.Function factory: u = Pmat W(F) at probe points, with the
    backward pass dF = H (H^T H)^{-1} Pmat^T dU computed by the library's adjoint
    solve.  Boundary-row gradients are returned with respect to the unscaled g."""

    @staticmethod
    def make(solver: Solver, Xq, Lq=None, tol=1e-12, maxiter=4000, method="cg"):
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, f, g):
                F = torch.cat([f, g], dim=0)
                W, info = solver.solve(F, tol=tol, maxiter=maxiter, method=method, stats=False)
                if info["status"] != RANN_OK:
                    raise RannError(info["status"], "forward solve did not reach the tolerance")
                return solver.eval(Xq, W, Lq)

            @staticmethod
            def backward(ctx, dU):
                dW = solver.eval_T(Xq, dU.contiguous(), Lq)
                dF, info = solver.solve_backward(dW, tol=tol, maxiter=maxiter, method=method)
                if info["status"] != RANN_OK:
                    raise RannError(info["status"], "adjoint solve did not reach the tolerance")
                n_int = solver.info.N_int
                return dF[:n_int], dF[n_int:]

        return _Fn.apply
