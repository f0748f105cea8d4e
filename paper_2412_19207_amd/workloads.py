"""Seeded synthetic inputs for the RaNN overlapping-Schwarz solver.

This module only *generates problem data*: collocation and boundary points,
the subdomain layout (centres and half-widths), the fixed random hidden-layer
weights, the coefficients of the linear operator at the collocation points,
the right-hand sides of manufactured problems, and probe points.  It contains
none of the method's arithmetic (no partition of unity, no features, no
assembly, no solver), so that the FP64 oracle and the GPU library can both be
fed from it without sharing any computation.

Problem statement: A[u] = f in the box, B[u] = g on its boundary (paper eq. (1)),
with A[u] = sum_i(-a_i d_ii u + beta_i d_i u) + c u and B the Dirichlet trace.

Layouts (paper Sec. 5, Example 1, subdomain formula):
  * "core"  : l_i uniform core cells of width h_i per dimension, each extended
              by e_i = overlap_i / 2 on every side (also outside the box);
              centre = core-cell centre, half-width sigma_i = h_i/2 + e_i.
  * "paper" : centres at the l_i nodes (j-1)/(l_i-1) (scaled to the box) with
              half-width sigma_i = (delta/2)/(l_i-1), delta > 1 the ratio of
              subdomain width to centre spacing.

Random draws (numpy PCG64): widths (seed_m) -> for each subdomain j in linear
order (dimension 0 fastest): R_j (m_j x d_in) then b_j (m_j), both scale*U[-1,1],
with d_in = d for one hidden layer.

Several hidden layers (paper eq. (net), inner_widths = (w_1, ..., w_{L})): the
inner layers come from a second stream seeded with seed_w + 7919, for each
subdomain j in turn and layer by layer: R (w_i x w_{i-1}, w_0 = d) then b
(w_i).  The first layer acts on the normalised input with weights and biases
U[-1,1] (Example 1's distribution); a layer fed by w tanh outputs (the deeper
inner layers and the last layer) has weights (2/sqrt(w))*U[-1,1] and biases
U[-1,1], which keeps its pre-activations of order one.  The last layer's R_j
is then m_j x w_L.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

PI = math.pi


@dataclasses.dataclass
class Problem:
    name: str
    d: int
    lo: np.ndarray            # (d,)
    hi: np.ndarray            # (d,)
    l: np.ndarray             # (d,) subdomains per dimension
    mu: List[np.ndarray]      # per dimension, centres (l_i,)
    sigma: np.ndarray         # (d,) half-widths
    m: np.ndarray             # (J,) int32 hidden widths
    R: List[np.ndarray]       # per subdomain (m_j, d) raw weights acting on normalised input
    b: List[np.ndarray]       # per subdomain (m_j,)
    X_int: np.ndarray         # (N_I, d)
    a: np.ndarray             # (N_I, d) diffusion coefficients
    beta: np.ndarray          # (N_I, d) advection coefficients
    c: np.ndarray             # (N_I,) reaction coefficient
    X_bnd: np.ndarray         # (N_B, d)
    lambda_B: float
    Lfun: Optional[np.ndarray]  # (N, 1+2d) [L, dL/dx_i, d2L/dx_i2] at interior then boundary rows, or None (L == 1)
    F: np.ndarray             # (N, k): rows f - A[G] (interior) then g - G (boundary), unscaled
    probes: np.ndarray        # (M, d)
    u_probe: Optional[np.ndarray]  # (M,) exact solution of RHS column 0 at probes (None if unknown)
    u_obs: Optional[np.ndarray]    # (M,) observations for the misfit loss
    meta: dict
    L_probe: Optional[np.ndarray] = None  # (M,) constraining multiplier at probes (None: L == 1)
    # inner hidden layers of each subdomain's network (paper eq. (net)), or None
    # for one hidden layer: inner[j] = [(R_1, b_1), ..., (R_L, b_L)], R_i (w_i x
    # w_{i-1}) with w_0 = d; R[j] then acts on the last inner layer's output
    inner: Optional[list] = None

    @property
    def J(self) -> int:
        return int(np.prod(self.l))

    @property
    def N_I(self) -> int:
        return self.X_int.shape[0]

    @property
    def N_B(self) -> int:
        return self.X_bnd.shape[0]

    @property
    def N(self) -> int:
        return self.N_I + self.N_B

    @property
    def k(self) -> int:
        return self.F.shape[1]

    def sub_coords(self, j: int) -> tuple:
        """Tensor index of subdomain j (dimension 0 fastest)."""
        out = []
        for i in range(self.d):
            out.append(j % int(self.l[i]))
            j //= int(self.l[i])
        return tuple(out)

    def centre(self, j: int) -> np.ndarray:
        cc = self.sub_coords(j)
        return np.array([self.mu[i][cc[i]] for i in range(self.d)])


# ----------------------------------------------------------------------------
# point sets
# ----------------------------------------------------------------------------

def cell_centred_grid(lo, hi, counts) -> np.ndarray:
    """Tensor grid of cell centres, dimension 0 fastest. counts per dimension."""
    axes = [lo[i] + (np.arange(counts[i]) + 0.5) * (hi[i] - lo[i]) / counts[i]
            for i in range(len(counts))]
    mesh = np.meshgrid(*axes, indexing="ij")
    # dimension 0 fastest -> flatten in Fortran order
    return np.stack([g.ravel(order="F") for g in mesh], axis=1)


def face_points(lo, hi, faces, counts) -> np.ndarray:
    """Cell-centred points on box faces (corners/edges excluded).

    faces: list of (dim, side) with side 0 = lo, 1 = hi.
    counts: per-dimension number of points along that dimension on a face.
    """
    d = len(lo)
    pts = []
    for (dim, side) in faces:
        if d == 1:
            pts.append(np.array([[lo[0] if side == 0 else hi[0]]]))
            continue
        others = [i for i in range(d) if i != dim]
        sub = cell_centred_grid([lo[i] for i in others], [hi[i] for i in others],
                                [counts[i] for i in others])
        full = np.empty((sub.shape[0], d))
        full[:, others] = sub
        full[:, dim] = lo[dim] if side == 0 else hi[dim]
        pts.append(full)
    if not pts:
        return np.zeros((0, d))
    return np.concatenate(pts, axis=0)


def core_layout(lo, hi, l, overlap):
    """Centres at core-cell centres, half-width = h/2 + overlap/2."""
    mu, sigma = [], []
    for i in range(len(l)):
        h = (hi[i] - lo[i]) / l[i]
        mu.append(lo[i] + (np.arange(l[i]) + 0.5) * h)
        sigma.append(h / 2 + overlap[i] / 2)
    return mu, np.array(sigma)


def paper_layout(lo, hi, l, delta):
    """Centres on the l_i nodes of the box, half-width (delta/2) * spacing."""
    mu, sigma = [], []
    for i in range(len(l)):
        if l[i] < 2:
            raise ValueError("paper layout needs at least 2 subdomains per dimension")
        sp = (hi[i] - lo[i]) / (l[i] - 1)
        mu.append(lo[i] + np.arange(l[i]) * sp)
        sigma.append(0.5 * delta * sp)
    return mu, np.array(sigma)


def draw_weights(J, m, d, scale, seed, inner_widths=None):
    """Last-layer weights R_j, b_j and, for several hidden layers, the inner
    layers of every subdomain (None for one hidden layer)."""
    inner = None
    d_in = d
    if inner_widths:
        widths = [int(w) for w in inner_widths]
        rng_in = np.random.default_rng(seed + 7919)
        inner = []
        for j in range(J):
            layers, w_prev = [], d
            for i, w in enumerate(widths):
                s_w = 1.0 if i == 0 else 2.0 / math.sqrt(w_prev)
                Ri = s_w * rng_in.uniform(-1.0, 1.0, size=(w, w_prev))
                bi = rng_in.uniform(-1.0, 1.0, size=w)
                layers.append((Ri, bi))
                w_prev = w
            inner.append(layers)
        d_in = widths[-1]
    rng = np.random.default_rng(seed)
    R, b = [], []
    for j in range(J):
        if inner is None:
            R.append(scale * rng.uniform(-1.0, 1.0, size=(int(m[j]), d)))
            b.append(scale * rng.uniform(-1.0, 1.0, size=int(m[j])))
        else:
            R.append(2.0 / math.sqrt(d_in) * rng.uniform(-1.0, 1.0, size=(int(m[j]), d_in)))
            b.append(rng.uniform(-1.0, 1.0, size=int(m[j])))
    return R, b, inner


def smooth_modes(d, kmax=6):
    """Integer wave vectors k in {1..kmax}^d with ||k||_2 <= kmax."""
    ks = []
    rng = [range(1, kmax + 1)] * d
    for k in np.array(np.meshgrid(*rng, indexing="ij")).reshape(d, -1).T:
        if np.sqrt((k.astype(float) ** 2).sum()) <= kmax + 1e-12:
            ks.append(k)
    return np.array(ks)


def random_smooth_rhs(X, ks, coef):
    """f(x) = sum_k coef_k prod_i sin(k_i pi x_i)."""
    out = np.zeros(X.shape[0])
    for kk, cc in zip(ks, coef):
        term = np.full(X.shape[0], cc)
        for i in range(X.shape[1]):
            term = term * np.sin(kk[i] * PI * X[:, i])
        out += term
    return out


# ----------------------------------------------------------------------------
# generic builder
# ----------------------------------------------------------------------------

def build_problem(name, d, l, m, weight_scale, pts_per_sub, *, overlap_frac=None,
                  overlap_abs=None, layout="core", delta=2.0, lo=None, hi=None,
                  faces=None, bnd_counts=None, coeff_fn=None, rhs_fn=None,
                  bnd_fn=None, exact_fn=None, Lfun_fn=None, lambda_B=100.0,
                  seed_w=0, probes_per_dim=None, obs_noise=0.0, seed_obs=3,
                  meta=None, inner_widths=None) -> Problem:
    lo = np.zeros(d) if lo is None else np.asarray(lo, float)
    hi = np.ones(d) if hi is None else np.asarray(hi, float)
    l = np.asarray(l, dtype=np.int64)
    J = int(np.prod(l))
    if layout == "core":
        if overlap_abs is None:
            overlap_abs = [overlap_frac * (hi[i] - lo[i]) / l[i] for i in range(d)]
        mu, sigma = core_layout(lo, hi, l, overlap_abs)
    else:
        mu, sigma = paper_layout(lo, hi, l, delta)
    m = np.broadcast_to(np.asarray(m, dtype=np.int32), (J,)).copy()
    R, b, inner = draw_weights(J, m, d, weight_scale, seed_w, inner_widths)
    counts = [int(pts_per_sub[i]) * int(l[i]) for i in range(d)]
    X_int = cell_centred_grid(lo, hi, counts)
    if faces is None:
        faces = []
    X_bnd = face_points(lo, hi, faces, bnd_counts if bnd_counts is not None else counts)
    a, beta, c = coeff_fn(X_int)
    f = rhs_fn(X_int)
    if f.ndim == 1:
        f = f[:, None]
    g = bnd_fn(X_bnd, f.shape[1]) if X_bnd.shape[0] else np.zeros((0, f.shape[1]))
    F = np.concatenate([f, g], axis=0)
    Lf = None
    if Lfun_fn is not None:
        Lf = Lfun_fn(np.concatenate([X_int, X_bnd], axis=0))
    if probes_per_dim is None:
        probes_per_dim = [max(4, 2 * int(pts_per_sub[i]) * int(l[i]) // 3) for i in range(d)]
    probes = cell_centred_grid(lo, hi, probes_per_dim)
    u_probe = exact_fn(probes) if exact_fn is not None else None
    u_obs = None
    if u_probe is not None:
        rng = np.random.default_rng(seed_obs)
        u_obs = u_probe + obs_noise * rng.standard_normal(u_probe.shape[0])
    L_probe = None if Lfun_fn is None else Lfun_fn(probes)[:, 0].copy()
    return Problem(name=name, d=d, lo=lo, hi=hi, l=l, mu=mu, sigma=sigma, m=m,
                   R=R, b=b, X_int=X_int, a=a, beta=beta, c=c, X_bnd=X_bnd,
                   lambda_B=float(lambda_B), Lfun=Lf, F=F, probes=probes,
                   u_probe=u_probe, u_obs=u_obs, meta=dict(meta or {}), L_probe=L_probe,
                   inner=inner)


def _laplace_coeffs(X):
    n, d = X.shape
    return np.ones((n, d)), np.zeros((n, d)), np.zeros(n)


def _all_faces(d):
    return [(i, s) for i in range(d) for s in (0, 1)]


def _zero_bnd(X, k):
    return np.zeros((X.shape[0], k))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def cfg1(**kw) -> Problem:
    """1D Poisson -u''=f, u = sin(2 pi x) + 0.1 sin(20 pi x); 4 subdomains,
    overlap 0.05, width 50, 5*U[-1,1], 100 points per subdomain + 2 boundary rows."""
    def rhs(X):
        x = X[:, 0]
        return 4 * PI ** 2 * (np.sin(2 * PI * x) + 10 * np.sin(20 * PI * x))

    def exact(X):
        x = X[:, 0]
        return np.sin(2 * PI * x) + 0.1 * np.sin(20 * PI * x)

    args = dict(name="poisson1d_l4_m50", d=1, l=[4], m=50, weight_scale=5.0,
                pts_per_sub=[100], overlap_abs=[0.05], faces=_all_faces(1),
                coeff_fn=_laplace_coeffs, rhs_fn=rhs,
                bnd_fn=lambda X, k: exact(X)[:, None].repeat(k, 1), exact_fn=exact,
                probes_per_dim=[1000],
                meta=dict(pca_tol=1e-10, tol=1e-10, stencil="full", method="cg",
                          precond="as"))
    args.update(kw)
    return build_problem(**args)


def cfg2(**kw) -> Problem:
    """2D Poisson, u = sin(pi x) sin(pi y) exp(x+y); 8x8 subdomains (overlap 10 %
    of the core width), width 300, U[-3,3], 30x30 points per subdomain plus 64
    cell-centred points per boundary edge."""
    def exact(X):
        x, y = X[:, 0], X[:, 1]
        return np.sin(PI * x) * np.sin(PI * y) * np.exp(x + y)

    def rhs(X):
        x, y = X[:, 0], X[:, 1]
        e = np.exp(x + y)
        return e * (2 * (PI ** 2 - 1) * np.sin(PI * x) * np.sin(PI * y)
                    - 2 * PI * (np.cos(PI * x) * np.sin(PI * y) + np.sin(PI * x) * np.cos(PI * y)))

    args = dict(name="poisson2d_8x8_m300", d=2, l=[8, 8], m=300, weight_scale=3.0,
                pts_per_sub=[30, 30], overlap_frac=0.1, faces=_all_faces(2),
                bnd_counts=[64, 64], coeff_fn=_laplace_coeffs, rhs_fn=rhs,
                bnd_fn=lambda X, k: exact(X)[:, None].repeat(k, 1), exact_fn=exact,
                probes_per_dim=[160, 160],
                meta=dict(pca_tol=1e-8, tol=1e-6, stencil="full", method="cg",
                          precond="as"))
    args.update(kw)
    return build_problem(**args)


def cfg3(k=32, **kw) -> Problem:
    """2D multiscale elliptic -div(a grad u) = f, a = 2 + sin(2 pi x/eps) sin(2 pi y/eps),
    eps = 1/16; 16x16 subdomains with widths drawn from U{200..600}; 24x24 points per
    subdomain, 24 boundary points per subdomain edge; k batched right-hand sides
    (column 0: f = 1, others random smooth), g = 0."""
    eps = 1.0 / 16.0
    l = kw.pop("l", [16, 16])
    pts = kw.pop("pts_per_sub", [24, 24])
    mrange = kw.pop("mrange", (200, 600))
    J = int(np.prod(l))
    rng_m = np.random.default_rng(2)
    m = rng_m.integers(mrange[0], mrange[1] + 1, size=J).astype(np.int32)

    def coeffs(X):
        x, y = X[:, 0], X[:, 1]
        w = 2 * PI / eps
        a = 2 + np.sin(w * x) * np.sin(w * y)
        ax = w * np.cos(w * x) * np.sin(w * y)
        ay = w * np.sin(w * x) * np.cos(w * y)
        return np.stack([a, a], 1), np.stack([-ax, -ay], 1), np.zeros(X.shape[0])

    ks = smooth_modes(2)
    rng_r = np.random.default_rng(1)
    coefs = rng_r.standard_normal((max(k - 1, 0), ks.shape[0]))

    def rhs(X):
        cols = [np.ones(X.shape[0])]
        for q in range(k - 1):
            cols.append(random_smooth_rhs(X, ks, coefs[q]))
        return np.stack(cols, 1)

    args = dict(name="multiscale2d_16x16_m200_600", d=2, l=l, m=m, weight_scale=1.0,
                pts_per_sub=pts, overlap_frac=0.1, faces=_all_faces(2),
                bnd_counts=[pts[0] * l[0], pts[1] * l[1]], coeff_fn=coeffs, rhs_fn=rhs,
                bnd_fn=_zero_bnd, exact_fn=None,
                meta=dict(pca_tol=1e-8, tol=1e-6, stencil="full", method="cg",
                          precond="as", precision="mixed"))
    args.update(kw)
    return build_problem(**args)


def gaussian_st(X, nu=0.01, sig=0.05, bx=1.0, by=0.5, x0=0.3, y0=0.3):
    x, y, t = X[:, 0], X[:, 1], X[:, 2]
    s2 = sig ** 2 + 2 * nu * t
    return sig ** 2 / s2 * np.exp(-((x - x0 - bx * t) ** 2 + (y - y0 - by * t) ** 2) / (2 * s2))


def cfg4(**kw) -> Problem:
    """Space-time advection-diffusion u_t + b.grad u - nu lap u = 0 on [0,1]^2 x [0,1],
    b = (1, 0.5), nu = 0.01, Gaussian bump initial data; 8x8x8 space-time subdomains,
    width 400, 12^3 points per subdomain; Dirichlet data on x=0,1, y=0,1 and t=0."""
    nu = 0.01
    l = kw.pop("l", [8, 8, 8])
    pts = kw.pop("pts_per_sub", [12, 12, 12])

    def coeffs(X):
        n = X.shape[0]
        a = np.tile(np.array([nu, nu, 0.0]), (n, 1))
        be = np.tile(np.array([1.0, 0.5, 1.0]), (n, 1))
        return a, be, np.zeros(n)

    faces = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)]
    args = dict(name="advdiff_st_8x8x8_m400", d=3, l=l, m=400, weight_scale=1.0,
                pts_per_sub=pts, overlap_frac=0.1, faces=faces,
                bnd_counts=[pts[i] * l[i] for i in range(3)], coeff_fn=coeffs,
                rhs_fn=lambda X: np.zeros(X.shape[0]),
                bnd_fn=lambda X, k: gaussian_st(X, nu)[:, None].repeat(k, 1),
                exact_fn=lambda X: gaussian_st(X, nu), probes_per_dim=[48, 48, 48],
                meta=dict(pca_tol=1e-8, tol=1e-6, stencil="face", method="gmres",
                          restart=50, precond="ras", precision="mixed"))
    args.update(kw)
    return build_problem(**args)


def cfg5(k=16, **kw) -> Problem:
    """3D Poisson, u = sin(pi x) sin(pi y) sin(pi z); 6x6x6 subdomains, width 500,
    14^3 points per subdomain, 14^2 boundary points per subdomain face; k batched
    right-hand sides (column 0 manufactured, others random smooth 3D modes);
    32^3 probe grid with noisy observations of the exact solution."""
    l = kw.pop("l", [6, 6, 6])
    pts = kw.pop("pts_per_sub", [14, 14, 14])
    ks = smooth_modes(3)
    rng_r = np.random.default_rng(1)
    coefs = rng_r.standard_normal((max(k - 1, 0), ks.shape[0]))

    def exact(X):
        return np.sin(PI * X[:, 0]) * np.sin(PI * X[:, 1]) * np.sin(PI * X[:, 2])

    def rhs(X):
        cols = [3 * PI ** 2 * exact(X)]
        for q in range(k - 1):
            cols.append(random_smooth_rhs(X, ks, coefs[q]))
        return np.stack(cols, 1)

    args = dict(name="poisson3d_6x6x6_m500", d=3, l=l, m=500, weight_scale=1.0,
                pts_per_sub=pts, overlap_frac=0.1, faces=_all_faces(3),
                bnd_counts=[pts[i] * l[i] for i in range(3)], coeff_fn=_laplace_coeffs,
                rhs_fn=rhs, bnd_fn=_zero_bnd, exact_fn=exact,
                probes_per_dim=[32, 32, 32], obs_noise=0.01,
                meta=dict(pca_tol=1e-8, tol=1e-6, stencil="full", method="cg",
                          precond="as"))
    args.update(kw)
    return build_problem(**args)


def ex1_replica(n=2, l=4, m=16, pts=40, delta=2.0, seed=0, **kw) -> Problem:
    """Paper Example 1 (multi-scale Laplacian, Dirichlet u = 0) in constrain mode:
    paper layout with ratio delta, U(-1,1) weights, L = prod tanh(x_i/rho) tanh((1-x_i)/rho)
    with rho = (1/2)^n, G = 0, no boundary rows.  The source term uses the squared
    frequencies (the printed form drops the square; it follows from -lap u)."""
    rho = 0.5 ** n
    omegas = [2.0 ** i for i in range(1, n + 1)]

    def exact(X):
        out = np.zeros(X.shape[0])
        for w in omegas:
            out += np.sin(w * PI * X[:, 0]) * np.sin(w * PI * X[:, 1])
        return out / n

    def rhs(X):
        out = np.zeros(X.shape[0])
        for w in omegas:
            out += w ** 2 * PI ** 2 * np.sin(w * PI * X[:, 0]) * np.sin(w * PI * X[:, 1])
        return 2.0 / n * out

    def Lfun(X):
        d = X.shape[1]
        # q(s) = tanh(s/rho) tanh((1-s)/rho) per dimension
        vals, d1, d2 = [], [], []
        for i in range(d):
            s = X[:, i]
            A_ = np.tanh(s / rho)
            B_ = np.tanh((1 - s) / rho)
            dA = (1 - A_ ** 2) / rho
            dB = -(1 - B_ ** 2) / rho
            ddA = -2 * A_ * (1 - A_ ** 2) / rho ** 2
            ddB = -2 * B_ * (1 - B_ ** 2) / rho ** 2
            vals.append(A_ * B_)
            d1.append(dA * B_ + A_ * dB)
            d2.append(ddA * B_ + 2 * dA * dB + A_ * ddB)
        Lv = np.prod(vals, axis=0)
        out = [Lv]
        for i in range(d):
            others = np.prod([vals[q] for q in range(d) if q != i], axis=0)
            out.append(d1[i] * others)
        for i in range(d):
            others = np.prod([vals[q] for q in range(d) if q != i], axis=0)
            out.append(d2[i] * others)
        return np.stack(out, 1)

    args = dict(name=f"ex1_n{n}_l{l}_m{m}", d=2, l=[l, l], m=m, weight_scale=1.0,
                pts_per_sub=[pts // l, pts // l], layout="paper", delta=delta, faces=[],
                coeff_fn=_laplace_coeffs, rhs_fn=rhs, bnd_fn=_zero_bnd, exact_fn=exact,
                Lfun_fn=Lfun, seed_w=seed, probes_per_dim=[100, 100],
                meta=dict(pca_tol=None, tol=1e-5, stencil="full", method="gmres",
                          precond="as"))
    args.update(kw)
    return build_problem(**args)


def small2d(l=(3, 2), m=(40, 57, 33, 64, 48, 71), pts=(11, 9), k=2, seed=0, scale=2.0,
            overlap_frac=0.2, **kw) -> Problem:
    """Small 2D problem with uneven widths and a ragged point count, for parity tests
    that span several kernel tiles and a ragged tail.  -lap u + 0.5 u_x + u = f."""
    def coeffs(X):
        n = X.shape[0]
        return (np.ones((n, 2)), np.tile([0.5, -0.25], (n, 1)), np.ones(n))

    def exact(X):
        return np.sin(PI * X[:, 0]) * np.cos(1.5 * X[:, 1]) + X[:, 0] * X[:, 1]

    def rhs(X):
        x, y = X[:, 0], X[:, 1]
        u = exact(X)
        uxx = -PI ** 2 * np.sin(PI * x) * np.cos(1.5 * y)
        uyy = -2.25 * np.sin(PI * x) * np.cos(1.5 * y)
        ux = PI * np.cos(PI * x) * np.cos(1.5 * y) + y
        uy = -1.5 * np.sin(PI * x) * np.sin(1.5 * y) + x
        f0 = -(uxx + uyy) + 0.5 * ux - 0.25 * uy + u
        cols = [f0] + [np.cos((q + 1) * X[:, 0]) * (1 + X[:, 1]) for q in range(k - 1)]
        return np.stack(cols, 1)

    def bnd(X, kk):
        cols = [exact(X)] + [X[:, 0] - X[:, 1] * q for q in range(1, kk)]
        return np.stack(cols, 1)

    l = list(l)
    J = int(np.prod(l))
    m = np.resize(np.asarray(m, dtype=np.int32), J)
    args = dict(name="small2d", d=2, l=l, m=m, weight_scale=scale,
                pts_per_sub=list(pts), overlap_frac=overlap_frac, faces=_all_faces(2),
                bnd_counts=[7 * l[0], 5 * l[1]], coeff_fn=coeffs, rhs_fn=rhs,
                bnd_fn=bnd, exact_fn=exact, seed_w=seed, probes_per_dim=[23, 19],
                meta=dict(pca_tol=1e-10, tol=1e-12, stencil="full", method="cg",
                          precond="as"))
    args.update(kw)
    return build_problem(**args)


def small3d(l=(2, 2, 2), m=(30, 41, 25, 36, 44, 29, 33, 38), pts=(5, 6, 4), k=1, seed=1,
            **kw) -> Problem:
    """Small 3D Poisson problem (uneven widths) for parity tests."""
    def exact(X):
        return np.sin(PI * X[:, 0]) * np.sin(PI * X[:, 1]) * np.sin(PI * X[:, 2])

    def rhs(X):
        cols = [3 * PI ** 2 * exact(X)] + [np.cos(X[:, 0] + 2 * X[:, 1] * q) for q in range(1, k)]
        return np.stack(cols, 1)

    l = list(l)
    J = int(np.prod(l))
    m = np.resize(np.asarray(m, dtype=np.int32), J)
    args = dict(name="small3d", d=3, l=l, m=m, weight_scale=1.5, pts_per_sub=list(pts),
                overlap_frac=0.2, faces=_all_faces(3), bnd_counts=[4 * l[0], 3 * l[1], 3 * l[2]],
                coeff_fn=_laplace_coeffs, rhs_fn=rhs, bnd_fn=_zero_bnd, exact_fn=exact,
                seed_w=seed, probes_per_dim=[9, 8, 7],
                meta=dict(pca_tol=1e-10, tol=1e-12, stencil="full", method="cg",
                          precond="as"))
    args.update(kw)
    return build_problem(**args)


def semilinear2d(size="full", **kw) -> Problem:
    """Semilinear 2D problem -lap u + g(u) = f with the reaction g(u) = u^3
    (meta["gamma"]: coefficients of g in powers of u), u = sin(pi x) sin(pi y)
    exp(x+y) on the boundary; f from that manufactured solution.  The problem's
    own coefficients are those of the linear part (c = 0); a Picard or Newton
    step replaces c and the interior rows of F.  "full": the 8x8, width-300
    layout of the 2D Poisson workload; "small": 3x2 subdomains of uneven width."""
    def exact(X):
        x, y = X[:, 0], X[:, 1]
        return np.sin(PI * x) * np.sin(PI * y) * np.exp(x + y)

    def rhs(X):
        x, y = X[:, 0], X[:, 1]
        e = np.exp(x + y)
        mlap = e * (2 * (PI ** 2 - 1) * np.sin(PI * x) * np.sin(PI * y)
                    - 2 * PI * (np.cos(PI * x) * np.sin(PI * y) + np.sin(PI * x) * np.cos(PI * y)))
        return mlap + exact(X) ** 3

    # the paper's absolute singular-value threshold tau = 1e-3 on the value matrices
    meta = dict(pca_mode="abs_sigma", pca_tol=1e-3, tol=1e-10, stencil="full", method="cg",
                precond="as", gamma=[0.0, 0.0, 0.0, 1.0])
    if size == "small":
        l, m = [3, 2], np.resize(np.asarray((40, 57, 33, 64, 48, 71), dtype=np.int32), 6)
        args = dict(name="semilinear2d_small", d=2, l=l, m=m, weight_scale=2.0,
                    pts_per_sub=[11, 9], overlap_frac=0.2, faces=_all_faces(2),
                    bnd_counts=[21, 10], probes_per_dim=[23, 19])
        meta.update(pca_mode="rel_eig", pca_tol=1e-10, tol=1e-12)
    else:
        args = dict(name="semilinear2d_8x8_m300", d=2, l=[8, 8], m=300, weight_scale=3.0,
                    pts_per_sub=[30, 30], overlap_frac=0.1, faces=_all_faces(2),
                    bnd_counts=[64, 64], probes_per_dim=[160, 160])
    args.update(coeff_fn=_laplace_coeffs, rhs_fn=rhs,
                bnd_fn=lambda X, k: exact(X)[:, None].repeat(k, 1), exact_fn=exact, meta=meta)
    args.update(kw)
    return build_problem(**args)


def deep2d(**kw) -> Problem:
    """The 2D Poisson workload (8x8 subdomains, last hidden width 300, 30x30
    points per subdomain) with two fixed inner hidden layers of width 64
    before the last hidden layer (paper eq. (net))."""
    args = dict(inner_widths=(64, 64), name="poisson2d_8x8_m300_inner64x64")
    args.update(kw)
    return cfg2(**args)


WORKLOADS = {
    "cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4, "cfg5": cfg5,
    "ex1": ex1_replica, "small2d": small2d, "small3d": small3d,
    "semilinear2d": semilinear2d, "deep2d": deep2d,
}


def make(name: str, **kw) -> Problem:
    return WORKLOADS[name](**kw)
