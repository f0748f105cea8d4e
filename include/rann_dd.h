/*
 * rann_dd.h -- C interface of the MI355X library that assembles and solves the
 * collocation least-squares system of randomized neural networks (RaNNs) with
 * overlapping Schwarz domain decomposition (Shang, Heinlein, Mishra, Wang).
 *
 * Problem (paper eq. (1)): A[u] = f in a box, u = g on its boundary, with the
 * linear operator A[u] = sum_i (-a_i d_ii u + beta_i d_i u) + c u.
 * Ansatz (eq. (netdd), with the PCA layer of eq. (pca_net)):
 *     u(x) = L(x) sum_j w_j(x) W_j . (V_j^T Phi_j(x)) + G(x),
 * Phi_j = tanh(R_j x~ + b_j) with x~ = (x - mu_j) / sigma the input normalised
 * over the support box of subdomain j, w_j the window partition of unity
 * (Sec. 5, Example 1), V_j the PCA basis of the value matrix (Sec. 4).
 * System (eqs. (system), (system_new)): H W = F, solved through the normal
 * equations H^T H W = H^T F with CG + additive Schwarz or GMRES + restricted
 * additive Schwarz (Sec. 3).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers on the current HIP device, contiguous,
 *     FP64, unless the comment says "host".  Point and matrix arrays are
 *     row-major; multi-right-hand-side arrays are (rows, k) row-major (the
 *     right-hand-side index is fastest).
 *   - The caller owns every buffer it passes; the library copies what it keeps.
 *     The handle owns all internal device memory until rann_dd_destroy, which
 *     returns it to a process-wide cache of device blocks (reused by later
 *     handles on the same device; rann_dd_trim_cache gives it back to HIP).
 *   - Work is ordered on the stream given to rann_dd_assemble.  Calls marked
 *     "synchronous" return after the device work has finished.
 *   - Return value: 0 = success; negative = error (outputs undefined, message in
 *     rann_dd_last_error()); positive = warning (outputs valid).
 *   - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef RANN_DD_H
#define RANN_DD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RANN_API __attribute__((visibility("default")))

/* status codes */
#define RANN_OK            0
#define RANN_EINVAL       (-1)  /* invalid argument or descriptor */
#define RANN_ENOMEM       (-2)  /* device allocation failed */
#define RANN_EDEVICE      (-3)  /* HIP runtime error */
#define RANN_ENAN         (-4)  /* NaN or Inf in an input or in the iteration */
#define RANN_EBREAKDOWN   (-5)  /* Krylov breakdown (<p, H^T H p> <= 0 in FP64) */
#define RANN_ENOTCONV      1    /* iteration limit reached; outputs hold the last iterate */
#define RANN_WRANKTIE      2    /* a PCA eigenvalue lies within relative 1e-6 of the threshold */

/* precision of the preconditioner path (the Krylov vectors, dot products,
 * H and the residual are FP64 in both) */
#define RANN_FP64          0
#define RANN_MIXED         1    /* the local inverses are stored as FP32 triangular
                                   factors Y_i (A_i^{-1} = Y_i^T Y_i) and, when no
                                   block is wider than 6 tiles of 64, also as
                                   A_i^{-1} rounded to FP32; for k >= 16 right-hand
                                   sides they are applied in FP32 on the matrix
                                   cores (A_i^{-1} in one pass where it is stored),
                                   with FP64 accumulation below that */

/* Schwarz blocks: which subdomains' columns block i selects (Sec. 3, R_i) */
#define RANN_STENCIL_SELF  0    /* subdomain i only (block Jacobi) */
#define RANN_STENCIL_FACE  1    /* i and its face neighbours */
#define RANN_STENCIL_FULL  2    /* all subdomains whose supports intersect that of i */

#define RANN_PRECOND_NONE  0
#define RANN_PRECOND_AS    1    /* sum_i R_i^T A_i^{-1} R_i */
#define RANN_PRECOND_RAS   2    /* sum_i R_i^T D_i A_i^{-1} R_i, D_i Boolean: the columns
                                   of each subdomain belong to the first block (in
                                   increasing block order) whose stencil holds it */
#define RANN_PRECOND_SAS   3    /* D_i = 1 / multiplicity (Sec. 5, Example 1) */

#define RANN_PCA_REL_EIG   0    /* keep eigenvalues of Psi^T Psi above tol * largest */
#define RANN_PCA_ABS_SIGMA 1    /* keep singular values of Psi above tol (paper's tau) */
#define RANN_PCA_OFF       2    /* no truncation, V = I */

#define RANN_METHOD_CG     0
#define RANN_METHOD_GMRES  1        /* left-preconditioned (paper Sec. 5) */
#define RANN_METHOD_GMRES_RIGHT 2   /* right-preconditioned: minimises the true residual */
#define RANN_METHOD_CGS    3        /* conjugate gradients squared (Sec. 5, Table 1b) */
#define RANN_METHOD_BICG   4        /* biconjugate gradients (Sec. 5, Table 1b); applies the
                                       transposed preconditioner M^{-T} beside M^{-1} */

#define RANN_LIN_NEWTON    0        /* Newton (Gauss-Newton) linearisation of g */
#define RANN_LIN_PICARD    1        /* Picard: g(u) = gamma_0 + u q(u), q frozen */
#define RANN_MAX_GAMMA     16       /* coefficients of the polynomial reaction */

typedef struct rann_dd_handle rann_dd_handle;

/* Problem description (paper eq. (1), Sec. 2 local networks, Sec. 5 layout). */
typedef struct rann_dd_desc {
    int32_t d;                /* dimension (space-time counts t), 1..4 */
    int32_t l[4];             /* subdomains per dimension; J = prod l[i]; subdomain
                                 index j = c_0 + l_0 (c_1 + l_1 (...)) */
    const double* mu;         /* host, sum(l) centres: dimension 0's l[0] centres,
                                 then dimension 1's, ...; strictly increasing */
    double sigma[4];          /* support half-width per dimension (> 0) */
    const int32_t* m;         /* host, J hidden widths (1..1024) */
    const double* R;          /* device, sum(m) x d: rows of R_j (weights acting on
                                 the normalised input), subdomain after subdomain;
                                 sum(m) x inner_w[n_inner-1] with inner layers */
    const double* b;          /* device, sum(m) biases */
    int64_t n_int;            /* interior collocation points (>= 1) */
    const double* X_int;      /* device, n_int x d */
    const double* a;          /* device, n_int x d diffusion coefficients */
    const double* beta;       /* device, n_int x d advection coefficients */
    const double* c;          /* device, n_int reaction coefficient */
    int64_t n_bnd;            /* boundary points (>= 0) */
    const double* X_bnd;      /* device, n_bnd x d, or NULL when n_bnd == 0 */
    double lambda_B;          /* weight of the boundary rows (> 0) */
    const double* Lfun;       /* device, (n_int + n_bnd) x (1 + 2d): the constraining
                                 multiplier L and its first and pure second
                                 derivatives at every point (eq. (operator)), or NULL
                                 for L == 1 */
    int32_t precision;        /* RANN_FP64 or RANN_MIXED */
    int32_t stencil;          /* RANN_STENCIL_* */
    int32_t precond;          /* RANN_PRECOND_* */
    /* Several fixed hidden layers (paper Sec. 2, eq. (net)): each subdomain
       network applies n_inner tanh layers f(y) = tanh(R_i y + b_i) of widths
       inner_w[0..n_inner-1] to the normalised input before the last hidden
       layer, whose weights R then act on the last inner output (R is
       sum(m) x inner_w[n_inner-1]).  n_inner = 0 (one hidden layer): the
       fields below are ignored.  Limits: n_inner 0..3, widths 1..64. */
    int32_t n_inner;
    int32_t inner_w[3];
    const double* R_inner;    /* device: subdomain after subdomain, layer after layer, the
                                 w_i x w_{i-1} weights row-major (w_0 = d) */
    const double* b_inner;    /* device: subdomain after subdomain, layer after layer, the w_i
                                 biases */
} rann_dd_desc;

typedef struct rann_dd_solve_opts {
    double tol;               /* relative true normal residual ||H^T(F - H W)|| / ||H^T F|| */
    int32_t maxiter;          /* iteration limit (>= 1) */
    int32_t method;           /* RANN_METHOD_CG (AS), RANN_METHOD_GMRES, RANN_METHOD_GMRES_RIGHT,
                                 RANN_METHOD_CGS or RANN_METHOD_BICG */
    int32_t restart;          /* GMRES restart length (1..128); CGS and BiCG with
                                 RANN_MIXED: longest refinement cycle, after which
                                 the right-hand side restarts from its FP64
                                 residual (<= 0: no limit) */
    int32_t check_every;      /* host convergence check cadence (>= 1) */
} rann_dd_solve_opts;

typedef struct rann_dd_stats {
    int32_t iterations;       /* iterations taken (max over right-hand sides) */
    int32_t converged;        /* number of right-hand sides that met tol */
    double max_rel_residual;  /* max over RHS of the true FP64 relative normal residual */
    double* rel_residual;     /* host, k entries or NULL: per-RHS true residual */
    int32_t* rhs_iterations;  /* host, k entries or NULL: per-RHS iteration counts */
    int32_t shifts;           /* local factors that needed a diagonal shift */
    double setup_ms[4];       /* assemble, pca, factor, (unused) phase times */
} rann_dd_stats;

/* Launch parameters of the Krylov step (rann_dd_autotune picks them by timing).
 * tile_grid and use_graph change the speed only (bitwise the same results);
 * red_cap also sets the summation order of the dot products (results agree to
 * rounding). */
typedef struct rann_dd_tuning {
    int32_t tile_grid;        /* persistent workgroups of the FP64 local solves with one or two
                                 right-hand sides (64..4096; default 768) */
    int32_t red_cap;          /* most workgroups of the CG vector kernels (32..240; default 240)
                                 (their per-workgroup dot-product partials are summed by every
                                 consumer workgroup) */
    int32_t use_graph;        /* 1: the launches of each CG check window are captured once into
                                 a HIP graph and replayed (default); 0: launched one by one */
    int32_t pca_subspace;     /* 1 (default): rann_dd_pca finds the leading eigenvectors by
                                 subspace iteration (blocks of 64) when every hidden width is at
                                 least 128 and some width exceeds 480, and returns to the direct
                                 solver when a subdomain keeps more than 48 eigenvectors; 0: the
                                 direct tridiagonal eigensolver.  Set before rann_dd_pca.  With
                                 the subspace path the eigenvalues past each block are NaN. */
    int32_t gram32;           /* RANN_MIXED only, set before rann_dd_pca: 1 = the operator rows
                                 are also rounded to FP32 and the local Gram blocks of the
                                 Schwarz blocks A_i formed from them on the FP32 matrix cores
                                 with FP32 accumulation (the equilibrated Cholesky with its
                                 shift stays FP64); 0 (default) = A_i from the FP64 Gram blocks.
                                 The normal matrix and every residual use FP64 rows either way. */
    int32_t reserved;         /* 0 */
} rann_dd_tuning;

/* Layout sizes, for callers that allocate W, F and the diagnostic arrays. */
typedef struct rann_dd_info {
    int32_t d, J;
    int64_t N_int, N_bnd, N;  /* rows */
    int64_t P;                /* columns after PCA (0 before rann_dd_pca) */
    int64_t pairs;            /* sum_j n_j: stored rows of all blocks */
    int64_t nnz;              /* sum_j n_j p_j: stored entries of H */
    int64_t sum_m;            /* sum_j m_j */
    int64_t factor_elems;     /* stored entries of the local inverse operators */
    int32_t max_q;            /* largest Schwarz block */
    int32_t pca_done;
    int64_t normal_elems;     /* stored entries of the assembled normal matrix H^T H */
    int32_t cg_graphs;        /* captured CG check-window graphs held by the handle */
    int32_t graph_failed;     /* 1 when a capture failed (windows run eagerly since) */
} rann_dd_info;

/* Steps 1-3 of Algorithm 1 (paper Sec. 4): bin the points into the subdomain
 * supports (strict |x_i - mu_i| < sigma_i (1 - 1e-12) in every dimension), and
 * evaluate the window partition of unity with its derivatives and the operator
 * coefficients at every (point, subdomain) pair.  Synchronous.  Every input is
 * copied; the caller may free it on return.  Errors: RANN_EINVAL for a bad
 * descriptor or a point outside every support; RANN_ENOMEM; RANN_EDEVICE. */
RANN_API int rann_dd_assemble(const rann_dd_desc* desc, void* hip_stream, rann_dd_handle** out);

/* Step 4-6 set-up (Sec. 4, Sec. 3): local value-matrix Gram Psi_j^T Psi_j, its
 * FP64 symmetric eigendecomposition, truncation (mode RANN_PCA_*, threshold
 * tol), the operator rows H_j = A[L w_j Phi_j] V_j, the local Gram blocks
 * A_i = R_i H^T H R_i^T and their equilibrated Cholesky-based inverses.
 *   p_force  host J counts or NULL: override the truncation counts.
 *   V_force  device, sum_j m_j p_j (row-major m_j x p_j per subdomain, with p
 *            from p_force) or NULL: inject a PCA basis (requires p_force).
 *   p_out    host J or NULL: receives p_j.
 * Synchronous.  Returns RANN_WRANKTIE if an eigenvalue lies within relative
 * 1e-6 of the threshold.  Device scratch during the call: the value matrices
 * and, with one hidden layer, their tanh values for the operator rows
 * (sum_j n_j m_j doubles each, n_j the points in support j). */
RANN_API int rann_dd_pca(rann_dd_handle* h, double tol, int32_t mode, const int32_t* p_force,
                const double* V_force, int32_t* p_out);

/* Steps 6-7: solve min ||H W - F||_2 for k right-hand sides through the normal
 * equations (Sec. 2) with the handle's preconditioner.
 *   F   device (N, k): interior rows f - A[G], then boundary rows g - G
 *       (unscaled; the library multiplies them by lambda_B).
 *   W0  device (P, k) initial guess or NULL (zero).
 *   W   device (P, k) output, coefficients in the PCA basis.
 *   st  host or NULL; when given, the call synchronises and fills it.
 * Returns RANN_ENOTCONV when maxiter is reached, RANN_EBREAKDOWN, RANN_ENAN. */
RANN_API int rann_dd_solve(rann_dd_handle* h, const double* F, int32_t k, const double* W0,
                  const rann_dd_solve_opts* opts, double* W, rann_dd_stats* st);

/* Adjoint of rann_dd_solve: dF = H (H^T H)^{-1} dW with the boundary rows
 * multiplied by lambda_B, i.e. the gradient with respect to the unscaled
 * (f, g) rows of F of any loss whose gradient with respect to W is dW.
 *   dW device (P, k); dF device (N, k).
 * CG stops on its recurrence residual; CGS and BiCG confirm on the recomputed
 * FP64 residual ||dW - H^T H z|| / ||dW||, whose floor for a dW with weight on
 * the smallest singular directions is near 1e-16 kappa(H^T H). */
RANN_API int rann_dd_solve_backward(rann_dd_handle* h, const double* dW, int32_t k,
                           const rann_dd_solve_opts* opts, double* dF, rann_dd_stats* st);

/* u(x_q) = sum_j L(x_q) w_j(x_q) W_j . (V_j^T Phi_j(x_q)) at M probe points
 * (eq. (netdd) without G).  Xq device (M, d); Lq device (M) or NULL (L == 1);
 * W device (P, k); U device (M, k). */
RANN_API int rann_dd_eval(rann_dd_handle* h, const double* Xq, int64_t M, const double* Lq,
                 const double* W, int32_t k, double* U);

/* Transpose of rann_dd_eval: dW = Pmat^T dU.  dU device (M, k); dW device (P, k). */
RANN_API int rann_dd_eval_T(rann_dd_handle* h, const double* Xq, int64_t M, const double* Lq,
                   const double* dU, int32_t k, double* dW);

/* One Picard or Newton linearisation of a semilinear problem A[u] + g(u) = f
 * with g(u) = sum_{p < n_gamma} gamma[p] u^p (Sec. 2, the remark after eq.
 * (sum): each step of the nonlinear iteration is one linear least-squares
 * problem).  From the values u (device, n: the current iterate at the n
 * interior collocation points, e.g. from rann_dd_eval at X_int), the reaction
 * c0 (device, n) and source f (device, n) of the linear part, it writes the
 * reaction c_out and interior right-hand side f_out (device, n) of the next
 * step's linear problem:
 *   RANN_LIN_NEWTON: c_out = c0 + g'(u),  f_out = f - g(u) + g'(u) u
 *   RANN_LIN_PICARD: c_out = c0 + q(u),   f_out = f - gamma[0],  g = gamma[0] + u q(u)
 * gamma: host, 1 <= n_gamma <= RANN_MAX_GAMMA.  u_prev (device, n) or NULL;
 * when given with inc (host), *inc = ||u - u_prev|| / ||u|| (synchronous).
 * Runs on the handle's stream (h needs no PCA), or on the default stream when
 * h is NULL (then without the increment).  RANN_EINVAL for bad sizes. */
RANN_API int rann_dd_linearize(rann_dd_handle* h, const double* u, const double* c0, const double* f,
                  int64_t n, const double* gamma, int32_t n_gamma, int32_t mode, double* c_out,
                  double* f_out, const double* u_prev, double* inc);

/* Raw-neuron coefficients c_j = V_j W_j (device, sum_j m_j x k). */
RANN_API int rann_dd_coeffs(rann_dd_handle* h, const double* W, int32_t k, double* c);

/* Products with the assembled operators, for verification:
 * y = H x (x (P,k), y (N,k));  x = H^T y;  s = H^T H x;  z = M^{-1} r. */
RANN_API int rann_dd_matvec(rann_dd_handle* h, const double* x, int32_t k, double* y);
RANN_API int rann_dd_rmatvec(rann_dd_handle* h, const double* y, int32_t k, double* x);
RANN_API int rann_dd_apply_normal(rann_dd_handle* h, const double* x, int32_t k, double* s);
RANN_API int rann_dd_apply_precond(rann_dd_handle* h, const double* r, int32_t k, double* z);
/* z = M^{-1} r as rann_dd_apply_precond computes it, without allocating device
 * memory: for callers that cannot allocate (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  The local solves use a
 * static device array of the library (32 MiB on every device the library runs
 * on, held until the process ends) instead of allocated scratch; a problem that
 * needs more ((2 sum_i q_i + 2 S) k doubles, S the slots of the row and column
 * sums) returns RANN_EINVAL.  r, z device (P, k), k >= 1, not aliased.
 * Asynchronous on the handle's stream (no synchronisation, no event).  Every call
 * on one GPU shares that array and leaves its contents behind: calls that may
 * overlap on one GPU (other streams, threads or handles) race and must be
 * serialised by the caller. */
RANN_API int rann_dd_apply_precond_noalloc(rann_dd_handle* h, const double* r, int32_t k, double* z);
/* z = M^{-T} r, the transposed Schwarz preconditioner that BiCG's shadow
 * recurrence applies (Sec. 5, Table 1b): the weights D_i move from the local
 * results onto the restricted input, sum_i R_i^T A_i^{-1} D_i R_i r.  r, z
 * device (P, k), k >= 1, not aliased.  Equal to rann_dd_apply_precond for AS and
 * no preconditioner.  Synchronous. */
RANN_API int rann_dd_apply_precond_T(rann_dd_handle* h, const double* r, int32_t k, double* z);

/* Current launch parameters of a handle / replace them (RANN_EINVAL outside the
 * stated ranges).  Host-only; no device work. */
RANN_API int rann_dd_get_tuning(const rann_dd_handle* h, rann_dd_tuning* out);
RANN_API int rann_dd_set_tuning(rann_dd_handle* h, const rann_dd_tuning* t);
/* Autotuner of the Krylov step: times `iters` CG iterations with k right-hand
 * sides (a fixed pseudo-random right-hand side, tolerance 0) for every candidate
 * of tile_grid (FP64 with k <= 2 only), red_cap and use_graph, keeps the fastest
 * on the handle and returns it in *best (host) with its time per iteration in
 * *best_us (host, may be NULL).  Synchronous; needs rann_dd_pca; 1 <= k <= 256,
 * 2 <= iters <= 1000. */
RANN_API int rann_dd_autotune(rann_dd_handle* h, int32_t k, int32_t iters, rann_dd_tuning* best,
                              double* best_us);

/* Sizes; valid after rann_dd_assemble (P, nnz after rann_dd_pca). */
RANN_API int rann_dd_get_info(const rann_dd_handle* h, rann_dd_info* out);

/* Copies of internal arrays, for verification.  Host arrays:
 *   row_off (J+1), rows (pairs): the row sets S_j (sorted global row indices);
 *   p (J).  Device arrays: blocks (nnz, H_j row-major n_j x p_j, subdomain after
 *   subdomain); V (sum_j m_j p_j, row-major m_j x p_j); eig (sum_j m_j,
 *   descending eigenvalues of Psi_j^T Psi_j).  Any pointer may be NULL. */
RANN_API int rann_dd_get_layout(const rann_dd_handle* h, int64_t* row_off, int32_t* rows, int32_t* p);
RANN_API int rann_dd_get_arrays(const rann_dd_handle* h, double* blocks, double* V, double* eig);

/* Host copy of the Schwarz block sizes q_i (J entries; zeros without a
 * preconditioner).  Valid after rann_dd_pca. */
RANN_API int rann_dd_get_blocks(const rann_dd_handle* h, int64_t* q);

/* Kernel timing for measurement (process-wide, off by default).  When enabled,
 * the main kernels are bracketed by HIP events on the stream they run on;
 * rann_dd_ktime_enable(on) also clears the accumulated times.  Query by kernel
 * name ("k_eig", "k_factor", "k_pca_gram", "k_feat_rows", "k_normal",
 * "k_local_gram", "k_Hx", "k_HTy_part", "k_tile_apply", "k_slot_reduce"): total milliseconds
 * and number of launches since the last enable.  Query synchronises on the
 * recorded events. */
RANN_API int rann_dd_ktime_enable(int32_t on);
RANN_API int rann_dd_ktime_query(const char* name, double* total_ms, int64_t* launches);

/* Release the handle and its device memory (NULL is ignored).  The memory goes
 * to the process-wide block cache. */
RANN_API void rann_dd_destroy(rann_dd_handle* h);

/* Free every cached device block and pinned staging buffer not held by a live
 * handle, after a device synchronisation.  Returns the number of bytes
 * released.  Not to be called while another thread uses the library. */
RANN_API size_t rann_dd_trim_cache(void);

/* Message of the last error on the calling thread ("" if none). */
RANN_API const char* rann_dd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RANN_DD_H */
