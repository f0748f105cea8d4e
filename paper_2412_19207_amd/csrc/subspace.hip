// Eigen-PCA by subspace iteration with Rayleigh-Ritz (paper Sec. 4: the leading
// eigenvectors of the value Gram G_j = Psi_j^T Psi_j above a threshold).
//
// The truncation keeps p_j of the m_j eigenvectors (about a tenth on the
// benchmark workloads), so a full tridiagonalisation of every G_j, whose
// column-by-column panel reduction reads the trailing matrix once per column,
// does far more work than needed.  Here each subdomain keeps an orthonormal
// block Q_j of s_j > p_j columns:
//
//   Y = G Q,  T = Q^T Y,  T = C Theta C^T (FP64 symmetric eigensolver on s x s),
//   U = Q C (Ritz vectors),  Z = Y C = G U,  residuals r_k = Z_k - theta_k U_k,
//   next Q = orthonormal basis of Z (columns scaled to unit norm),
//
// until the Ritz pairs that decide the truncation (k <= p_j, and p_j + 1) have
// residuals below 10 m_j u theta_1 and the block has at least kMargin columns
// beyond p_j (else the direct tridiagonal path takes over).  The count p_j
// comes from the Ritz values with
// the same threshold as the direct path.  The orthonormal bases come from
// shifted Cholesky QR (three passes, the first with a diagonal shift of
// 11 (m s + s (s + 1)) u tr(X^T X)), which is backward stable like Householder
// QR for any conditioning of the block.  The products are batched FP64
// matrix-core GEMMs over all subdomains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace rdd {

namespace {

constexpr int kS0 = 64;        // first block width
constexpr int kMargin = 16;    // columns beyond p_j the block keeps
// Widest block.  The Rayleigh-Ritz eigensolve and the Cholesky QR of a block
// cost about as much per round as they save once the block passes about a
// hundred columns (measured: the 2D Poisson workload, p_j about 81 of 300,
// took 36 ms with blocks of 144 against 9 ms for the direct path), so a block
// keeps 64 columns and subdomains that keep more than 48 eigenvectors send
// the whole batch to the direct path.
constexpr int kSMax = 64;
constexpr int kMaxRounds = 16; // subspace steps before giving up
constexpr int kCT = 1024;      // threads of the small factorisation kernels

// one batched product: C = alpha op(A) B + beta C, row-major, per subdomain
struct BG {
    int64_t a, b, c;  // offsets into the three base arrays
    int M, N, K, lda, ldb, ldc, pad;
};

// 64 x 64 output tile (task.y, task.z) of product task.x
template <bool TA>
__global__ void __launch_bounds__(256) k_bgemm(const int4* __restrict__ tasks, const BG* __restrict__ d,
                                               const double* __restrict__ A, const double* __restrict__ B,
                                               double* __restrict__ C, double alpha, double beta) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const int4 tk = tasks[blockIdx.x];
    const BG g = d[tk.x];
    const int64_t m0 = (int64_t)tk.y * kTM, n0 = (int64_t)tk.z * kTN;
    const int mv = (int)std::min<int64_t>(kTM, g.M - m0), nv = (int)std::min<int64_t>(kTN, g.N - n0);
    TileAcc<double> acc;
    acc.zero();
    if (TA)  // op(A) = A^T with A stored K x M: element (k, m) = A[k lda + m]
        tile_gemm<double, true, true>(acc, As, Bs, A + g.a, g.lda, 0, m0, mv, B + g.b, g.ldb, 0, n0, nv, g.K);
    else     // A stored M x K: element (k, m) = A[m lda + k]
        tile_gemm<double, false, true>(acc, As, Bs, A + g.a, g.lda, m0, 0, mv, B + g.b, g.ldb, 0, n0, nv, g.K);
    double* Cj = C + g.c;
    acc.each([&](int r, int c, double v) {
        if (r < mv && c < nv) {
            double* o = Cj + (m0 + r) * g.ldc + n0 + c;
            *o = (beta == 0.0) ? alpha * v : fma(beta, *o, alpha * v);
        }
    });
}

// X_j[r][c] for c >= col0: pseudo-random values in [-1, 1) from a 64-bit mix of
// (j, r, c) (SplitMix64), a fixed start block
__global__ void k_seed(const int32_t* __restrict__ mv, const int32_t* __restrict__ sv,
                       const int64_t* __restrict__ xo, const int32_t* __restrict__ col0v, double* __restrict__ X) {
    const int j = blockIdx.x;
    const int m = mv[j], s = sv[j];
    const int col0 = col0v ? col0v[j] : 0;
    for (int64_t e = threadIdx.x; e < (int64_t)m * s; e += blockDim.x) {
        const int r = (int)(e / s), c = (int)(e % s);
        if (c < col0) continue;
        uint64_t z = ((uint64_t)j << 40) ^ ((uint64_t)r << 20) ^ (uint64_t)c;
        z = z * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        X[xo[j] + e] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

// T = (T + T^T) / 2 for every s_j x s_j block
__global__ void k_symm(const int32_t* __restrict__ sv, const int64_t* __restrict__ to, double* __restrict__ T) {
    const int j = blockIdx.x;
    const int s = sv[j];
    double* Tj = T + to[j];
    for (int64_t e = threadIdx.x; e < (int64_t)s * s; e += blockDim.x) {
        const int r = (int)(e / s), c = (int)(e % s);
        if (c <= r) continue;
        const double v = 0.5 * (Tj[(int64_t)r * s + c] + Tj[(int64_t)c * s + r]);
        Tj[(int64_t)r * s + c] = v;
        Tj[(int64_t)c * s + r] = v;
    }
}

// ||column c||^2 of an m x s block (s <= 64), 256 threads: column tid % 64,
// rows tid / 64, + 4, ...; the four partial sums meet in LDS
__device__ inline double col_sumsq(const double* A, const double* B, const double* thv, int m, int s,
                                   double* sh) {
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    double nn = 0.0;
    if (c < s) {
        const double th = thv ? thv[c] : 0.0;
        for (int r = g; r < m; r += 4) {
            const double d = B ? A[(int64_t)r * s + c] - th * B[(int64_t)r * s + c] : A[(int64_t)r * s + c];
            nn = fma(d, d, nn);
        }
    }
    sh[threadIdx.x] = nn;
    __syncthreads();
    const double tot = (sh[c] + sh[64 + c]) + (sh[128 + c] + sh[192 + c]);
    __syncthreads();
    return tot;
}

// columns of Z scaled to unit length (zero columns stay zero), into X
__global__ void __launch_bounds__(256) k_colscale(const int32_t* __restrict__ mv, const int32_t* __restrict__ sv,
                                                  const int64_t* __restrict__ xo, const double* __restrict__ Z,
                                                  double* __restrict__ X) {
    __shared__ double sh[256];
    const int j = blockIdx.x;
    const int m = mv[j], s = sv[j];
    const double* Zj = Z + xo[j];
    double* Xj = X + xo[j];
    const double nn = col_sumsq(Zj, nullptr, nullptr, m, s, sh);
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    if (c < s) {
        const double f = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int r = g; r < m; r += 4) Xj[(int64_t)r * s + c] = Zj[(int64_t)r * s + c] * f;
    }
}

// Cholesky R^T R = S + shift I of the s x s Gram S (s <= kSMax; the lower
// factor L = R^T in LDS) and Rinv = R^{-1} (upper, written whole to global
// memory); the shift is 11 (m s + s (s + 1)) u tr(S) when `shifted`.  Column k
// is eliminated in one pass (each thread scales the pivot column's entries it
// needs itself), one barrier per column.  A non-positive pivot sets flags[0].
// L_true^{-1} comes from forward substitution organised by columns of L: once
// rows 0 .. l of the inverse have all their updates, row l updates every
// later row (a rank-one step over the whole lower triangle, one barrier per
// column), and each row is divided by its pivot at the end.  Entries are
// indexed by e = 64 r + c over the kSMax x kSMax square.
__global__ void __launch_bounds__(kCT) k_chol_inv(const int32_t* __restrict__ mv, const int32_t* __restrict__ sv,
                                                  const int64_t* __restrict__ to, const double* __restrict__ S,
                                                  double* __restrict__ Rinv, int shifted, int32_t* __restrict__ flags) {
    static_assert(kSMax == 64, "entries indexed by 64 r + c");
    __shared__ double L[kSMax][kSMax + 1];
    __shared__ double X[kSMax][kSMax + 1];  // L_true^{-1}, lower
    __shared__ double red[kCT / 64];
    __shared__ double sdiag[kSMax];
    const int j = blockIdx.x;
    const int s = sv[j], m = mv[j];
    const double* Sj = S + to[j];
    double* Rj = Rinv + to[j];
    const int tid = threadIdx.x;
    constexpr int kPer = kSMax * kSMax / kCT;  // entries per thread
    double tr = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + kCT * u, r = e >> 6, c = e & 63;
        if (r < s && c < s) {
            const double v = Sj[r * s + c];
            L[r][c] = v;
            if (r == c) tr += v;
        }
    }
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off);
    if ((tid & 63) == 0) red[tid >> 6] = tr;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kCT / 64; ++w) t += red[w];
    const double shift = shifted ? 11.0 * ((double)m * s + (double)s * (s + 1)) * 1.1102230246251565e-16 * t : 0.0;
    for (int r = tid; r < s; r += kCT) L[r][r] += shift;
    __syncthreads();
    for (int k = 0; k < s; ++k) {
        double dk = L[k][k];
        if (!(dk > 0.0)) {
            if (tid == 0) flags[0] = 1;
            dk = 1e-300;
        }
        const double inv = 1.0 / dk;  // L[r][c] -= L[r][k] L[c][k] / d_k
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + kCT * u, r = e >> 6, c = e & 63;
            if (c > k && c <= r && r < s) L[r][c] -= L[r][k] * L[c][k] * inv;
        }
        __syncthreads();
    }
    // the factor is L_true[r][k] = L[r][k] / sqrt(d_k), d_k = L[k][k]
    for (int k = tid; k < s; k += kCT) sdiag[k] = sqrt(L[k][k] > 0.0 ? L[k][k] : 1e-300);
    __syncthreads();
    // the factor's entries L_true[r][c] = L[r][c] / sqrt(d_c) below the
    // diagonal; X starts as the identity
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + kCT * u, r = e >> 6, c = e & 63;
        if (r < s && c < r) L[r][c] /= sdiag[c];
        X[r][c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    // step l: row l of X is complete up to its division by the pivot; every
    // row i > l takes X[i][c] -= L_true[i][l] X[l][c] / d_l for c <= l
    for (int l = 0; l + 1 < s; ++l) {
        const double invd = 1.0 / sdiag[l];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + kCT * u, i = e >> 6, c = e & 63;
            if (i > l && i < s && c <= l) X[i][c] -= L[i][l] * (X[l][c] * invd);
        }
        __syncthreads();
    }
    // Rinv = L_true^{-T}: Rinv[r][c] = X[c][r] / d_c for c >= r
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int e = tid + kCT * u, r = e >> 6, c = e & 63;
        if (r < s && c < s) Rj[r * s + c] = (c < r) ? 0.0 : X[c][r] / sdiag[c];
    }
}

// res[so + k] = || Z_k - theta_k U_k || for every column k of every block
__global__ void __launch_bounds__(256) k_resid(const int32_t* __restrict__ mv, const int32_t* __restrict__ sv,
                                               const int64_t* __restrict__ xo, const int64_t* __restrict__ so,
                                               const double* __restrict__ Z, const double* __restrict__ U,
                                               const double* __restrict__ theta, double* __restrict__ res) {
    __shared__ double sh[256];
    const int j = blockIdx.x;
    const int m = mv[j], s = sv[j];
    const double nn = col_sumsq(Z + xo[j], U + xo[j], theta + so[j], m, s, sh);
    if (threadIdx.x < s) res[so[j] + threadIdx.x] = sqrt(nn);
}

// The first p_j Ritz vectors as the columns of Yfull (row-major m x m at g_off,
// the layout of the direct path) and the Ritz values as the eigenvalues
// (descending; NaN past the block, which this path does not compute)
__global__ void k_pack(const int32_t* __restrict__ mv, const int32_t* __restrict__ sv,
                       const int32_t* __restrict__ pv, const int64_t* __restrict__ xo,
                       const int64_t* __restrict__ so, const int64_t* __restrict__ g_off,
                       const int64_t* __restrict__ m_off, const double* __restrict__ U,
                       const double* __restrict__ theta, double* __restrict__ Yfull, double* __restrict__ eig) {
    const int j = blockIdx.x;
    const int m = mv[j], s = sv[j], p = pv[j];
    for (int64_t e = threadIdx.x; e < (int64_t)m * p; e += blockDim.x) {
        const int r = (int)(e / p), c = (int)(e % p);
        Yfull[g_off[j] + (int64_t)r * m + c] = U[xo[j] + (int64_t)r * s + c];
    }
    for (int c = threadIdx.x; c < m; c += blockDim.x)
        eig[m_off[j] + c] = (c < s) ? theta[so[j] + c] : __builtin_nan("");
}

}  // namespace

namespace {

struct Batch {
    int J = 0;
    std::vector<int32_t> m, s;
    std::vector<int64_t> xo, to, so;  // offsets: m s, s s, s
    int64_t xtot = 0, ttot = 0, stot = 0;
};

struct Gemm {
    BG* d = nullptr;
    int4* tasks = nullptr;
    int64_t n = 0;
};

int make_gemm(Handle& h, const std::vector<BG>& g, Gemm& out) {
    std::vector<int4> t;
    for (int j = 0; j < (int)g.size(); ++j) {
        if (g[j].M <= 0 || g[j].N <= 0) continue;
        const int tm = (g[j].M + kTM - 1) / kTM, tn = (g[j].N + kTN - 1) / kTN;
        for (int a = 0; a < tm; ++a)
            for (int b = 0; b < tn; ++b) t.push_back(make_int4(j, a, b, 0));
    }
    out.n = (int64_t)t.size();
    RDD_TRY(dev_alloc(h, &out.d, g.size()));
    RDD_TRY(dev_alloc(h, &out.tasks, std::max<size_t>(t.size(), 1)));
    RDD_TRY(upload(h, out.d, g.data(), sizeof(BG) * g.size()));
    if (!t.empty()) RDD_TRY(upload(h, out.tasks, t.data(), sizeof(int4) * t.size()));
    return RANN_OK;
}

int run_gemm(Handle& h, const Gemm& g, bool ta, const double* A, const double* B, double* C) {
    if (g.n == 0) return RANN_OK;
    if (ta)
        hipLaunchKernelGGL(k_bgemm<true>, dim3((unsigned)g.n), dim3(256), 0, h.stream, g.tasks, g.d, A, B, C, 1.0,
                           0.0);
    else
        hipLaunchKernelGGL(k_bgemm<false>, dim3((unsigned)g.n), dim3(256), 0, h.stream, g.tasks, g.d, A, B, C, 1.0,
                           0.0);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace

int eig_subspace(Handle& h, const double* G, const std::vector<int64_t>& g_off, const int64_t* d_g_off,
                 double tol, int mode, int32_t* d_p, double* d_eig, int32_t* d_flags, double* Yfull) {
    const int J = h.geo.J;
    KTimer kt_(h.stream, "k_eig");
    Batch bt;
    bt.J = J;
    bt.m.assign(h.m.begin(), h.m.end());
    bt.s.resize(J);
    bt.xo.assign(J + 1, 0);
    bt.to.assign(J + 1, 0);
    bt.so.assign(J + 1, 0);
    std::vector<int64_t> e_off(J + 1, 0);
    for (int j = 0; j < J; ++j) {
        bt.s[j] = std::min<int32_t>(bt.m[j], kSMax);
        bt.xo[j + 1] = bt.xo[j] + (int64_t)bt.m[j] * bt.s[j];
        bt.to[j + 1] = bt.to[j] + (int64_t)bt.s[j] * bt.s[j];
        bt.so[j + 1] = bt.so[j] + bt.s[j];
        e_off[j + 1] = e_off[j] + eig_scratch_elems(bt.s[j]);
    }
    std::vector<void*> owned;  // freed on every exit
    auto release = [&]() {
        for (void* p : owned) dev_free(h, p);
        owned.clear();
    };
    int rc = RANN_OK;
    auto alloc = [&](auto** ptr, size_t n) {
        if (rc == RANN_OK) rc = dev_alloc(h, ptr, std::max<size_t>(n, 1));
        if (rc == RANN_OK) owned.push_back(*ptr);
    };
    int32_t *d_m = nullptr, *d_s = nullptr, *d_fl = nullptr;
    int64_t *d_xo = nullptr, *d_to = nullptr, *d_so = nullptr, *d_eoff = nullptr;
    double *X = nullptr, *Q = nullptr, *Y = nullptr, *U = nullptr, *Z = nullptr;
    double *T = nullptr, *Cm = nullptr, *Rinv = nullptr, *Sg = nullptr, *theta = nullptr, *res = nullptr, *scr = nullptr;
    alloc(&d_m, J);
    alloc(&d_s, J);
    alloc(&d_fl, 2);
    alloc(&d_xo, J + 1);
    alloc(&d_to, J + 1);
    alloc(&d_so, J + 1);
    alloc(&d_eoff, J + 1);
    for (double** b : {&X, &Q, &Y, &U, &Z}) alloc(b, (size_t)bt.xo[J]);
    for (double** b : {&T, &Cm, &Rinv, &Sg}) alloc(b, (size_t)bt.to[J]);
    alloc(&theta, (size_t)bt.so[J]);
    alloc(&res, (size_t)bt.so[J]);
    alloc(&scr, (size_t)e_off[J]);
    if (rc == RANN_OK) rc = upload(h, d_m, bt.m.data(), sizeof(int32_t) * J);
    if (rc == RANN_OK) rc = upload(h, d_s, bt.s.data(), sizeof(int32_t) * J);
    if (rc == RANN_OK) rc = upload(h, d_xo, bt.xo.data(), sizeof(int64_t) * (J + 1));
    if (rc == RANN_OK) rc = upload(h, d_to, bt.to.data(), sizeof(int64_t) * (J + 1));
    if (rc == RANN_OK) rc = upload(h, d_so, bt.so.data(), sizeof(int64_t) * (J + 1));
    if (rc == RANN_OK) rc = upload(h, d_eoff, e_off.data(), sizeof(int64_t) * (J + 1));
    // the three product shapes: G Q (m x s x m), X^T X and Q^T Y (s x s x m),
    // X C (m x s x s)
    Gemm g_GQ, g_QtY, g_XC;
    {
        std::vector<BG> gq(J), qty(J), xc(J);
        for (int j = 0; j < J; ++j) {
            const int m = bt.m[j], sj = bt.s[j];
            gq[j] = BG{g_off[j], bt.xo[j], bt.xo[j], m, sj, m, m, sj, sj, 0};
            qty[j] = BG{bt.xo[j], bt.xo[j], bt.to[j], sj, sj, m, sj, sj, sj, 0};
            xc[j] = BG{bt.xo[j], bt.to[j], bt.xo[j], m, sj, sj, sj, sj, sj, 0};
        }
        if (rc == RANN_OK) rc = make_gemm(h, gq, g_GQ);
        if (rc == RANN_OK) rc = make_gemm(h, qty, g_QtY);
        if (rc == RANN_OK) rc = make_gemm(h, xc, g_XC);
        for (void* p : {(void*)g_GQ.d, (void*)g_GQ.tasks, (void*)g_QtY.d, (void*)g_QtY.tasks, (void*)g_XC.d,
                        (void*)g_XC.tasks})
            if (p) owned.push_back(p);
    }
    if (rc != RANN_OK) {
        release();
        return rc;
    }
    auto decline = [&]() {
        release();
        return kSubspaceDecline;
    };
    hipLaunchKernelGGL(k_seed, dim3(J), dim3(256), 0, h.stream, d_m, d_s, d_xo, (const int32_t*)nullptr, X);
    RDD_HIP(hipGetLastError());
    for (int round = 0; round < kMaxRounds; ++round) {
        // Q = orthonormal basis of X: shifted Cholesky QR, then two plain passes
        RDD_HIP(hipMemsetAsync(d_fl, 0, sizeof(int32_t) * 2, h.stream));
        RDD_HIP(hipMemsetAsync(d_flags, 0, sizeof(int32_t) * 2, h.stream));
        double* src = X;
        for (int pass = 0; pass < 3; ++pass) {
            double* dst = (pass % 2 == 0) ? Q : X;
            RDD_TRY(run_gemm(h, g_QtY, true, src, src, Sg));  // X^T X
            hipLaunchKernelGGL(k_chol_inv, dim3(J), dim3(kCT), 0, h.stream, d_m, d_s, d_to, Sg, Rinv,
                               pass == 0 ? 1 : 0, d_fl);
            RDD_TRY(run_gemm(h, g_XC, false, src, Rinv, dst));  // X R^{-1}
            src = dst;
        }
        // Rayleigh-Ritz in span(Q)
        RDD_TRY(run_gemm(h, g_GQ, false, G, Q, Y));  // Y = G Q
        RDD_TRY(run_gemm(h, g_QtY, true, Q, Y, T));  // T = Q^T Y
        hipLaunchKernelGGL(k_symm, dim3(J), dim3(256), 0, h.stream, d_s, d_to, T);
        RDD_HIP(hipGetLastError());
        const EigDims dims{J, bt.s.data(), d_s, d_so, bt.so[J]};
        {
            KTimeOff inner;  // inside this path's own timer
            RDD_TRY(eig_batched_dims(h, dims, T, d_to, scr, d_eoff, Cm, tol, mode, d_p, theta, d_flags, d_s));
        }
        RDD_TRY(run_gemm(h, g_XC, false, Q, Cm, U));  // U = Q C
        RDD_TRY(run_gemm(h, g_XC, false, Y, Cm, Z));  // Z = Y C = G U
        hipLaunchKernelGGL(k_resid, dim3(J), dim3(256), 0, h.stream, d_m, d_s, d_xo, d_so, Z, U, theta, res);
        RDD_HIP(hipGetLastError());
        std::vector<int32_t> p(J), fl(2);
        std::vector<double> th((size_t)bt.so[J]), rs((size_t)bt.so[J]);
        RDD_TRY(download(h, p.data(), d_p, sizeof(int32_t) * J));
        RDD_TRY(download(h, fl.data(), d_fl, sizeof(int32_t) * 2));
        RDD_TRY(download(h, th.data(), theta, sizeof(double) * th.size()));
        RDD_TRY(download(h, rs.data(), res, sizeof(double) * rs.size()));
        if (fl[0]) return decline();  // a Cholesky pivot failed
        bool done = true;
        for (int j = 0; j < J; ++j) {
            const int m = bt.m[j], sj = bt.s[j];
            if (sj < m && p[j] + kMargin > sj) return decline();  // the block is too narrow
            const int64_t o = bt.so[j];
            const double eta = 10.0 * m * 1.1102230246251565e-16 * std::max(th[o], 0.0);
            const int need = std::min(p[j] + 1, sj);
            for (int c = 0; c < need; ++c)
                if (!(rs[o + c] <= eta)) done = false;
        }
        if (done) {
            hipLaunchKernelGGL(k_pack, dim3(J), dim3(256), 0, h.stream, d_m, d_s, d_p, d_xo, d_so, d_g_off,
                               h.d_m_off, U, theta, Yfull, d_eig);
            RDD_HIP(hipGetLastError());
            kt_.stop();
            RDD_HIP(hipStreamSynchronize(h.stream));
            release();
            return RANN_OK;
        }
        // next block: the columns of Z = G U scaled to unit length
        hipLaunchKernelGGL(k_colscale, dim3(J), dim3(256), 0, h.stream, d_m, d_s, d_xo, Z, X);
        RDD_HIP(hipGetLastError());
    }
    return decline();
}

}  // namespace rdd
