// Batched FP64 symmetric eigensolver for the PCA step (paper Sec. 4).
//
// The reduced SVD of the value matrix Psi_j gives the right singular vectors V
// and sigma^2 = eigenvalues of Psi_j^T Psi_j; this file computes the latter
// eigendecomposition of the m_j x m_j Gram matrices of all subdomains:
//   1. blocked Householder reduction to tridiagonal form A = Q T Q^T.  Per
//      panel of kNB columns, one workgroup per matrix runs the kNB reflector
//      steps against the panel-start matrix (corrected by the panel's earlier
//      reflectors, so the matrix is only read), then one batched matrix-core
//      launch applies the rank-2 kNB update A -= V W^T + W V^T to the trailing
//      part of every matrix;
//   2. every eigenvalue of T by Sturm-count bisection, four interleaved
//      evaluation points per thread; the truncation count p is the Sturm
//      count at the threshold;
//   3. eigenvectors of T for the p largest eigenvalues by inverse iteration
//      (tridiagonal LU with partial pivoting, one thread per vector, vectors
//      interleaved in memory), then classical Gram-Schmidt applied twice in
//      descending eigenvalue order;
//   4. y = Q z with the reflectors of each panel applied as one block
//      reflector I - V T V^T (last panel first).
// The reflector of step k is kept in row k of A right of the diagonal; Y
// receives the leading eigenvectors as columns of an m_j x m_j row-major matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace rdd {

namespace {

constexpr int kNB = 32;                  // panel width of the blocked reduction
constexpr int kPT = 1024;                // threads of the panel and solve kernels
constexpr int kPC = 64, kPG = kPT / kPC; // 64 columns x 16 row groups
constexpr int kTC = 128;                 // eigenvector columns per back-transform pass

// per-matrix scratch: W (kNB x m), the tridiagonal (d, e, tau: 3 m), and the
// inverse-iteration LU factors (5 fields x m x m, vector index fastest)
__host__ __device__ inline int64_t scr_tri(int64_t m) { return kNB * m; }
__host__ __device__ inline int64_t scr_LU(int64_t m) { return kNB * m + 3 * m; }

__device__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kPT / 64; ++w) s += red[w];
    return s;
}

// ---------------------------------------------------------------- 1. panel
// Steps k = k0 .. k0 + kNB - 1 of the reduction of every matrix.  With V the
// panel's reflectors (rows of A) and W its update vectors (rows of Wb), the
// current matrix is A_start - V W^T - W V^T on rows/columns >= k.
__global__ void __launch_bounds__(kPT) k_tri_panel(const int32_t* __restrict__ mvec,
                                                   const int64_t* __restrict__ g_off,
                                                   double* __restrict__ Gall,
                                                   double* __restrict__ Sall,
                                                   const int64_t* __restrict__ s_off, int k0) {
    __shared__ double x[kMaxWidth];
    __shared__ double v[kMaxWidth];
    __shared__ double w[kMaxWidth];
    __shared__ double part[kPG][kPC + 1];
    __shared__ double hv[kNB], hw[kNB];
    __shared__ double red[kPT / 64];
    const int j = blockIdx.x;
    const int m = mvec[j];
    if (k0 >= m) return;
    const int64_t mm = m;
    double* A = Gall + g_off[j];
    double* Wb = Sall + s_off[j];
    double* tri = Sall + s_off[j] + scr_tri(mm);
    double* dd = tri;
    double* ee = tri + mm;
    double* taus = tri + 2 * mm;
    const int tid = threadIdx.x;
    const int tc = tid % kPC, tr = tid / kPC;
    const int lane = tid & 63, wave = tid >> 6;
    const int kend = (k0 + kNB < m) ? k0 + kNB : m;
    for (int k = k0; k < kend; ++k) {
        const int i = k - k0;
        const int n1 = m - k - 1;
        // row k of the current matrix, entries c >= k
        for (int c = k + tid; c < m; c += kPT) {
            double s = A[(int64_t)k * mm + c];
            for (int q = 0; q < i; ++q) {
                const double* Vq = A + (int64_t)(k0 + q) * mm;
                const double* Wq = Wb + (int64_t)q * mm;
                s -= Vq[k] * Wq[c] + Wq[k] * Vq[c];
            }
            x[c - k] = s;
        }
        __syncthreads();
        if (n1 < 2) {  // no reflector: the last 2 x 2 block is already tridiagonal
            if (tid == 0) {
                dd[k] = x[0];
                ee[k] = (n1 == 1) ? x[1] : 0.0;
                taus[k] = 0.0;
            }
            for (int c = tid; c < n1; c += kPT) A[(int64_t)k * mm + k + 1 + c] = 0.0;
            for (int c = tid; c < m; c += kPT) Wb[(int64_t)i * mm + c] = 0.0;
            __syncthreads();
            continue;
        }
        double pp = 0.0;
        for (int c = tid; c < n1; c += kPT) pp += x[1 + c] * x[1 + c];
        const double nrm2 = block_sum(pp, red);
        const double v0 = x[1];
        const double alpha = (v0 >= 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
        const double tau = (nrm2 > 0.0) ? 1.0 / (nrm2 - v0 * alpha) : 0.0;  // 2 / v^T v
        for (int c = tid; c < n1; c += kPT) {
            const double vc = (nrm2 > 0.0) ? ((c == 0) ? v0 - alpha : x[1 + c]) : 0.0;
            v[c] = vc;
            A[(int64_t)k * mm + k + 1 + c] = vc;
        }
        if (tid == 0) {
            dd[k] = x[0];
            ee[k] = (nrm2 > 0.0) ? alpha : 0.0;
            taus[k] = tau;
        }
        __syncthreads();
        // p = A_start[k+1.., k+1..] v  (column sums, 16 row groups)
        const double* Ap = A + (int64_t)(k + 1) * mm + (k + 1);
        for (int c0 = 0; c0 < n1; c0 += kPC) {
            const int c = c0 + tc;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            if (c < n1) {
                int r = tr;
                for (; r + 3 * kPG < n1; r += 4 * kPG) {
                    s0 = fma(Ap[(int64_t)r * mm + c], v[r], s0);
                    s1 = fma(Ap[(int64_t)(r + kPG) * mm + c], v[r + kPG], s1);
                    s2 = fma(Ap[(int64_t)(r + 2 * kPG) * mm + c], v[r + 2 * kPG], s2);
                    s3 = fma(Ap[(int64_t)(r + 3 * kPG) * mm + c], v[r + 3 * kPG], s3);
                }
                for (; r < n1; r += kPG) s0 = fma(Ap[(int64_t)r * mm + c], v[r], s0);
            }
            part[tr][tc] = (s0 + s1) + (s2 + s3);
            __syncthreads();
            if (tr == 0 && c < n1) {
                double s = 0.0;
                for (int g = 0; g < kPG; ++g) s += part[g][tc];
                w[c] = s;
            }
            __syncthreads();
        }
        // hv = W^T v, hw = V^T v over rows k+1 .. m-1 (one wave per dot product)
        for (int dq = wave; dq < 2 * i; dq += kPT / 64) {
            const int q = dq >> 1;
            const double* src = (dq & 1) ? A + (int64_t)(k0 + q) * mm : Wb + (int64_t)q * mm;
            double s = 0.0;
            for (int c = lane; c < n1; c += 64) s = fma(src[k + 1 + c], v[c], s);
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (lane == 0) {
                if (dq & 1)
                    hw[q] = s;
                else
                    hv[q] = s;
            }
        }
        __syncthreads();
        // w = tau (p - V hv - W hw), then w -= (tau/2)(w^T v) v
        double pv = 0.0;
        for (int c = tid; c < n1; c += kPT) {
            double s = w[c];
            for (int q = 0; q < i; ++q)
                s -= A[(int64_t)(k0 + q) * mm + k + 1 + c] * hv[q] +
                     Wb[(int64_t)q * mm + k + 1 + c] * hw[q];
            s *= tau;
            w[c] = s;
            pv += s * v[c];
        }
        const double K = 0.5 * tau * block_sum(pv, red);
        double* Wi = Wb + (int64_t)i * mm;
        for (int c = tid; c < m; c += kPT) {
            const int cc = c - (k + 1);
            Wi[c] = (cc >= 0) ? w[cc] - K * v[cc] : 0.0;
        }
        __syncthreads();
    }
}

// trailing update A[r][c] -= sum_i V[r][i] W[c][i] + W[r][i] V[c][i] on the
// 64 x 64 tile (y, z) of rows/columns >= k1 = k0 + kNB (both triangles)
__global__ void __launch_bounds__(256) k_tri_update(const int4* __restrict__ tasks,
                                                    const int32_t* __restrict__ mvec,
                                                    const int64_t* __restrict__ g_off,
                                                    double* __restrict__ Gall,
                                                    const double* __restrict__ Sall,
                                                    const int64_t* __restrict__ s_off, int k0) {
    __shared__ double As[kTK][kTM + kPad];
    __shared__ double Bs[kTK][kTN + kPad];
    const int4 tk = tasks[blockIdx.x];
    const int j = tk.x;
    const int64_t mm = mvec[j];
    const int64_t k1 = k0 + kNB;
    const int64_t r0 = k1 + (int64_t)tk.y * kTM, c0 = k1 + (int64_t)tk.z * kTN;
    const int rv = (int)((mm - r0) < kTM ? (mm - r0) : kTM);
    const int cv = (int)((mm - c0) < kTN ? (mm - c0) : kTN);
    double* A = Gall + g_off[j];
    const double* Vr = A + (int64_t)k0 * mm;  // row i of V: A[k0 + i][*]
    const double* Wr = Sall + s_off[j];       // row i of W
    TileAcc<double> acc;
    acc.zero();
    const int t = threadIdx.x;
    for (int half = 0; half < 2; ++half) {
        const double* L = half ? Wr : Vr;  // left operand rows, k = reflector index
        const double* R = half ? Vr : Wr;
        for (int kk0 = 0; kk0 < kNB; kk0 += kTK) {
            const int kk = t >> 4, m4 = (t & 15) * 4;
            for (int e = 0; e < 4; ++e) {
                const int mi = m4 + e;
                As[kk][mi] = (mi < rv) ? L[(int64_t)(kk0 + kk) * mm + r0 + mi] : 0.0;
                Bs[kk][mi] = (mi < cv) ? R[(int64_t)(kk0 + kk) * mm + c0 + mi] : 0.0;
            }
            __syncthreads();
            acc.step(As, Bs);
            __syncthreads();
        }
    }
    acc.each([&](int r, int c, double val) {
        if (r < rv && c < cv) A[(r0 + r) * mm + c0 + c] -= val;
    });
}

// ---------------------------------------------------------------- 2-4. solve
// counts of eigenvalues of the tridiagonal (d, e2 = e^2) below x[0..3]
__device__ inline void sturm_count4(const double* d, const double* e2, int m, const double* x,
                                    double pivmin, int* cnt) {
    double q[4];
    int c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        q[u] = d[0] - x[u];
        if (fabs(q[u]) < pivmin) q[u] = -pivmin;
        c[u] = (q[u] < 0.0) ? 1 : 0;
    }
    for (int i = 1; i < m; ++i) {
        const double di = d[i], ei = e2[i - 1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            q[u] = (di - x[u]) - ei / q[u];
            if (fabs(q[u]) < pivmin) q[u] = -pivmin;
            c[u] += (q[u] < 0.0) ? 1 : 0;
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) cnt[u] = c[u];
}

__device__ int sturm_count(const double* d, const double* e2, int m, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0) ? 1 : 0;
    for (int i = 1; i < m; ++i) {
        q = (d[i] - x) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0) ? 1 : 0;
    }
    return cnt;
}

__global__ void __launch_bounds__(kPT) k_tri_solve(const int32_t* __restrict__ mvec,
                                                   const int64_t* __restrict__ g_off,
                                                   const double* __restrict__ Gall,
                                                   double* __restrict__ Sall,
                                                   const int64_t* __restrict__ s_off,
                                                   double* __restrict__ Yall, double tol, int mode,
                                                   int32_t* __restrict__ p_out,
                                                   double* __restrict__ eig_out,
                                                   const int64_t* __restrict__ m_off,
                                                   int32_t* __restrict__ flags) {
    __shared__ double dd[kMaxWidth];
    __shared__ double e2[kMaxWidth];
    __shared__ double ee[kMaxWidth];
    __shared__ double lam[kMaxWidth];  // ascending eigenvalues of T
    __shared__ double hcoef[kMaxWidth];
    __shared__ double part[kPG][kPC + 1];
    __shared__ double Tm[kNB][kNB + 1];
    __shared__ double Z1[kNB][kTC + 1];
    __shared__ double red[kPT / 64];
    const int j = blockIdx.x;
    const int m = mvec[j];
    const int64_t mm = m;
    const double* A = Gall + g_off[j];
    double* Y = Yall + g_off[j];
    const double* tri = Sall + s_off[j] + scr_tri(mm);
    const double* taus = tri + 2 * mm;
    double* LU = Sall + s_off[j] + scr_LU(mm);
    const int tid = threadIdx.x;
    const int tc = tid % kPC, tr = tid / kPC;
    for (int i = tid; i < m; i += kPT) {
        dd[i] = tri[i];
        ee[i] = (i + 1 < m) ? tri[mm + i] : 0.0;
    }
    __syncthreads();
    // ---- 2. eigenvalues by bisection (Gershgorin bounds, Sturm counts)
    double gl = 0.0, gu = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < m ? fabs(ee[i]) : 0.0);
        const double lo_i = dd[i] - r, hi_i = dd[i] + r;
        gl = (i == 0 || lo_i < gl) ? lo_i : gl;
        gu = (i == 0 || hi_i > gu) ? hi_i : gu;
    }
    const double tnorm = fmax(fabs(gl), fabs(gu));
    for (int i = tid; i < m; i += kPT) e2[i] = (i + 1 < m) ? ee[i] * ee[i] : 0.0;
    __syncthreads();
    const double pivmin = DBL_MIN * fmax(1.0, tnorm * tnorm);
    const double atol = 2.0 * DBL_EPSILON * tnorm + pivmin;
    for (int idx = tid; idx < m; idx += kPT) {
        // the idx-th smallest eigenvalue: count(lo) <= idx < count(hi); each
        // round evaluates 4 interior points and keeps one of the 5 pieces
        double lo = gl - atol, hi = gu + atol;
        for (int it = 0; it < 100; ++it) {
            if (!((hi - lo) > atol + 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) break;
            double xs[4];
            int cs[4];
            for (int u = 0; u < 4; ++u) xs[u] = lo + (hi - lo) * (0.2 * (u + 1));
            sturm_count4(dd, e2, m, xs, pivmin, cs);
            double nlo = xs[3], nhi = hi;
            for (int u = 3; u >= 0; --u)
                if (cs[u] > idx) {
                    nhi = xs[u];
                    nlo = (u > 0) ? xs[u - 1] : lo;
                }
            lo = nlo;
            hi = nhi;
        }
        lam[idx] = 0.5 * (lo + hi);
    }
    __syncthreads();
    const double lam1 = lam[m - 1];
    const double thr = (mode == RANN_PCA_REL_EIG) ? tol * lam1 : tol * tol;
    int p = m;
    if (mode != RANN_PCA_OFF) p = m - sturm_count(dd, e2, m, thr, pivmin);  // same in every thread
    if (p < 0) p = 0;
    for (int i = tid; i < m; i += kPT) eig_out[m_off[j] + i] = lam[m - 1 - i];
    if (tid == 0) {
        p_out[j] = p;
        int tie = 0;
        for (int i = 0; i < m; ++i) tie |= (fabs(lam[i] - thr) <= 1e-6 * fabs(thr)) ? 1 : 0;
        if (tie && mode != RANN_PCA_OFF) flags[1] = 1;
    }
    // ---- 3. inverse iteration for the p largest: vector t <-> eigenvalue
    // lam[m-1-t], z_t stored as column t of Y; LU field f of row i at
    // LU[(f m + i) m + t]
    const double eps_piv = DBL_EPSILON * tnorm + pivmin;
    for (int t = tid; t < p; t += kPT) {
        const double lmb = lam[m - 1 - t];
        double* fa = LU + t;                // diagonal of U
        double* fb = LU + mm * mm + t;      // first superdiagonal
        double* fc = LU + 2 * mm * mm + t;  // second superdiagonal (fill-in)
        double* fm = LU + 3 * mm * mm + t;  // multipliers
        double* fp = LU + 4 * mm * mm + t;  // 1.0 where rows i, i+1 were swapped
        double ai = dd[0] - lmb, bi = ee[0];
        for (int i = 0; i + 1 < m; ++i) {
            const double sub = ee[i];
            const double an = dd[i + 1] - lmb;                // a[i+1] before step i
            const double bn = (i + 2 < m) ? ee[i + 1] : 0.0;  // b[i+1] before step i
            const int64_t o = (int64_t)i * mm;
            if (fabs(ai) >= fabs(sub)) {
                double a = ai;
                if (fabs(a) < eps_piv) a = (a < 0.0) ? -eps_piv : eps_piv;
                const double mu = sub / a;
                fa[o] = a;
                fb[o] = bi;
                fc[o] = 0.0;
                fm[o] = mu;
                fp[o] = 0.0;
                ai = an - mu * bi;
                bi = bn;
            } else {
                const double mu = ai / sub;
                fa[o] = sub;
                fb[o] = an;
                fc[o] = bn;
                fm[o] = mu;
                fp[o] = 1.0;
                ai = bi - mu * an;
                bi = -mu * bn;
            }
        }
        if (fabs(ai) < eps_piv) ai = (ai < 0.0) ? -eps_piv : eps_piv;
        fa[(int64_t)(m - 1) * mm] = ai;
        double* z = Y + t;
        for (int i = 0; i < m; ++i)
            z[(int64_t)i * mm] = 1.0 + 0.5 * sin(0.7 * (double)(i + 1) + 1.3 * (double)(t + 1));
        for (int iter = 0; iter < 3; ++iter) {
            // forward: row swaps and multipliers
            double zc = z[0];
            for (int i = 0; i + 1 < m; ++i) {
                const int64_t o = (int64_t)i * mm;
                const double zn = z[o + mm];
                const double mu = fm[o];
                if (fp[o] != 0.0) {
                    z[o] = zn;
                    zc = zc - mu * zn;
                } else {
                    z[o] = zc;
                    zc = zn - mu * zc;
                }
            }
            // backward: U z = y
            double z1 = zc / fa[(int64_t)(m - 1) * mm], z2 = 0.0;
            z[(int64_t)(m - 1) * mm] = z1;
            double nn = z1 * z1;
            for (int i = m - 2; i >= 0; --i) {
                const int64_t o = (int64_t)i * mm;
                const double zi = (z[o] - fb[o] * z1 - fc[o] * z2) / fa[o];
                z[o] = zi;
                nn = fma(zi, zi, nn);
                z2 = z1;
                z1 = zi;
            }
            const double inv = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
            for (int i = 0; i < m; ++i) z[(int64_t)i * mm] *= inv;
        }
    }
    __syncthreads();
    // classical Gram-Schmidt, twice, in descending eigenvalue order (columns of Y)
    for (int t = 1; t < p; ++t) {
        for (int pass = 0; pass < 2; ++pass) {
            for (int q0 = 0; q0 < t; q0 += kPC) {
                const int q = q0 + tc;
                double s = 0.0;
                if (q < t)
                    for (int i = tr; i < m; i += kPG)
                        s = fma(Y[(int64_t)i * mm + q], Y[(int64_t)i * mm + t], s);
                part[tr][tc] = s;
                __syncthreads();
                if (tr == 0 && q < t) {
                    double h = 0.0;
                    for (int g = 0; g < kPG; ++g) h += part[g][tc];
                    hcoef[q] = h;
                }
                __syncthreads();
            }
            for (int i = tid; i < m; i += kPT) {
                const double* yi = Y + (int64_t)i * mm;
                double acc = yi[t];
                for (int q = 0; q < t; ++q) acc -= hcoef[q] * yi[q];
                Y[(int64_t)i * mm + t] = acc;
            }
            __syncthreads();
        }
        double pp2 = 0.0;
        for (int i = tid; i < m; i += kPT) pp2 += Y[(int64_t)i * mm + t] * Y[(int64_t)i * mm + t];
        const double nn = block_sum(pp2, red);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int i = tid; i < m; i += kPT) Y[(int64_t)i * mm + t] *= inv;
        __syncthreads();
    }
    // ---- 4. y = Q z, Q = H_0 ... H_{m-3}: panels last to first, each applied
    // as I - V T V^T with V[r][q] = A[k0 + q][r] for r > k0 + q (zero otherwise)
    const int nref = (m >= 2) ? m - 2 : 0;
    for (int k0 = ((nref - 1) / kNB) * kNB; nref > 0 && k0 >= 0; k0 -= kNB) {
        const int nb = (k0 + kNB < nref) ? kNB : nref - k0;
        // V^T V above the diagonal, zero elsewhere
        for (int e = tid; e < kNB * kNB; e += kPT) {
            const int a = e / kNB, b = e % kNB;
            double s = 0.0;
            if (a < b && b < nb) {
                const double* va = A + (int64_t)(k0 + a) * mm;
                const double* vb = A + (int64_t)(k0 + b) * mm;
                for (int r = k0 + b + 1; r < m; ++r) s = fma(va[r], vb[r], s);
            }
            Tm[a][b] = s;
        }
        __syncthreads();
        // T[b][b] = tau_b, T[a][b] = -tau_b sum_{c=a}^{b-1} T[a][c] (V^T V)[c][b]
        for (int b = 0; b < nb; ++b) {
            double s = 0.0;
            if (tid < b)
                for (int c = tid; c < b; ++c) s = fma(Tm[tid][c], Tm[c][b], s);
            __syncthreads();
            if (tid < b) Tm[tid][b] = -taus[k0 + b] * s;
            if (tid == b) Tm[b][b] = taus[k0 + b];
            __syncthreads();
        }
        for (int t0 = 0; t0 < p; t0 += kTC) {
            const int nc = (p - t0 < kTC) ? p - t0 : kTC;
            // Z1 = V^T Y[:, t0 .. t0 + nc)
            for (int e = tid; e < nb * kTC; e += kPT) {
                const int q = e / kTC, c = e % kTC;
                double s = 0.0;
                if (c < nc) {
                    const double* vq = A + (int64_t)(k0 + q) * mm;
                    for (int r = k0 + q + 1; r < m; ++r) s = fma(vq[r], Y[(int64_t)r * mm + t0 + c], s);
                }
                Z1[q][c] = s;
            }
            __syncthreads();
            // Z2 = T Z1 in place (row q reads rows >= q)
            for (int c = tid; c < nc; c += kPT) {
                for (int q = 0; q < nb; ++q) {
                    double s = 0.0;
                    for (int b = q; b < nb; ++b) s = fma(Tm[q][b], Z1[b][c], s);
                    Z1[q][c] = s;
                }
            }
            __syncthreads();
            // Y -= V Z2 on rows > k0
            for (int64_t e = tid; e < (int64_t)(m - k0 - 1) * nc; e += kPT) {
                const int r = k0 + 1 + (int)(e / nc), c = (int)(e % nc);
                double s = 0.0;
                const int qmax = (r - k0 < nb) ? r - k0 : nb;  // V[r][q] != 0 for q < r - k0
                for (int q = 0; q < qmax; ++q) s = fma(A[(int64_t)(k0 + q) * mm + r], Z1[q][c], s);
                Y[(int64_t)r * mm + t0 + c] -= s;
            }
            __syncthreads();
        }
    }
}

__global__ void k_compact_V(const int32_t* __restrict__ mvec, const int32_t* __restrict__ p,
                            const int64_t* __restrict__ g_off, const int64_t* __restrict__ v_off,
                            const double* __restrict__ Vfull, double* __restrict__ V) {
    const int j = blockIdx.x;
    const int m = mvec[j], pj = p[j];
    for (int64_t e = threadIdx.x; e < (int64_t)m * pj; e += blockDim.x) {
        int r = (int)(e / pj), k = (int)(e % pj);
        V[v_off[j] + e] = Vfull[g_off[j] + (int64_t)r * m + k];
    }
}

}  // namespace

int64_t eig_scratch_elems(int m) { return scr_LU(m) + 5LL * m * m; }

int eig_batched(Handle& h, double* G, const int64_t* d_g_off, double* S, const int64_t* d_s_off,
                double* Y, double tol, int mode, int32_t* d_p, double* d_eig, int32_t* d_flags) {
    const int J = h.geo.J;
    KTimer kt_(h.stream, "k_eig");
    int mmax = 0;
    for (int j = 0; j < J; ++j) mmax = std::max(mmax, h.m[j]);
    // tile lists of the trailing updates, one group per panel
    std::vector<int4> tasks;
    std::vector<int64_t> off;
    for (int k0 = 0; k0 < mmax; k0 += kNB) {
        off.push_back((int64_t)tasks.size());
        for (int j = 0; j < J; ++j) {
            const int n2 = h.m[j] - (k0 + kNB);
            if (n2 <= 0) continue;
            const int nt = (n2 + kTM - 1) / kTM;
            for (int a = 0; a < nt; ++a)
                for (int b = 0; b < nt; ++b) tasks.push_back(make_int4(j, a, b, 0));
        }
    }
    off.push_back((int64_t)tasks.size());
    int4* d_tasks = nullptr;
    RDD_TRY(dev_alloc(h, &d_tasks, tasks.size()));
    if (!tasks.empty())
        RDD_HIP(hipMemcpy(d_tasks, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice));
    int pi = 0;
    for (int k0 = 0; k0 < mmax; k0 += kNB, ++pi) {
        hipLaunchKernelGGL(k_tri_panel, dim3(J), dim3(kPT), 0, h.stream, h.d_m, d_g_off, G, S,
                           d_s_off, k0);
        const int64_t cnt = off[pi + 1] - off[pi];
        if (cnt > 0)
            hipLaunchKernelGGL(k_tri_update, dim3((unsigned)cnt), dim3(256), 0, h.stream,
                               d_tasks + off[pi], h.d_m, d_g_off, G, S, d_s_off, k0);
        RDD_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_tri_solve, dim3(J), dim3(kPT), 0, h.stream, h.d_m, d_g_off, G, S, d_s_off,
                       Y, tol, mode, d_p, d_eig, h.d_m_off, d_flags);
    kt_.stop();
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, d_tasks);
    return RANN_OK;
}

int compact_V(Handle& h, const double* Vfull, const int64_t* d_g_off, double* V) {
    hipLaunchKernelGGL(k_compact_V, dim3(h.geo.J), dim3(256), 0, h.stream, h.d_m, h.d_p, d_g_off,
                       h.d_v_off, Vfull, V);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace rdd
