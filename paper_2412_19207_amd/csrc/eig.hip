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
//   2. every eigenvalue of T by Sturm-count bisection, one thread per
//      eigenvalue across many workgroups; the truncation count p is the Sturm
//      count at the threshold;
//   3. eigenvectors of T for the p largest eigenvalues by inverse iteration
//      (tridiagonal LU with partial pivoting, one thread per vector), then an
//      orthonormal basis in descending eigenvalue order by Cholesky QR applied
//      twice (classical Gram-Schmidt twice when p is large or the vectors are
//      nearly dependent);
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

constexpr int kNB = 16;                  // panel width of the blocked reduction (a multiple of kTK)
constexpr int kPT = 1024;                // threads of the panel and solve kernels
constexpr int kPC = 64, kPG = kPT / kPC; // 64 columns x 16 row groups

// per-matrix scratch: W (kNB x m), the tridiagonal (d, e, tau: 3 m), the
// inverse-iteration LU factors (5 rows of m per vector) and the vectors (m x m)
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

// block_sum without its leading barrier, for a caller whose buffer red has
// not been read since its last barrier
__device__ double block_sum_fresh(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kPT / 64; ++w) s += red[w];
    return s;
}

// ---------------------------------------------------------------- 1. panel
// The panel product p = A v runs on G row groups of C column lanes, C = the
// trailing size rounded up to 64 (G C <= kPT), so that small trailing
// matrices still keep every thread busy; loops over the panel's reflectors
// and over rows take 8 entries per round to keep many loads in flight.

// Steps k = k0 .. k0 + kNB - 1 of the reduction of every matrix.  With V the
// panel's reflectors (rows of A) and W its update vectors (rows of Wb), the
// current matrix is A_start - V W^T - W V^T on rows/columns >= k.  With kInLds
// (every m <= kPanelCols) the panel's V and W rows are also kept in LDS from
// column k0 on, and the steps read them there; the trailing block of A_start
// is read from global memory either way.
constexpr int kPanelCols = 480;  // widest matrix whose panel rows fit in LDS

template <bool kInLds>
__global__ void __launch_bounds__(kPT) k_tri_panel(const int32_t* __restrict__ mvec,
                                                   const int64_t* __restrict__ g_off,
                                                   double* __restrict__ Gall,
                                                   double* __restrict__ Sall,
                                                   const int64_t* __restrict__ s_off, int k0) {
    __shared__ double x[kMaxWidth];
    __shared__ double v[kMaxWidth];
    __shared__ double w[kMaxWidth];
    __shared__ double part[kPT];
    __shared__ double hv[kNB], hw[kNB], sv[kNB], sw[kNB];
    __shared__ double red_n[kPT / 64], red_k[kPT / 64];  // one buffer per block sum of a step
    __shared__ double Vl[kInLds ? kNB * kPanelCols : 1];  // Vl[q][c - k0] = A[k0 + q][c]
    __shared__ double Wl[kInLds ? kNB * kPanelCols : 1];  // Wl[q][c - k0] = Wb[q][c]
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
    // row q of the panel's V and W at column c >= k0
    auto Vr = [&](int q, int c) -> double {
        if constexpr (kInLds) return Vl[q * kPanelCols + (c - k0)];
        else return A[(int64_t)(k0 + q) * mm + c];
    };
    auto Wr = [&](int q, int c) -> double {
        if constexpr (kInLds) return Wl[q * kPanelCols + (c - k0)];
        else return Wb[(int64_t)q * mm + c];
    };
    const int kend = (k0 + kNB < m) ? k0 + kNB : m;
    // LDS mode (m - k <= kPT: one column per thread): x[tid] holds A_start[k][k + tid]
    // on entry to step k; later rows are fetched one step ahead, beside the
    // loads of the panel product
    if constexpr (kInLds)
        if (k0 + tid < m) x[tid] = A[(int64_t)k0 * mm + k0 + tid];
    for (int k = k0; k < kend; ++k) {
        const int i = k - k0;
        const int n1 = m - k - 1;
        // the panel's earlier reflectors at row k: V[k][q] and W[k][q] (staged
        // from global memory; read in place from LDS)
        if constexpr (!kInLds) {
            if (tid < i) {
                sv[tid] = Vr(tid, k);
                sw[tid] = Wr(tid, k);
            }
            __syncthreads();
        }
        auto Vk = [&](int q) -> double {
            if constexpr (kInLds) return Vl[q * kPanelCols + (k - k0)];
            else return sv[q];
        };
        auto Wk = [&](int q) -> double {
            if constexpr (kInLds) return Wl[q * kPanelCols + (k - k0)];
            else return sw[q];
        };
        // row k of the current matrix, entries c >= k
        for (int c = k + tid; c < m; c += kPT) {
            double s8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) s8[u] = 0.0;
            int q = 0;
            for (; q + 7 < i; q += 8) {
                double wv[8], vv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    wv[u] = Wr(q + u, c);
                    vv[u] = Vr(q + u, c);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s8[u] -= Vk(q + u) * wv[u] + Wk(q + u) * vv[u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u < i) s8[u] -= Vk(q + u) * Wr(q + u, c) + Wk(q + u) * Vr(q + u, c);
            double a_kc;
            if constexpr (kInLds) a_kc = x[c - k];  // fetched by this thread
            else a_kc = A[(int64_t)k * mm + c];
            x[c - k] = a_kc + (((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7])));
        }
        __syncthreads();
        if (n1 < 2) {  // no reflector: the last 2 x 2 block is already tridiagonal
            if (tid == 0) {
                dd[k] = x[0];
                ee[k] = (n1 == 1) ? x[1] : 0.0;
                taus[k] = 0.0;
            }
            for (int c = tid; c < n1; c += kPT) {
                A[(int64_t)k * mm + k + 1 + c] = 0.0;
                if constexpr (kInLds) Vl[i * kPanelCols + (k + 1 + c - k0)] = 0.0;
            }
            for (int c = tid; c < m; c += kPT) {
                Wb[(int64_t)i * mm + c] = 0.0;
                if constexpr (kInLds)
                    if (c >= k0) Wl[i * kPanelCols + (c - k0)] = 0.0;
            }
            __syncthreads();
            if constexpr (kInLds)
                if (k + 1 < kend && k + 1 + tid < m) x[tid] = A[(int64_t)(k + 1) * mm + k + 1 + tid];
            continue;
        }
        double pp = 0.0;
        for (int c = tid; c < n1; c += kPT) pp += x[1 + c] * x[1 + c];
        const double nrm2 = block_sum_fresh(pp, red_n);
        const double x1 = x[1];
        const double alpha = (x1 >= 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
        const double tau = (nrm2 > 0.0) ? 1.0 / (nrm2 - x1 * alpha) : 0.0;  // 2 / v^T v
        for (int c = tid; c < n1; c += kPT) {
            const double vc = (nrm2 > 0.0) ? ((c == 0) ? x1 - alpha : x[1 + c]) : 0.0;
            v[c] = vc;
            A[(int64_t)k * mm + k + 1 + c] = vc;
            if constexpr (kInLds) Vl[i * kPanelCols + (k + 1 + c - k0)] = vc;
        }
        if (tid == 0) {
            dd[k] = x[0];
            ee[k] = (nrm2 > 0.0) ? alpha : 0.0;
            taus[k] = tau;
        }
        __syncthreads();
        // p = A_start[k+1.., k+1..] v: thread (g, c) sums rows r = g (mod G)
        // of column c, 8 rows per batch of loads; partial sums part[g C + c]
        const double* Ap = A + (int64_t)(k + 1) * mm + (k + 1);
        const int C = (n1 + 63) / 64 * 64;
        const int G = kPT / C;
        {
            const int g = tid / C, c = tid % C;
            double a_next = 0.0;
            if constexpr (kInLds)
                if (k + 1 < kend && k + 1 + tid < m) a_next = A[(int64_t)(k + 1) * mm + k + 1 + tid];
            double acc8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc8[u] = 0.0;
            if (g < G && c < n1) {
                int r = g;
                for (; r + 7 * G < n1; r += 8 * G) {
                    double av[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) av[u] = Ap[(int64_t)(r + u * G) * mm + c];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc8[u] = fma(av[u], v[r + u * G], acc8[u]);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (r + u * G < n1) acc8[u] = fma(Ap[(int64_t)(r + u * G) * mm + c], v[r + u * G], acc8[u]);
            }
            if (g < G)
                part[g * C + c] = ((acc8[0] + acc8[1]) + (acc8[2] + acc8[3])) + ((acc8[4] + acc8[5]) + (acc8[6] + acc8[7]));
            // x is free until step k + 1 reads its own entry
            if constexpr (kInLds)
                if (k + 1 < kend && k + 1 + tid < m) x[tid] = a_next;
        }
        // hv = W^T v, hw = V^T v over rows k+1 .. m-1: 16 lanes per dot product
        {
            const int dq = tid >> 4, g = tid & 15;
            double sacc = 0.0;
            if (dq < 2 * i) {
                const int q = dq >> 1;
                const double* src;
                if constexpr (kInLds)
                    src = ((dq & 1) ? Vl : Wl) + q * kPanelCols + (k + 1 - k0);
                else
                    src = ((dq & 1) ? A + (int64_t)(k0 + q) * mm : Wb + (int64_t)q * mm) + k + 1;
                double s4[4] = {0.0, 0.0, 0.0, 0.0};
                int c = g;
                for (; c + 48 < n1; c += 64) {
                    double tv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) tv[u] = src[c + 16 * u];
#pragma unroll
                    for (int u = 0; u < 4; ++u) s4[u] = fma(tv[u], v[c + 16 * u], s4[u]);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (c + 16 * u < n1) s4[u] = fma(src[c + 16 * u], v[c + 16 * u], s4[u]);
                sacc = (s4[0] + s4[1]) + (s4[2] + s4[3]);
            }
            for (int off = 8; off > 0; off >>= 1) sacc += __shfl_xor(sacc, off);
            if (dq < 2 * i && g == 0) {
                if (dq & 1)
                    hw[dq >> 1] = sacc;
                else
                    hv[dq >> 1] = sacc;
            }
        }
        __syncthreads();
        // w = tau (p - V hv - W hw), then w -= (tau/2)(w^T v) v
        double pv = 0.0;
        for (int c = tid; c < n1; c += kPT) {
            double s0 = 0.0;
            for (int g = 0; g < G; ++g) s0 += part[g * C + c];
            double s8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) s8[u] = 0.0;
            int q = 0;
            for (; q + 7 < i; q += 8) {
                double av[8], bv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    av[u] = Vr(q + u, k + 1 + c);
                    bv[u] = Wr(q + u, k + 1 + c);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s8[u] -= av[u] * hv[q + u] + bv[u] * hw[q + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q + u < i) s8[u] -= Vr(q + u, k + 1 + c) * hv[q + u] + Wr(q + u, k + 1 + c) * hw[q + u];
            const double wc = tau * (s0 + (((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]))));
            w[c] = wc;
            pv += wc * v[c];
        }
        const double K = 0.5 * tau * block_sum_fresh(pv, red_k);
        double* Wi = Wb + (int64_t)i * mm;
        for (int c = tid; c < m; c += kPT) {
            const int cc = c - (k + 1);
            const double wc = (cc >= 0) ? w[cc] - K * v[cc] : 0.0;
            Wi[c] = wc;
            if constexpr (kInLds)
                if (c >= k0) Wl[i * kPanelCols + (c - k0)] = wc;
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
    static_assert(kNB % kTK == 0, "whole staging slices of reflector rows");
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

// ---------------------------------------------------------------- 2. eigenvalues
// count of eigenvalues of the tridiagonal (d, e2 = e^2) below x, with IEEE division
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

// the same count with 1/q from the hardware reciprocal refined by two Newton
// steps (full FP64 accuracy at a third of the cost of the division); |q| >=
// pivmin keeps e2 / q finite
__device__ int sturm_count_fast(const double* d, const double* e2, int m, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0) ? 1 : 0;
    for (int i = 1; i < m; ++i) {
        double r = __builtin_amdgcn_rcp(q);
        r = fma(r, fma(-q, r, 1.0), r);
        r = fma(r, fma(-q, r, 1.0), r);
        q = (d[i] - x) - e2[i - 1] * r;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0) ? 1 : 0;
    }
    return cnt;
}

struct TriBounds {
    double gl, gu, tnorm, pivmin, atol;
};

// Gershgorin interval of the tridiagonal (d, |e|) by one wave
__device__ TriBounds tri_bounds(const double* d, const double* ea, int m) {
    double lo = 0.0, hi = 0.0;
    bool any = false;
    for (int i = (threadIdx.x & 63); i < m; i += 64) {
        const double r = (i > 0 ? ea[i - 1] : 0.0) + (i + 1 < m ? ea[i] : 0.0);
        const double l = d[i] - r, u = d[i] + r;
        lo = any ? fmin(lo, l) : l;
        hi = any ? fmax(hi, u) : u;
        any = true;
    }
    if (!any) {
        lo = d[0];
        hi = d[0];
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off));
        hi = fmax(hi, __shfl_xor(hi, off));
    }
    TriBounds b;
    b.gl = lo;
    b.gu = hi;
    b.tnorm = fmax(fabs(lo), fabs(hi));
    b.pivmin = DBL_MIN * fmax(1.0, b.tnorm * b.tnorm);
    b.atol = 2.0 * DBL_EPSILON * b.tnorm + b.pivmin;
    return b;
}

// every eigenvalue by multisection: 4 lanes per eigenvalue, 16 eigenvalues
// per workgroup.  In each round the 4 lanes count the eigenvalues below the 4
// inner points of 5 equal parts of the interval, and the part that holds the
// idx-th smallest eigenvalue (count(lo) <= idx < count(hi)) becomes the new
// interval; the same stopping width as plain bisection.
__global__ void __launch_bounds__(64) k_bisect(const int32_t* __restrict__ mvec,
                                               const double* __restrict__ Sall,
                                               const int64_t* __restrict__ s_off,
                                               double* __restrict__ lam_all,
                                               const int64_t* __restrict__ m_off,
                                               double* __restrict__ eig_out) {
    __shared__ double dd[kMaxWidth];
    __shared__ double e2[kMaxWidth];
    __shared__ double ea[kMaxWidth];
    const int j = blockIdx.x;
    const int m = mvec[j];
    const int lane = threadIdx.x, sub = lane & 3;
    const int idx = blockIdx.y * 16 + (lane >> 2);
    if ((int)blockIdx.y * 16 >= m) return;  // uniform per workgroup
    const int64_t mm = m;
    const double* tri = Sall + s_off[j] + scr_tri(mm);
    for (int i = lane; i < m; i += 64) {
        const double e = (i + 1 < m) ? tri[mm + i] : 0.0;
        dd[i] = tri[i];
        ea[i] = fabs(e);
        e2[i] = e * e;
    }
    __syncthreads();
    const TriBounds tb = tri_bounds(dd, ea, m);
    const bool live = idx < m;
    double lo = tb.gl - tb.atol, hi = tb.gu + tb.atol;
    for (int it = 0; it < 200; ++it) {
        const bool go = live && (hi - lo) > tb.atol + 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi));
        if (!__any(go)) break;  // wave-uniform: the shuffles below need every lane
        const double h = (hi - lo) * 0.2;
        double pt[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pt[u] = (u == 3) ? hi - h : lo + h * (u + 1);
        const int cnt = go ? sturm_count_fast(dd, e2, m, pt[sub], tb.pivmin) : 0;
        const int base = lane & ~3;
        const int c0 = __shfl(cnt, base), c1 = __shfl(cnt, base + 1);
        const int c2 = __shfl(cnt, base + 2), c3 = __shfl(cnt, base + 3);
        if (go) {
            if (c0 > idx) {
                hi = pt[0];
            } else if (c1 > idx) {
                lo = pt[0];
                hi = pt[1];
            } else if (c2 > idx) {
                lo = pt[1];
                hi = pt[2];
            } else if (c3 > idx) {
                lo = pt[2];
                hi = pt[3];
            } else {
                lo = pt[3];
            }
        }
    }
    if (live && sub == 0) {
        const double l = 0.5 * (lo + hi);
        lam_all[m_off[j] + idx] = l;
        eig_out[m_off[j] + m - 1 - idx] = l;
    }
}

// ---------------------------------------------------------------- 3-4. vectors
constexpr int kLds = 18432;  // doubles of LDS shared by the phases of k_vectors
constexpr int kQRMax = 120;  // Cholesky QR for p <= kQRMax, Gram-Schmidt beyond
constexpr int kStg = 16;     // vector entries per staging chunk of the Gram matrix
constexpr int kRC = 64;      // rows per staging chunk of the back-transform

// Orthonormal rows Q = L^{-1} Z of the p x m matrix Z (rows = vectors, t < p)
// with Z Z^T = L L^T: Gram matrix, Cholesky (one barrier per column; column c
// of L is kept scaled in row c of the unused upper triangle), X = L^{-1} in
// the lower triangle, then Q = X Z in chunks of kStg columns.  Q goes to Zout;
// returns false (nothing written) when a pivot shows near dependence.
__device__ bool chol_qr(const double* __restrict__ Zin, double* __restrict__ Zout, int p, int m,
                        double* lds) {
    const int tid = threadIdx.x;
    const int ldg = p + 1;
    double* Gs = lds;            // p x (p + 1)
    double* Zs = lds + p * ldg;  // p x (kStg + 1)
    __shared__ double gdiag[kQRMax], ldiag[kQRMax];
    __shared__ int fail;
    const int npair = p * (p + 1) / 2;
    constexpr int kMaxPairs = (kQRMax * (kQRMax + 1) / 2 + kPT - 1) / kPT;
    double acc[kMaxPairs];
    int pa[kMaxPairs], pb[kMaxPairs];
#pragma unroll
    for (int u = 0; u < kMaxPairs; ++u) {
        acc[u] = 0.0;
        const int pr = tid + u * kPT;
        int a = (int)((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
        while ((a + 1) * (a + 2) / 2 <= pr) ++a;
        while (a * (a + 1) / 2 > pr) --a;
        pa[u] = a;
        pb[u] = pr - a * (a + 1) / 2;
    }
    for (int i0 = 0; i0 < m; i0 += kStg) {
        for (int e = tid; e < p * kStg; e += kPT) {
            const int t = e / kStg, ii = e % kStg;
            Zs[t * (kStg + 1) + ii] = (i0 + ii < m) ? Zin[(int64_t)t * m + i0 + ii] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kMaxPairs; ++u) {
            if (tid + u * kPT < npair) {
                const double* za = Zs + pa[u] * (kStg + 1);
                const double* zb = Zs + pb[u] * (kStg + 1);
                double sacc = acc[u];
#pragma unroll
                for (int ii = 0; ii < kStg; ++ii) sacc = fma(za[ii], zb[ii], sacc);
                acc[u] = sacc;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kMaxPairs; ++u)
        if (tid + u * kPT < npair) Gs[pa[u] * ldg + pb[u]] = acc[u];
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int c = tid; c < p; c += kPT) gdiag[c] = Gs[c * ldg + c];
    __syncthreads();
    // lower Cholesky: step c reads column c unscaled, updates the trailing lower
    // part and stores L[r][c] = G[r][c] / l in Gs[c][r] (r > c)
    for (int c = 0; c < p; ++c) {
        const double piv = Gs[c * ldg + c];
        if (!(piv > 1e-10 * gdiag[c])) {  // uniform: every thread reads the same pivot
            if (tid == 0) fail = 1;
            break;
        }
        const double l = sqrt(piv), il = 1.0 / l, ip = 1.0 / piv;
        const int n = p - c - 1;
        for (int e = tid; e < n * n + n; e += kPT) {
            if (e < n * n) {
                const int r = c + 1 + e / n, t = c + 1 + e % n;
                if (t <= r) Gs[r * ldg + t] -= Gs[r * ldg + c] * Gs[t * ldg + c] * ip;
            } else {
                const int r = c + 1 + (e - n * n);
                Gs[c * ldg + r] = Gs[r * ldg + c] * il;
            }
        }
        if (tid == 0) ldiag[c] = l;
        __syncthreads();
    }
    __syncthreads();
    if (fail) return false;
    // X = L^{-1} (lower, diagonal included) into the lower triangle, by forward
    // substitution organised by columns of L: once rows 0 .. l of X have all
    // their updates, row l (divided by its pivot) updates every later row, one
    // barrier per column; each row is divided by its pivot at the end
    for (int e = tid; e < p * p; e += kPT) {
        const int r = e / p, c = e % p;
        if (c <= r) Gs[r * ldg + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int l = 0; l + 1 < p; ++l) {
        const double il = 1.0 / ldiag[l];
        const int w = l + 1, n = (p - 1 - l) * w;
        for (int e = tid; e < n; e += kPT) {
            const int i = l + 1 + e / w, c = e % w;
            Gs[i * ldg + c] -= Gs[l * ldg + i] * (Gs[l * ldg + c] * il);  // L[i][l] X[l][c]
        }
        __syncthreads();
    }
    for (int e = tid; e < p * p; e += kPT) {
        const int r = e / p, c = e % p;
        if (c <= r) Gs[r * ldg + c] /= ldiag[r];
    }
    __syncthreads();
    // Q = X Z, kStg columns at a time
    for (int i0 = 0; i0 < m; i0 += kStg) {
        for (int e = tid; e < p * kStg; e += kPT) {
            const int t = e / kStg, ii = e % kStg;
            Zs[t * (kStg + 1) + ii] = (i0 + ii < m) ? Zin[(int64_t)t * m + i0 + ii] : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < p * kStg; e += kPT) {
            const int t = e / kStg, ii = e % kStg;
            if (i0 + ii < m) {
                double sacc = 0.0;
                for (int a2 = 0; a2 <= t; ++a2) sacc = fma(Gs[t * ldg + a2], Zs[a2 * (kStg + 1) + ii], sacc);
                Zout[(int64_t)t * m + i0 + ii] = sacc;
            }
        }
        __syncthreads();
    }
    return true;
}

// classical Gram-Schmidt twice, descending order, on the rows of Zt
__device__ void cgs2(double* Zt, int p, int m, double* hcoef, double* red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int t = 1; t < p; ++t) {
        double* zt = Zt + (int64_t)t * m;
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = wave; q < t; q += kPT / 64) {
                const double* zq = Zt + (int64_t)q * m;
                double s = 0.0;
                for (int i = lane; i < m; i += 64) s = fma(zq[i], zt[i], s);
                for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
                if (lane == 0) hcoef[q] = s;
            }
            __syncthreads();
            for (int i = tid; i < m; i += kPT) {
                double acc = zt[i];
                for (int q = 0; q < t; ++q) acc -= hcoef[q] * Zt[(int64_t)q * m + i];
                zt[i] = acc;
            }
            __syncthreads();
        }
        double pp = 0.0;
        for (int i = tid; i < m; i += kPT) pp += zt[i] * zt[i];
        const double nn = block_sum(pp, red);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int i = tid; i < m; i += kPT) zt[i] *= inv;
        __syncthreads();
    }
}

// element i of a vector stored with a fixed stride (vectors interleaved so
// that the lanes of a wave touch adjacent addresses)
struct StridedRef {
    double* base;
    int64_t stride;
    __device__ __forceinline__ double& operator[](int64_t i) const { return base[i * stride]; }
};

// p (the Sturm count at the truncation threshold) and the tie flag; one
// workgroup per matrix
__global__ void __launch_bounds__(256) k_pcount(const int32_t* __restrict__ mvec,
                                                const double* __restrict__ Sall,
                                                const int64_t* __restrict__ s_off,
                                                const double* __restrict__ lam_all, double tol,
                                                int mode, int32_t* __restrict__ p_out,
                                                const int64_t* __restrict__ m_off,
                                                int32_t* __restrict__ flags) {
    __shared__ double dd[kMaxWidth];
    __shared__ double e2[kMaxWidth];
    __shared__ double ea[kMaxWidth];
    const int j = blockIdx.x;
    const int m = mvec[j];
    const int64_t mm = m;
    const double* tri = Sall + s_off[j] + scr_tri(mm);
    const double* lam = lam_all + m_off[j];  // ascending
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += blockDim.x) {
        const double e = (i + 1 < m) ? tri[mm + i] : 0.0;
        dd[i] = tri[i];
        ea[i] = fabs(e);
        e2[i] = e * e;
    }
    __syncthreads();
    const TriBounds tb = tri_bounds(dd, ea, m);
    const double thr = (mode == RANN_PCA_REL_EIG) ? tol * lam[m - 1] : tol * tol;
    int tie = 0;
    for (int i = tid; i < m; i += blockDim.x) tie |= (fabs(lam[i] - thr) <= 1e-6 * fabs(thr)) ? 1 : 0;
    tie = __syncthreads_or(tie);
    if (tid == 0) {
        int p = m;
        if (mode != RANN_PCA_OFF) p = m - sturm_count(dd, e2, m, thr, tb.pivmin);
        p_out[j] = (p < 0) ? 0 : p;
        if (tie && mode != RANN_PCA_OFF) flags[1] = 1;
    }
}

// eigenvectors of T for the p largest eigenvalues by inverse iteration, one
// thread per vector (vector t <-> lam[m-1-t]); entry i of vector t is kept at
// Zt[i m + t] and its LU factors at LU[(f m + i) m + t]
constexpr int kIvLds = 17152;  // doubles of LDS for the factors and iterates of inverse iteration

// vectors of one inverse-iteration workgroup for width m: per vector five LDS
// arrays of m doubles (the factors of T - lam I and the iterate) and m bytes of
// swap flags, 41 m bytes.  The LDS sets how many workgroups run at once, so the
// workgroup takes as many vectors as fit.
__host__ __device__ inline int inviter_vectors(int m) {
    const int v = (int)((8LL * kIvLds) / (41LL * (m > 0 ? m : 1)));
    return v < 1 ? 1 : (v > 64 ? 64 : v);
}

// Inverse iteration on the tridiagonal T for the p largest eigenvalues: lane v
// of the workgroup takes vector t = y V + v (V = inviter_vectors(m)) <-> lam[m-1-t].
// T - lam I is factored once with partial pivoting (rows i, i+1 swapped when
// |sub| > |a_i|, tiny pivots replaced by +-eps_piv), the factors kept in LDS;
// then three sweeps (swaps and multipliers, then U z = y) from a fixed start
// vector, the normalisation of each iterate folded into the next sweep.  The
// result goes to Zt[i m + t].
__global__ void __launch_bounds__(64) k_inviter(const int32_t* __restrict__ mvec,
                                                double* __restrict__ Sall,
                                                const int64_t* __restrict__ s_off,
                                                const double* __restrict__ lam_all,
                                                const int32_t* __restrict__ p_out,
                                                const int64_t* __restrict__ m_off) {
    __shared__ double dd[kMaxWidth];
    __shared__ double ee[kMaxWidth];
    __shared__ double ea[kMaxWidth];
    __shared__ double fs[kIvLds];
    const int j = blockIdx.x;
    const int m = mvec[j];
    const int p = p_out[j];
    const int V = inviter_vectors(m);
    if ((int)blockIdx.y * V >= p) return;  // uniform per workgroup
    const int64_t mm = m;
    const double* tri = Sall + s_off[j] + scr_tri(mm);
    const double* lam = lam_all + m_off[j];
    double* Zt = Sall + s_off[j] + scr_LU(mm) + 5 * mm * mm;
    for (int i = threadIdx.x; i < m; i += 64) {
        const double e = (i + 1 < m) ? tri[mm + i] : 0.0;
        dd[i] = tri[i];
        ee[i] = e;
        ea[i] = fabs(e);
    }
    __syncthreads();
    const TriBounds tb = tri_bounds(dd, ea, m);
    const int v = threadIdx.x;
    const int t = blockIdx.y * V + v;
    if (v >= V || t >= p) return;
    const double eps_piv = DBL_EPSILON * tb.tnorm + tb.pivmin;
    const double lmb = lam[m - 1 - t];
    // entry i of this lane's arrays at [i V + v]
    const int64_t mv = (int64_t)m * V;
    double* fr = fs + v;           // reciprocal of the diagonal of U
    double* fb = fs + mv + v;      // first superdiagonal
    double* fc = fs + 2 * mv + v;  // second superdiagonal (fill-in)
    double* fm = fs + 3 * mv + v;  // multipliers
    double* z = fs + 4 * mv + v;   // the iterate
    unsigned char* fp = reinterpret_cast<unsigned char*>(fs + 5 * mv) + v;  // 1 where rows i, i+1 were swapped
    double ai = dd[0] - lmb, bi = ee[0];
    for (int i = 0; i + 1 < m; ++i) {
        const double sub = ee[i];
        const double an = dd[i + 1] - lmb;                 // a[i+1] before step i
        const double bn = (i + 2 < m) ? ee[i + 1] : 0.0;   // b[i+1] before step i
        const bool swap = fabs(ai) < fabs(sub);
        double a = swap ? sub : ai;
        if (!swap && fabs(a) < eps_piv) a = (a < 0.0) ? -eps_piv : eps_piv;
        const double ra = 1.0 / a;
        const double mu = (swap ? ai : sub) * ra;
        fr[i * V] = ra;
        fb[i * V] = swap ? an : bi;
        fc[i * V] = swap ? bn : 0.0;
        fm[i * V] = mu;
        fp[i * V] = swap ? 1 : 0;
        const double ai_n = swap ? bi - mu * an : an - mu * bi;
        bi = swap ? -mu * bn : bn;
        ai = ai_n;
    }
    if (fabs(ai) < eps_piv) ai = (ai < 0.0) ? -eps_piv : eps_piv;
    const double rlast = 1.0 / ai;
    // start vector 1 + sin(0.7 (i + 1) + 1.3 (t + 1)) / 2 by the angle-addition recurrence
    {
        double sn = sin(0.7 + 1.3 * (double)(t + 1)), cs = cos(0.7 + 1.3 * (double)(t + 1));
        const double s7 = sin(0.7), c7 = cos(0.7);
        for (int i = 0; i < m; ++i) {
            z[i * V] = 1.0 + 0.5 * sn;
            const double sn2 = sn * c7 + cs * s7;
            cs = cs * c7 - sn * s7;
            sn = sn2;
        }
    }
    double sc = 1.0;
    for (int iter = 0; iter < 3; ++iter) {
        // forward: the swaps and multipliers on the scaled iterate
        double zc = z[0] * sc;
        for (int i = 0; i + 1 < m; ++i) {
            const double zn = z[(i + 1) * V] * sc;
            const double mu = fm[i * V];
            const bool swap = fp[i * V] != 0;
            z[i * V] = swap ? zn : zc;
            zc = swap ? zc - mu * zn : zn - mu * zc;
        }
        // backward: U z = y
        double z1 = zc * rlast, z2 = 0.0;
        z[(m - 1) * V] = z1;
        double nn = z1 * z1;
        for (int i = m - 2; i >= 0; --i) {
            const double zi = (z[i * V] - fb[i * V] * z1 - fc[i * V] * z2) * fr[i * V];
            z[i * V] = zi;
            nn = fma(zi, zi, nn);
            z2 = z1;
            z1 = zi;
        }
        sc = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
    }
    for (int i = 0; i < m; ++i) Zt[(int64_t)i * mm + t] = z[i * V] * sc;
}

// orthonormalisation and y = Q z for the p vectors; one workgroup per matrix
__global__ void __launch_bounds__(kPT) k_vectors(const int32_t* __restrict__ mvec,
                                                 const int64_t* __restrict__ g_off,
                                                 const double* __restrict__ Gall,
                                                 double* __restrict__ Sall,
                                                 const int64_t* __restrict__ s_off,
                                                 double* __restrict__ Yall,
                                                 const int32_t* __restrict__ p_out) {
    __shared__ double lds[kLds];
    __shared__ double red[kPT / 64];
    __shared__ double Tm[kNB][kNB + 1];
    const int j = blockIdx.x;
    const int m = mvec[j];
    const int p = p_out[j];
    const int64_t mm = m;
    const double* A = Gall + g_off[j];
    double* Y = Yall + g_off[j];
    const double* tri = Sall + s_off[j] + scr_tri(mm);
    const double* taus = tri + 2 * mm;
    double* LU = Sall + s_off[j] + scr_LU(mm);
    double* Zt = LU + 5 * mm * mm;
    const int tid = threadIdx.x;
    // vectors as rows ([t][i]) in the LU area, which is free again
    for (int64_t e = tid; e < (int64_t)m * p; e += kPT) {
        const int i = (int)(e / p), t = (int)(e % p);
        LU[(int64_t)t * mm + i] = Zt[(int64_t)i * mm + t];
    }
    __syncthreads();
    // orthonormal basis in descending order
    double* Z = LU;
    double* Zb = Zt;
    bool done = false;
    if (p <= kQRMax && p > 1) {
        if (chol_qr(Z, Zb, p, m, lds)) {
            double* tsw = Z;
            Z = Zb;
            Zb = tsw;
            if (chol_qr(Z, Zb, p, m, lds)) {
                tsw = Z;
                Z = Zb;
                Zb = tsw;
                done = true;
            }
        }
    }
    if (!done) cgs2(Z, p, m, lds, red);
    __syncthreads();
    // leave the orthonormal rows in the LU area for the back-transform
    if (Z != LU)
        for (int64_t e = tid; e < (int64_t)m * p; e += kPT) {
            const int t = (int)(e / m), i = (int)(e % m);
            LU[(int64_t)t * mm + i] = Z[(int64_t)t * mm + i];
        }
}

// ---- 4. y = Q z for the vectors t0 .. t0 + nc - 1 of matrix j (workgroup
// (j, slice)), Q = H_0 ... H_{m-3}: panels last to first, each applied as
// I - V T V^T with V[q][r] = A[k0 + q][r] for r > k0 + q (zero otherwise).
// T^{-1} = diag(1 / tau) + strict_upper(V V^T), so T Z1 is one
// upper-triangular back substitution per column.  The slices are independent.
constexpr int kSlice = 24;  // vectors per back-transform workgroup
__global__ void __launch_bounds__(kPT) k_backxf(const int32_t* __restrict__ mvec,
                                                const int64_t* __restrict__ g_off,
                                                const double* __restrict__ Gall,
                                                double* __restrict__ Sall,
                                                const int64_t* __restrict__ s_off,
                                                double* __restrict__ Yall,
                                                const int32_t* __restrict__ p_out) {
    __shared__ double Vs[kNB * (kRC + 1)];
    __shared__ double Zs[kSlice * (kRC + 1)];
    __shared__ double Z1[kNB * (kSlice + 1)];
    __shared__ double Tm[kNB][kNB + 1];
    const int j = blockIdx.x;
    const int m = mvec[j];
    const int p = p_out[j];
    const int t0 = blockIdx.y * kSlice;
    if (t0 >= p) return;
    const int nc = (p - t0 < kSlice) ? p - t0 : kSlice;
    const int64_t mm = m;
    const double* A = Gall + g_off[j];
    double* Y = Yall + g_off[j];
    const double* tri = Sall + s_off[j] + scr_tri(mm);
    const double* taus = tri + 2 * mm;
    double* Z = Sall + s_off[j] + scr_LU(mm) + (int64_t)t0 * mm;  // rows of this slice
    const int tid = threadIdx.x;
    const int nref = (m >= 2) ? m - 2 : 0;
    const int ga = (tid < kNB * kNB) ? tid / kNB : 0, gb = (tid < kNB * kNB) ? tid % kNB : 0;
    // thread (q, t) of the V Z^T product
    static_assert(kNB * kSlice <= kPT, "one thread per (q, t)");
    const bool pact = tid < kNB * kSlice;
    const int pq = pact ? tid / kSlice : 0, pt = pact ? tid % kSlice : 0;
    for (int k0 = ((nref - 1) / kNB) * kNB; nref > 0 && k0 >= 0; k0 -= kNB) {
        const int nb = (k0 + kNB < nref) ? kNB : nref - k0;
        double acc = 0.0;
        double gacc = 0.0;  // (V V^T)[ga][gb]
        for (int r0 = k0 + 1; r0 < m; r0 += kRC) {
            for (int e = tid; e < kNB * kRC; e += kPT) {
                const int q = e / kRC, rr = e % kRC, r = r0 + rr;
                Vs[q * (kRC + 1) + rr] = (q < nb && r < m && r > k0 + q) ? A[(int64_t)(k0 + q) * mm + r] : 0.0;
            }
            for (int e = tid; e < nc * kRC; e += kPT) {
                const int t = e / kRC, rr = e % kRC, r = r0 + rr;
                Zs[t * (kRC + 1) + rr] = (r < m) ? Z[(int64_t)t * mm + r] : 0.0;
            }
            __syncthreads();
            if (pact && pq < nb && pt < nc) {
                const double* vq = Vs + pq * (kRC + 1);
                const double* zt = Zs + pt * (kRC + 1);
#pragma unroll 16
                for (int rr = 0; rr < kRC; ++rr) acc = fma(vq[rr], zt[rr], acc);
            }
            if (tid < kNB * kNB && ga < gb && gb < nb) {
                const double* va = Vs + ga * (kRC + 1);
                const double* vb = Vs + gb * (kRC + 1);
                for (int rr = 0; rr < kRC; ++rr) gacc = fma(va[rr], vb[rr], gacc);
            }
            __syncthreads();
        }
        if (pact) Z1[pq * (kSlice + 1) + pt] = (pq < nb && pt < nc) ? acc : 0.0;
        if (tid < kNB * kNB) Tm[ga][gb] = (ga < gb && gb < nb) ? gacc : 0.0;
        __syncthreads();
        // Z2 = T Z1: Z2[q] = tau_q (Z1[q] - sum_{b > q} (V V^T)[q][b] Z2[b])
        for (int c = tid; c < nc; c += kPT) {
            for (int q = nb - 1; q >= 0; --q) {
                double sacc = Z1[q * (kSlice + 1) + c];
                for (int b2 = q + 1; b2 < nb; ++b2) sacc -= Tm[q][b2] * Z1[b2 * (kSlice + 1) + c];
                Z1[q * (kSlice + 1) + c] = taus[k0 + q] * sacc;
            }
        }
        __syncthreads();
        // z_t[r] -= sum_q V[q][r] Z2[q][t] on rows > k0
        for (int r0 = k0 + 1; r0 < m; r0 += kRC) {
            for (int e = tid; e < kNB * kRC; e += kPT) {
                const int q = e / kRC, rr = e % kRC, r = r0 + rr;
                Vs[q * (kRC + 1) + rr] = (q < nb && r < m && r > k0 + q) ? A[(int64_t)(k0 + q) * mm + r] : 0.0;
            }
            __syncthreads();
            for (int e = tid; e < nc * kRC; e += kPT) {
                const int t = e / kRC, rr = e % kRC, r = r0 + rr;
                if (r < m) {
                    double sacc = 0.0;
                    for (int q = 0; q < nb; ++q) sacc = fma(Vs[q * (kRC + 1) + rr], Z1[q * (kSlice + 1) + t], sacc);
                    Z[(int64_t)t * mm + r] -= sacc;
                }
            }
            __syncthreads();
        }
    }
    // eigenvectors as columns of Y
    for (int64_t e = tid; e < (int64_t)m * nc; e += kPT) {
        const int i = (int)(e / nc), t = (int)(e % nc);
        Y[(int64_t)i * mm + t0 + t] = Z[(int64_t)t * mm + i];
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

int64_t eig_scratch_elems(int m) { return scr_LU(m) + 6LL * m * m; }

int eig_batched(Handle& h, double* G, const int64_t* d_g_off, double* S, const int64_t* d_s_off,
                double* Y, double tol, int mode, int32_t* d_p, double* d_eig, int32_t* d_flags) {
    const EigDims dims{h.geo.J, h.m.data(), h.d_m, h.d_m_off, h.sum_m};
    return eig_batched_dims(h, dims, G, d_g_off, S, d_s_off, Y, tol, mode, d_p, d_eig, d_flags, nullptr);
}

int eig_batched_dims(Handle& h, const EigDims& dm, double* G, const int64_t* d_g_off, double* S,
                     const int64_t* d_s_off, double* Y, double tol, int mode, int32_t* d_p, double* d_eig,
                     int32_t* d_flags, const int32_t* d_nvec) {
    const int J = dm.J;
    const int32_t* d_vec = d_nvec ? d_nvec : d_p;  // vectors computed per matrix
    KTimer kt_(h.stream, "k_eig");
    int mmax = 0;
    for (int j = 0; j < J; ++j) mmax = std::max(mmax, dm.m[j]);
    // tile lists of the trailing updates, one group per panel
    std::vector<int4> tasks;
    std::vector<int64_t> off;
    for (int k0 = 0; k0 < mmax; k0 += kNB) {
        off.push_back((int64_t)tasks.size());
        for (int j = 0; j < J; ++j) {
            const int n2 = dm.m[j] - (k0 + kNB);
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
        RDD_TRY(upload(h, d_tasks, tasks.data(), sizeof(int4) * tasks.size()));
    int pi = 0;
    for (int k0 = 0; k0 < mmax; k0 += kNB, ++pi) {
        if (mmax <= kPanelCols)
            hipLaunchKernelGGL(k_tri_panel<true>, dim3(J), dim3(kPT), 0, h.stream, dm.d_m, d_g_off, G, S,
                               d_s_off, k0);
        else
            hipLaunchKernelGGL(k_tri_panel<false>, dim3(J), dim3(kPT), 0, h.stream, dm.d_m, d_g_off, G, S,
                               d_s_off, k0);
        const int64_t cnt = off[pi + 1] - off[pi];
        if (cnt > 0)
            hipLaunchKernelGGL(k_tri_update, dim3((unsigned)cnt), dim3(256), 0, h.stream,
                               d_tasks + off[pi], dm.d_m, d_g_off, G, S, d_s_off, k0);
        RDD_HIP(hipGetLastError());
    }
    double* d_lam = nullptr;
    RDD_TRY(dev_alloc(h, &d_lam, (size_t)dm.sum_m));
    hipLaunchKernelGGL(k_bisect, dim3(J, (unsigned)((mmax + 15) / 16)), dim3(64), 0, h.stream, dm.d_m, S,
                       d_s_off, d_lam, dm.d_m_off, d_eig);
    hipLaunchKernelGGL(k_pcount, dim3(J), dim3(256), 0, h.stream, dm.d_m, S, d_s_off, d_lam, tol, mode,
                       d_p, dm.d_m_off, d_flags);
    int iv_y = 1;  // workgroups per matrix: enough for all m vectors
    for (int jj = 0; jj < J; ++jj) {
        const int V = inviter_vectors(dm.m[jj]);
        iv_y = std::max(iv_y, (dm.m[jj] + V - 1) / V);
    }
    hipLaunchKernelGGL(k_inviter, dim3(J, (unsigned)iv_y), dim3(64), 0, h.stream, dm.d_m, S,
                       d_s_off, d_lam, d_vec, dm.d_m_off);
    hipLaunchKernelGGL(k_vectors, dim3(J), dim3(kPT), 0, h.stream, dm.d_m, d_g_off, G, S, d_s_off, Y, d_vec);
    hipLaunchKernelGGL(k_backxf, dim3(J, (unsigned)((mmax + kSlice - 1) / kSlice)), dim3(kPT), 0, h.stream, dm.d_m,
                       d_g_off, G, S, d_s_off, Y, d_vec);
    kt_.stop();
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, d_tasks);
    dev_free(h, d_lam);
    return RANN_OK;
}

int compact_V(Handle& h, const double* Vfull, const int64_t* d_g_off, double* V) {
    hipLaunchKernelGGL(k_compact_V, dim3(h.geo.J), dim3(256), 0, h.stream, h.d_m, h.d_p, d_g_off,
                       h.d_v_off, Vfull, V);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace rdd
