// Batched FP64 symmetric eigensolver for the PCA step (paper Sec. 4).
//
// The reduced SVD of the value matrix Psi_j gives the right singular vectors V
// and sigma^2 = eigenvalues of Psi_j^T Psi_j; this kernel computes the latter
// eigendecomposition of the m_j x m_j Gram matrix, one workgroup per subdomain:
//   1. Householder reduction to tridiagonal form A = Q T Q^T (2D thread map:
//      64 columns x 8 row groups per pass over the trailing block),
//   2. every eigenvalue of T by Sturm-count bisection, one thread per
//      eigenvalue; the truncation count p is the Sturm count at the threshold,
//   3. eigenvectors of T for the p largest eigenvalues by inverse iteration
//      (tridiagonal LU with partial pivoting, one thread per vector), then
//      classical Gram-Schmidt applied twice in descending order,
//   4. y = Q z for the p vectors (reflectors stored row-wise, 2D thread map),
//      written as columns of an m_j x m_j row-major matrix.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "common.h"

namespace rdd {

namespace {

constexpr int kEigThreads = 512;
constexpr int kCols = 64, kRowGroups = kEigThreads / kCols;

__device__ double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kEigThreads / 64; ++w) s += red[w];
    return s;
}

// number of eigenvalues of the tridiagonal (d, e) smaller than x (e2 = e^2)
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

// A (m x m, row-major, symmetric) is reduced in place; the reflector of step k
// is kept in row k right of the diagonal (untouched by later steps).  S is the
// per-subdomain scratch (6 m^2 doubles): the tridiagonal eigenvectors (m x m)
// followed by the LU factors of the inverse iterations (5m per vector).  Y
// receives the leading eigenvectors of A as columns, descending eigenvalues.
__global__ void __launch_bounds__(kEigThreads) k_eig(const int32_t* __restrict__ mvec,
                                                     const int64_t* __restrict__ g_off,
                                                     double* __restrict__ Gall,
                                                     double* __restrict__ Sall,
                                                     double* __restrict__ Yall,
                                                     const int64_t* __restrict__ s_off,
                                                     double tol, int mode,
                                                     int32_t* __restrict__ p_out,
                                                     double* __restrict__ eig_out,
                                                     const int64_t* __restrict__ m_off,
                                                     int32_t* __restrict__ flags) {
    __shared__ double v[kMaxWidth];
    __shared__ double w[kMaxWidth];
    __shared__ double dd[kMaxWidth];
    __shared__ double ee[kMaxWidth];
    __shared__ double e2[kMaxWidth];
    __shared__ double lam[kMaxWidth];   // ascending eigenvalues of T
    __shared__ double taus[kMaxWidth];
    __shared__ double hcoef[kMaxWidth];
    __shared__ double part[kRowGroups][kCols + 1];
    __shared__ double red[kEigThreads / 64];
    const int j = blockIdx.x;
    const int m = mvec[j];
    double* A = Gall + g_off[j];
    double* Y = Yall + g_off[j];
    double* S = Sall + s_off[j];
    const int tid = threadIdx.x;
    const int tc = tid % kCols, tr = tid / kCols;
    const int64_t mm = m;

    // ---- 1. Householder tridiagonalisation
    for (int k = 0; k + 2 < m; ++k) {
        const int n1 = m - k - 1;
        for (int i = tid; i < n1; i += kEigThreads) v[i] = A[(int64_t)k * mm + k + 1 + i];
        __syncthreads();
        double pp = 0.0;
        for (int i = tid; i < n1; i += kEigThreads) pp += v[i] * v[i];
        const double nrm2 = block_sum(pp, red);
        const double v0 = v[0];
        if (tid == 0) dd[k] = A[(int64_t)k * mm + k];
        if (nrm2 == 0.0) {
            if (tid == 0) {
                ee[k] = 0.0;
                taus[k] = 0.0;
            }
            __syncthreads();
            continue;
        }
        const double alpha = (v0 >= 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
        const double tau = 1.0 / (nrm2 - v0 * alpha);  // 2 / v^T v
        __syncthreads();
        if (tid == 0) {
            v[0] = v0 - alpha;
            ee[k] = alpha;
            taus[k] = tau;
        }
        __syncthreads();
        // w = tau A' v: columns in passes of 64, 8 row groups each
        const double* Ap = A + (int64_t)(k + 1) * mm + (k + 1);
        double pv_part = 0.0;
        for (int c0 = 0; c0 < n1; c0 += kCols) {
            const int c = c0 + tc;
            double s0 = 0.0, s1 = 0.0;
            if (c < n1) {
                int jj = tr;
                for (; jj + kRowGroups < n1; jj += 2 * kRowGroups) {
                    s0 = fma(Ap[(int64_t)jj * mm + c], v[jj], s0);
                    s1 = fma(Ap[(int64_t)(jj + kRowGroups) * mm + c], v[jj + kRowGroups], s1);
                }
                if (jj < n1) s0 = fma(Ap[(int64_t)jj * mm + c], v[jj], s0);
            }
            part[tr][tc] = s0 + s1;
            __syncthreads();
            if (tr == 0 && c < n1) {
                double s = 0.0;
                for (int g = 0; g < kRowGroups; ++g) s += part[g][tc];
                s *= tau;
                w[c] = s;
                pv_part += s * v[c];
            }
            __syncthreads();
        }
        const double pv = block_sum(pv_part, red);
        const double K = 0.5 * tau * pv;
        for (int i = tid; i < n1; i += kEigThreads) w[i] -= K * v[i];
        __syncthreads();
        double* Aw = A + (int64_t)(k + 1) * mm + (k + 1);
        for (int c0 = 0; c0 < n1; c0 += kCols) {
            const int c = c0 + tc;
            if (c < n1) {
                const double vc = v[c], wc = w[c];
                for (int jj = tr; jj < n1; jj += kRowGroups) {
                    double* a = Aw + (int64_t)jj * mm + c;
                    *a -= v[jj] * wc + w[jj] * vc;
                }
            }
        }
        __syncthreads();
        // keep the reflector in row k right of the diagonal
        for (int i = tid; i < n1; i += kEigThreads) A[(int64_t)k * mm + k + 1 + i] = v[i];
        __syncthreads();
    }
    if (tid == 0) {
        if (m >= 2) {
            dd[m - 2] = A[(int64_t)(m - 2) * mm + m - 2];
            ee[m - 2] = A[(int64_t)(m - 1) * mm + m - 2];
            taus[m - 2] = 0.0;
        }
        dd[m - 1] = A[(int64_t)(m - 1) * mm + m - 1];
        ee[m - 1] = 0.0;
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
    for (int i = tid; i < m; i += kEigThreads) e2[i] = (i + 1 < m) ? ee[i] * ee[i] : 0.0;
    __syncthreads();
    const double pivmin = DBL_MIN * fmax(1.0, tnorm * tnorm);
    const double atol = 2.0 * DBL_EPSILON * tnorm + pivmin;
    for (int idx = tid; idx < m; idx += kEigThreads) {
        // the idx-th smallest eigenvalue: count(lo) <= idx < count(hi)
        double lo = gl - atol, hi = gu + atol;
        for (int it = 0; it < 200; ++it) {
            if (!((hi - lo) > atol + 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)))) break;
            const double mid = 0.5 * (lo + hi);
            if (sturm_count(dd, e2, m, mid, pivmin) > idx) hi = mid; else lo = mid;
        }
        lam[idx] = 0.5 * (lo + hi);
    }
    __syncthreads();
    const double lam1 = lam[m - 1];
    const double thr = (mode == RANN_PCA_REL_EIG) ? tol * lam1 : tol * tol;
    int p = m;
    if (mode != RANN_PCA_OFF) p = m - sturm_count(dd, e2, m, thr, pivmin);  // same in every thread
    if (p < 0) p = 0;
    for (int i = tid; i < m; i += kEigThreads) eig_out[m_off[j] + i] = lam[m - 1 - i];
    if (tid == 0) {
        p_out[j] = p;
        int tie = 0;
        for (int i = 0; i < m; ++i) tie |= (fabs(lam[i] - thr) <= 1e-6 * fabs(thr)) ? 1 : 0;
        if (tie && mode != RANN_PCA_OFF) flags[1] = 1;
    }
    // ---- 3. inverse iteration for the p largest: vector t <-> eigenvalue lam[m-1-t]
    double* Z = S;
    double* LU = S + mm * mm;
    const double eps_piv = DBL_EPSILON * tnorm + pivmin;
    for (int t = tid; t < p; t += kEigThreads) {
        const double lmb = lam[m - 1 - t];
        double* a = LU + (int64_t)t * 5 * mm;  // diagonal of U
        double* b = a + mm;                     // first superdiagonal
        double* c2 = b + mm;                    // second superdiagonal (fill-in)
        double* ml = c2 + mm;                   // multipliers
        double* pv = ml + mm;                   // 1.0 where rows i, i+1 were swapped
        for (int i = 0; i < m; ++i) {
            a[i] = dd[i] - lmb;
            b[i] = (i + 1 < m) ? ee[i] : 0.0;
            c2[i] = 0.0;
        }
        for (int i = 0; i + 1 < m; ++i) {
            const double sub = ee[i];
            if (fabs(a[i]) >= fabs(sub)) {
                double ai = a[i];
                if (fabs(ai) < eps_piv) ai = (ai < 0.0) ? -eps_piv : eps_piv;
                a[i] = ai;
                const double mu = sub / ai;
                ml[i] = mu;
                pv[i] = 0.0;
                a[i + 1] -= mu * b[i];
            } else {
                const double mu = a[i] / sub;
                ml[i] = mu;
                pv[i] = 1.0;
                a[i] = sub;
                const double tmp = a[i + 1];
                a[i + 1] = b[i] - mu * tmp;
                b[i] = tmp;
                if (i + 2 < m) {
                    c2[i] = b[i + 1];
                    b[i + 1] = -mu * b[i + 1];
                }
            }
        }
        if (fabs(a[m - 1]) < eps_piv) a[m - 1] = (a[m - 1] < 0.0) ? -eps_piv : eps_piv;
        double* z = Z + (int64_t)t * mm;
        for (int i = 0; i < m; ++i) z[i] = 1.0 + 0.5 * sin(0.7 * (double)(i + 1) + 1.3 * (double)(t + 1));
        for (int iter = 0; iter < 3; ++iter) {
            for (int i = 0; i + 1 < m; ++i) {
                if (pv[i] != 0.0) {
                    const double tmp = z[i];
                    z[i] = z[i + 1];
                    z[i + 1] = tmp - ml[i] * z[i + 1];
                } else {
                    z[i + 1] -= ml[i] * z[i];
                }
            }
            z[m - 1] /= a[m - 1];
            if (m >= 2) z[m - 2] = (z[m - 2] - b[m - 2] * z[m - 1]) / a[m - 2];
            for (int i = m - 3; i >= 0; --i) z[i] = (z[i] - b[i] * z[i + 1] - c2[i] * z[i + 2]) / a[i];
            double nn = 0.0;
            for (int i = 0; i < m; ++i) nn = fma(z[i], z[i], nn);
            const double inv = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
            for (int i = 0; i < m; ++i) z[i] *= inv;
        }
    }
    __syncthreads();
    // classical Gram-Schmidt, twice, in descending eigenvalue order
    for (int t = 1; t < p; ++t) {
        double* zt = Z + (int64_t)t * mm;
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = tid; q < t; q += kEigThreads) {
                const double* zq = Z + (int64_t)q * mm;
                double s = 0.0;
                for (int i = 0; i < m; ++i) s = fma(zq[i], zt[i], s);
                hcoef[q] = s;
            }
            __syncthreads();
            for (int i = tid; i < m; i += kEigThreads) {
                double acc = zt[i];
                for (int q = 0; q < t; ++q) acc -= hcoef[q] * Z[(int64_t)q * mm + i];
                zt[i] = acc;
            }
            __syncthreads();
        }
        double pp2 = 0.0;
        for (int i = tid; i < m; i += kEigThreads) pp2 += zt[i] * zt[i];
        const double nn = block_sum(pp2, red);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int i = tid; i < m; i += kEigThreads) zt[i] *= inv;
        __syncthreads();
    }
    // ---- 4. y_t = Q z_t with Q = H_0 ... H_{m-3}; Y[i][t]
    for (int64_t e = tid; e < (int64_t)m * p; e += kEigThreads) {
        const int i = (int)(e / p), t = (int)(e % p);
        Y[(int64_t)i * mm + t] = Z[(int64_t)t * mm + i];
    }
    __syncthreads();
    for (int k = m - 3; k >= 0; --k) {
        const double tau = taus[k];
        if (tau == 0.0) continue;  // uniform across the workgroup
        const int n1 = m - k - 1;
        for (int i = tid; i < n1; i += kEigThreads) v[i] = A[(int64_t)k * mm + k + 1 + i];
        __syncthreads();
        for (int c0 = 0; c0 < p; c0 += kCols) {
            const int t = c0 + tc;
            double s0 = 0.0;
            if (t < p)
                for (int i = tr; i < n1; i += kRowGroups) s0 = fma(v[i], Y[(int64_t)(k + 1 + i) * mm + t], s0);
            part[tr][tc] = s0;
            __syncthreads();
            if (tr == 0 && t < p) {
                double s = 0.0;
                for (int g = 0; g < kRowGroups; ++g) s += part[g][tc];
                w[t] = tau * s;
            }
            __syncthreads();
        }
        for (int64_t e = tid; e < (int64_t)n1 * p; e += kEigThreads) {
            const int i = (int)(e / p), t = (int)(e % p);
            Y[(int64_t)(k + 1 + i) * mm + t] -= w[t] * v[i];
        }
        __syncthreads();
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

int eig_batched(Handle& h, double* G, const int64_t* d_g_off, double* S, const int64_t* d_s_off,
                double* Y, double tol, int mode, int32_t* d_p, double* d_eig, int32_t* d_flags) {
    KTimer kt_(h.stream, "k_eig");
    hipLaunchKernelGGL(k_eig, dim3(h.geo.J), dim3(kEigThreads), 0, h.stream, h.d_m, d_g_off, G, S, Y,
                       d_s_off, tol, mode, d_p, d_eig, h.d_m_off, d_flags);
    kt_.stop();
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    return RANN_OK;
}

int compact_V(Handle& h, const double* Vfull, const int64_t* d_g_off, double* V) {
    hipLaunchKernelGGL(k_compact_V, dim3(h.geo.J), dim3(256), 0, h.stream, h.d_m, h.d_p, d_g_off,
                       h.d_v_off, Vfull, V);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace rdd
