// Batched FP64 symmetric eigensolver for the PCA step (paper Sec. 4).
//
// The reduced SVD of the value matrix Psi_j gives the right singular vectors V
// and sigma^2 = eigenvalues of Psi_j^T Psi_j; this kernel computes the latter
// eigendecomposition of the m_j x m_j Gram matrix, one workgroup per subdomain:
//   1. Householder reduction to tridiagonal form A = Q T Q^T,
//   2. Z = Q^T accumulated from the reflectors,
//   3. implicit symmetric QR steps with Wilkinson shifts on (d, e); each step's
//      Givens rotations are chained by one thread and applied to the rows of Z
//      by the whole workgroup (every thread owns columns of Z),
//   4. eigenvalues sorted in descending order, the truncation count p_j, and
//      the eigenvectors written as columns of an m_j x m_j row-major matrix.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "common.h"

namespace rdd {

namespace {

constexpr int kEigThreads = 256;

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

__global__ void __launch_bounds__(kEigThreads) k_eig(const int32_t* __restrict__ mvec,
                                                     const int64_t* __restrict__ g_off,
                                                     double* __restrict__ Gall,
                                                     double* __restrict__ Zall, double tol,
                                                     int mode, int32_t* __restrict__ p_out,
                                                     double* __restrict__ eig_out,
                                                     const int64_t* __restrict__ m_off,
                                                     int32_t* __restrict__ flags) {
    __shared__ double v[kMaxWidth];
    __shared__ double w[kMaxWidth];
    __shared__ double dd[kMaxWidth];
    __shared__ double ee[kMaxWidth];
    __shared__ double cs[kMaxWidth];
    __shared__ double sn[kMaxWidth];
    __shared__ double taus[kMaxWidth];
    __shared__ double red[kEigThreads / 64];
    __shared__ int ctrl[4];
    const int j = blockIdx.x;
    const int m = mvec[j];
    double* A = Gall + g_off[j];
    double* Z = Zall + g_off[j];
    const int tid = threadIdx.x;

    // ---- 1. tridiagonalisation
    for (int k = 0; k + 2 < m; ++k) {
        const int n1 = m - k - 1;
        for (int i = tid; i < n1; i += kEigThreads) v[i] = A[(int64_t)k * m + k + 1 + i];
        __syncthreads();
        double part = 0.0;
        for (int i = tid; i < n1; i += kEigThreads) part += v[i] * v[i];
        const double nrm2 = block_sum(part, red);
        const double v0 = v[0];
        if (tid == 0) dd[k] = A[(int64_t)k * m + k];
        if (nrm2 == 0.0) {
            if (tid == 0) {
                ee[k] = 0.0;
                taus[k] = 0.0;
            }
            __syncthreads();
            continue;
        }
        const double alpha = (v0 >= 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
        const double vtv = 2.0 * (nrm2 - v0 * alpha);
        const double tau = 2.0 / vtv;
        __syncthreads();
        if (tid == 0) {
            v[0] = v0 - alpha;
            ee[k] = alpha;
            taus[k] = tau;
        }
        __syncthreads();
        // p = tau A' v  (A' = trailing block, symmetric; read by rows for coalescing)
        const double* Ap = A + (int64_t)(k + 1) * m + (k + 1);
        double pv_part = 0.0;
        for (int i = tid; i < n1; i += kEigThreads) {
            double s = 0.0;
            for (int jj = 0; jj < n1; ++jj) s = fma(Ap[(int64_t)jj * m + i], v[jj], s);
            s *= tau;
            w[i] = s;
            pv_part += s * v[i];
        }
        const double pv = block_sum(pv_part, red);
        const double K = 0.5 * tau * pv;
        for (int i = tid; i < n1; i += kEigThreads) w[i] -= K * v[i];
        __syncthreads();
        double* Aw = A + (int64_t)(k + 1) * m + (k + 1);
        for (int i = tid; i < n1; i += kEigThreads) {
            const double vi = v[i], wi = w[i];
            for (int jj = 0; jj < n1; ++jj) {
                double* a = Aw + (int64_t)jj * m + i;
                *a -= v[jj] * wi + w[jj] * vi;
            }
        }
        // keep the reflector in row k (beyond the diagonal) for step 2
        for (int i = tid; i < n1; i += kEigThreads) A[(int64_t)k * m + k + 1 + i] = v[i];
        __syncthreads();
    }
    if (tid == 0) {
        if (m >= 2) {
            dd[m - 2] = A[(int64_t)(m - 2) * m + m - 2];
            ee[m - 2] = A[(int64_t)(m - 2) * m + m - 1];
            taus[m - 2] = 0.0;
        }
        dd[m - 1] = A[(int64_t)(m - 1) * m + m - 1];
        ee[m - 1] = 0.0;
    }
    // ---- 2. Z = Q^T = H_{m-3} ... H_0
    for (int64_t e = tid; e < (int64_t)m * m; e += kEigThreads)
        Z[e] = ((e / m) == (e % m)) ? 1.0 : 0.0;
    __syncthreads();
    for (int k = 0; k + 2 < m; ++k) {
        const int n1 = m - k - 1;
        const double tau = taus[k];
        if (tau == 0.0) continue;  // uniform across the workgroup
        for (int i = tid; i < n1; i += kEigThreads) v[i] = A[(int64_t)k * m + k + 1 + i];
        __syncthreads();
        for (int c = tid; c < m; c += kEigThreads) {
            double u = 0.0;
            for (int i = 0; i < n1; ++i) u = fma(v[i], Z[(int64_t)(k + 1 + i) * m + c], u);
            u *= tau;
            if (u != 0.0)
                for (int i = 0; i < n1; ++i) Z[(int64_t)(k + 1 + i) * m + c] -= v[i] * u;
        }
        __syncthreads();
    }
    // ---- 3. implicit symmetric QR with Wilkinson shifts
    int hi = m - 1;
    int guard = 0;
    const int max_steps = 40 * m + 40;
    while (true) {
        if (tid == 0) {
            int lo = -1;
            while (hi > 0) {
                double t = fabs(dd[hi - 1]) + fabs(dd[hi]);
                if (fabs(ee[hi - 1]) <= DBL_EPSILON * t) {
                    ee[hi - 1] = 0.0;
                    --hi;
                } else {
                    break;
                }
            }
            if (hi > 0 && guard < max_steps) {
                lo = hi - 1;
                while (lo > 0) {
                    double t = fabs(dd[lo - 1]) + fabs(dd[lo]);
                    if (fabs(ee[lo - 1]) <= DBL_EPSILON * t) {
                        ee[lo - 1] = 0.0;
                        break;
                    }
                    --lo;
                }
                // one shifted QR step on [lo, hi]
                double delta = 0.5 * (dd[hi - 1] - dd[hi]);
                double eh = ee[hi - 1];
                double den = delta + copysign(hypot(delta, eh), delta);
                double mu = dd[hi] - (den != 0.0 ? eh * eh / den : 0.0);
                double x = dd[lo] - mu, z = ee[lo];
                for (int k = lo; k < hi; ++k) {
                    double r = hypot(x, z);
                    double c = 1.0, s = 0.0;
                    if (r != 0.0) {
                        c = x / r;
                        s = z / r;
                    }
                    if (k > lo) ee[k - 1] = r;
                    double a = dd[k], b = ee[k], d1 = dd[k + 1];
                    double cc = c * c, ss = s * s, csb = 2.0 * c * s * b;
                    dd[k] = cc * a + csb + ss * d1;
                    dd[k + 1] = ss * a - csb + cc * d1;
                    ee[k] = c * s * (d1 - a) + (cc - ss) * b;
                    if (k + 1 < hi) {
                        x = ee[k];
                        z = s * ee[k + 1];
                        ee[k + 1] *= c;
                    }
                    cs[k] = c;
                    sn[k] = s;
                }
                ++guard;
            }
            ctrl[0] = lo;
            ctrl[1] = hi;
            ctrl[2] = guard;
        }
        __syncthreads();
        const int lo_s = ctrl[0], hi_s = ctrl[1];
        if (lo_s < 0) break;
        for (int c = tid; c < m; c += kEigThreads) {
            double carry = Z[(int64_t)lo_s * m + c];
            for (int k = lo_s; k < hi_s; ++k) {
                double b = Z[(int64_t)(k + 1) * m + c];
                Z[(int64_t)k * m + c] = cs[k] * carry + sn[k] * b;
                carry = -sn[k] * carry + cs[k] * b;
            }
            Z[(int64_t)hi_s * m + c] = carry;
        }
        __syncthreads();
        guard = ctrl[2];
    }
    __syncthreads();
    if (tid == 0 && hi > 0) flags[0] = 1;  // did not converge
    // ---- 4. sort descending, threshold, write eigenvectors as columns
    __shared__ double lam1_s;
    for (int i = tid; i < m; i += kEigThreads) {
        double di = dd[i];
        int rank = 0;
        for (int q = 0; q < m; ++q) {
            double dq = dd[q];
            rank += (dq > di || (dq == di && q < i)) ? 1 : 0;
        }
        w[rank] = (double)i;  // permutation (exact small integers)
    }
    __syncthreads();
    if (tid == 0) lam1_s = dd[(int)w[0]];
    __syncthreads();
    const double lam1 = lam1_s;
    const double thr = (mode == RANN_PCA_REL_EIG) ? tol * lam1 : tol * tol;
    int cnt = 0, tie = 0;
    for (int i = tid; i < m; i += kEigThreads) {
        double li = dd[(int)w[i]];
        eig_out[m_off[j] + i] = li;
        cnt += (li > thr) ? 1 : 0;
        tie |= (fabs(li - thr) <= 1e-6 * fabs(thr)) ? 1 : 0;
    }
    double cnt_all = block_sum((double)cnt, red);
    double tie_all = block_sum((double)tie, red);
    if (tid == 0) {
        p_out[j] = (mode == RANN_PCA_OFF) ? m : (int)cnt_all;
        if (tie_all > 0.0 && mode != RANN_PCA_OFF) flags[1] = 1;
    }
    // A <- eigenvectors as columns: A[r][k] = Z[perm[k]][r]
    for (int64_t e = tid; e < (int64_t)m * m; e += kEigThreads) {
        int r = (int)(e / m), k = (int)(e % m);
        A[e] = Z[(int64_t)(int)w[k] * m + r];
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

int eig_batched(Handle& h, double* G, const int64_t* d_g_off, double* Z, double tol, int mode,
                int32_t* d_p, double* d_eig, int32_t* d_flags) {
    hipLaunchKernelGGL(k_eig, dim3(h.geo.J), dim3(kEigThreads), 0, h.stream, h.d_m, d_g_off, G, Z,
                       tol, mode, d_p, d_eig, h.d_m_off, d_flags);
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
