// Batched FP64 symmetric eigensolver for the PCA step (paper Sec. 4).
//
// The reduced SVD of the value matrix Psi_j gives the right singular vectors V
// and sigma^2 = eigenvalues of Psi_j^T Psi_j; this kernel computes the latter
// eigendecomposition of the m_j x m_j Gram matrix, one workgroup per subdomain:
//   1. Householder reduction to tridiagonal form A = Q T Q^T,
//   2. implicit symmetric QR steps with Wilkinson shifts on (d, e); each step's
//      Givens rotations are chained by one thread and applied to the rows of Z
//      (eigenvectors of T, from the identity) by the whole workgroup,
//   3. eigenvalues sorted in descending order and the truncation count p_j,
//   4. only the p_j kept eigenvectors are transformed back by the reflectors
//      (y = Q z) and written as columns of an m_j x m_j row-major matrix.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "common.h"

namespace rdd {

namespace {

constexpr int kEigThreads = 512;

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

// A (m x m, row-major, symmetric) is reduced in place; the reflector of step k
// is kept in column k below the subdiagonal (untouched by later steps).
// Z (m x m) accumulates the QR rotations starting from the identity, so row i
// ends as eigenvector i of the tridiagonal matrix; Y receives the leading
// eigenvectors of A (columns, descending eigenvalue order).
__global__ void __launch_bounds__(kEigThreads) k_eig(const int32_t* __restrict__ mvec,
                                                     const int64_t* __restrict__ g_off,
                                                     double* __restrict__ Gall,
                                                     double* __restrict__ Zall,
                                                     double* __restrict__ Yall, double tol,
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
    __shared__ int perm[kMaxWidth];
    __shared__ double red[kEigThreads / 64];
    __shared__ int ctrl[4];
    const int j = blockIdx.x;
    const int m = mvec[j];
    double* A = Gall + g_off[j];
    double* Z = Zall + g_off[j];
    double* Y = Yall + g_off[j];
    const int tid = threadIdx.x;
    const int64_t mm = m;

    // ---- 1. Householder tridiagonalisation
    for (int k = 0; k + 2 < m; ++k) {
        const int n1 = m - k - 1;
        for (int i = tid; i < n1; i += kEigThreads) v[i] = A[(int64_t)k * mm + k + 1 + i];
        __syncthreads();
        double part = 0.0;
        for (int i = tid; i < n1; i += kEigThreads) part += v[i] * v[i];
        const double nrm2 = block_sum(part, red);
        const double v0 = v[0];
        if (tid == 0) dd[k] = A[(int64_t)k * mm + k];
        if (nrm2 == 0.0) {
            if (tid == 0) {
                ee[k] = 0.0;
                taus[k] = 0.0;
            }
            for (int i = tid; i < n1; i += kEigThreads) A[(int64_t)(k + 1 + i) * mm + k] = 0.0;
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
        // p = tau A' v, four independent partial sums per thread
        const double* Ap = A + (int64_t)(k + 1) * mm + (k + 1);
        double pv_part = 0.0;
        for (int i = tid; i < n1; i += kEigThreads) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int jj = 0;
            for (; jj + 3 < n1; jj += 4) {
                s0 = fma(Ap[(int64_t)jj * mm + i], v[jj], s0);
                s1 = fma(Ap[(int64_t)(jj + 1) * mm + i], v[jj + 1], s1);
                s2 = fma(Ap[(int64_t)(jj + 2) * mm + i], v[jj + 2], s2);
                s3 = fma(Ap[(int64_t)(jj + 3) * mm + i], v[jj + 3], s3);
            }
            for (; jj < n1; ++jj) s0 = fma(Ap[(int64_t)jj * mm + i], v[jj], s0);
            const double s = tau * ((s0 + s1) + (s2 + s3));
            w[i] = s;
            pv_part += s * v[i];
        }
        const double pv = block_sum(pv_part, red);
        const double K = 0.5 * tau * pv;
        for (int i = tid; i < n1; i += kEigThreads) w[i] -= K * v[i];
        __syncthreads();
        double* Aw = A + (int64_t)(k + 1) * mm + (k + 1);
        for (int i = tid; i < n1; i += kEigThreads) {
            const double vi = v[i], wi = w[i];
            int jj = 0;
            for (; jj + 3 < n1; jj += 4) {
                double a0 = Aw[(int64_t)jj * mm + i], a1 = Aw[(int64_t)(jj + 1) * mm + i];
                double a2 = Aw[(int64_t)(jj + 2) * mm + i], a3 = Aw[(int64_t)(jj + 3) * mm + i];
                Aw[(int64_t)jj * mm + i] = a0 - (v[jj] * wi + w[jj] * vi);
                Aw[(int64_t)(jj + 1) * mm + i] = a1 - (v[jj + 1] * wi + w[jj + 1] * vi);
                Aw[(int64_t)(jj + 2) * mm + i] = a2 - (v[jj + 2] * wi + w[jj + 2] * vi);
                Aw[(int64_t)(jj + 3) * mm + i] = a3 - (v[jj + 3] * wi + w[jj + 3] * vi);
            }
            for (; jj < n1; ++jj) Aw[(int64_t)jj * mm + i] -= v[jj] * wi + w[jj] * vi;
        }
        __syncthreads();
        // keep the reflector in column k below the diagonal
        for (int i = tid; i < n1; i += kEigThreads) A[(int64_t)(k + 1 + i) * mm + k] = v[i];
        __syncthreads();
    }
    if (tid == 0) {
        if (m >= 2) {
            dd[m - 2] = A[(int64_t)(m - 2) * mm + m - 2];
            ee[m - 2] = A[(int64_t)(m - 2) * mm + m - 1];
            taus[m - 2] = 0.0;
        }
        dd[m - 1] = A[(int64_t)(m - 1) * mm + m - 1];
        ee[m - 1] = 0.0;
    }
    // ---- 2. Z = I
    for (int64_t e = tid; e < mm * mm; e += kEigThreads) Z[e] = ((e / mm) == (e % mm)) ? 1.0 : 0.0;
    __syncthreads();
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
                double delta = 0.5 * (dd[hi - 1] - dd[hi]);
                double eh = ee[hi - 1];
                double den = delta + copysign(sqrt(delta * delta + eh * eh), delta);
                double mu = dd[hi] - (den != 0.0 ? eh * eh / den : 0.0);
                double x = dd[lo] - mu, z = ee[lo];
                for (int k = lo; k < hi; ++k) {
                    double r2 = x * x + z * z;
                    double c = 1.0, s = 0.0, r = 0.0;
                    if (r2 > 0.0) {
                        r = sqrt(r2);
                        double inv = 1.0 / r;
                        c = x * inv;
                        s = z * inv;
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
        }
        __syncthreads();
        const int lo_s = ctrl[0], hi_s = ctrl[1];
        if (lo_s < 0) break;
        for (int c = tid; c < m; c += kEigThreads) {
            double carry = Z[(int64_t)lo_s * mm + c];
            int k = lo_s;
            for (; k + 3 < hi_s; k += 4) {
                const double b0 = Z[(int64_t)(k + 1) * mm + c], b1 = Z[(int64_t)(k + 2) * mm + c];
                const double b2 = Z[(int64_t)(k + 3) * mm + c], b3 = Z[(int64_t)(k + 4) * mm + c];
                Z[(int64_t)k * mm + c] = cs[k] * carry + sn[k] * b0;
                carry = -sn[k] * carry + cs[k] * b0;
                Z[(int64_t)(k + 1) * mm + c] = cs[k + 1] * carry + sn[k + 1] * b1;
                carry = -sn[k + 1] * carry + cs[k + 1] * b1;
                Z[(int64_t)(k + 2) * mm + c] = cs[k + 2] * carry + sn[k + 2] * b2;
                carry = -sn[k + 2] * carry + cs[k + 2] * b2;
                Z[(int64_t)(k + 3) * mm + c] = cs[k + 3] * carry + sn[k + 3] * b3;
                carry = -sn[k + 3] * carry + cs[k + 3] * b3;
            }
            for (; k < hi_s; ++k) {
                const double b = Z[(int64_t)(k + 1) * mm + c];
                Z[(int64_t)k * mm + c] = cs[k] * carry + sn[k] * b;
                carry = -sn[k] * carry + cs[k] * b;
            }
            Z[(int64_t)hi_s * mm + c] = carry;
        }
        __syncthreads();
    }
    if (tid == 0 && hi > 0) flags[0] = 1;  // did not converge
    // ---- 4. sort descending, threshold
    __shared__ double lam1_s;
    for (int i = tid; i < m; i += kEigThreads) {
        double di = dd[i];
        int rank = 0;
        for (int q = 0; q < m; ++q) {
            double dq = dd[q];
            rank += (dq > di || (dq == di && q < i)) ? 1 : 0;
        }
        perm[rank] = i;
    }
    __syncthreads();
    if (tid == 0) lam1_s = dd[perm[0]];
    __syncthreads();
    const double lam1 = lam1_s;
    const double thr = (mode == RANN_PCA_REL_EIG) ? tol * lam1 : tol * tol;
    int cnt = 0, tie = 0;
    for (int i = tid; i < m; i += kEigThreads) {
        double li = dd[perm[i]];
        eig_out[m_off[j] + i] = li;
        cnt += (li > thr) ? 1 : 0;
        tie |= (fabs(li - thr) <= 1e-6 * fabs(thr)) ? 1 : 0;
    }
    const double cnt_all = block_sum((double)cnt, red);
    const double tie_all = block_sum((double)tie, red);
    const int p = (mode == RANN_PCA_OFF) ? m : (int)cnt_all;
    if (tid == 0) {
        p_out[j] = p;
        if (tie_all > 0.0 && mode != RANN_PCA_OFF) flags[1] = 1;
    }
    // ---- 5. eigenvectors of A for the leading p: y = Q z, Q = H_0 H_1 ... H_{m-3}
    // thread per vector; Y[i][kk] holds component i of vector kk
    for (int kk = tid; kk < p; kk += kEigThreads) {
        const double* zr = Z + (int64_t)perm[kk] * mm;
        for (int i = 0; i < m; ++i) Y[(int64_t)i * mm + kk] = zr[i];
        for (int k = m - 3; k >= 0; --k) {
            const double tau = taus[k];
            if (tau == 0.0) continue;
            double s = 0.0;
            for (int i = k + 1; i < m; ++i) s = fma(A[(int64_t)i * mm + k], Y[(int64_t)i * mm + kk], s);
            s *= tau;
            for (int i = k + 1; i < m; ++i) Y[(int64_t)i * mm + kk] -= s * A[(int64_t)i * mm + k];
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

int eig_batched(Handle& h, double* G, const int64_t* d_g_off, double* Z, double* Y, double tol,
                int mode, int32_t* d_p, double* d_eig, int32_t* d_flags) {
    KTimer kt_(h.stream, "k_eig");
    hipLaunchKernelGGL(k_eig, dim3(h.geo.J), dim3(kEigThreads), 0, h.stream, h.d_m, d_g_off, G, Z, Y,
                       tol, mode, d_p, d_eig, h.d_m_off, d_flags);
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
