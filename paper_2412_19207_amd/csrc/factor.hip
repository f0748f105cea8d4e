// Local inverses of the Schwarz blocks on matrix cores (paper Sec. 3: the
// local inverse A_i^{-1} of A_i = R_i H^T H R_i^T).
//
// One workgroup per block, 64x64 tiles, three blocked phases:
//   1. right-looking Cholesky of D A D + eps I = L L^T (D = diag(A)^{-1/2}):
//      diagonal tile factored in LDS, panel = A_ik L_kk^{-T} and trailing
//      update A_ij -= P_i P_j^T on MFMA;
//   2. X = L^{-1}: diagonal tiles inverted in LDS, then
//      X_ik = -X_ii sum_{j=k}^{i-1} L_ij X_jk on MFMA;
//   3. A^{-1} = D X^T X D, lower tiles on MFMA, mirrored.
// A pivot that is not positive restarts the factorisation with a diagonal
// shift eps = 10 u q, growing tenfold (counted in `shifts`).
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "common.h"
#include "mfma.h"

namespace rdd {

namespace {

template <class T>
struct Unit;
template <>
struct Unit<double> { static constexpr double u = DBL_EPSILON; };
template <>
struct Unit<float> { static constexpr double u = FLT_EPSILON; };

constexpr int kFT = 256;  // threads

// Stage one BK slice of a 64-wide operand into LDS (k-major).
//  kAlongRows: element (kk, m) = src[(r0 + k0 + kk) * ld + c0 + m]
//  otherwise : element (kk, m) = src[(r0 + m) * ld + c0 + k0 + kk]
template <class T, bool kAlongRows>
__device__ __forceinline__ void stage(T (*S)[kTM + kPad], const T* src, int64_t ld, int64_t r0,
                                      int64_t c0, int k0, int kvalid, int mvalid) {
    const int t = threadIdx.x;
    if (kAlongRows) {
        const int kk = t >> 4, m4 = (t & 15) * 4;
        for (int e = 0; e < 4; ++e) {
            const int m = m4 + e;
            S[kk][m] = (k0 + kk < kvalid && m < mvalid) ? src[(r0 + k0 + kk) * ld + c0 + m] : T(0);
        }
    } else {
        const int m = t >> 2, k4 = (t & 3) * 4;
        for (int e = 0; e < 4; ++e) {
            const int kk = k4 + e;
            S[kk][m] = (k0 + kk < kvalid && m < mvalid) ? src[(r0 + m) * ld + c0 + k0 + kk] : T(0);
        }
    }
}

// acc = op(A) op(B) over K = kvalid (<= 64 per call chunk handled by the caller loop)
template <class T, bool kAAlongRows, bool kBAlongRows>
__device__ void tile_gemm(TileAcc<T>& acc, T (*As)[kTM + kPad], T (*Bs)[kTN + kPad], const T* A,
                          int64_t lda, int64_t ar0, int64_t ac0, int amv, const T* B, int64_t ldb,
                          int64_t br0, int64_t bc0, int bmv, int kvalid) {
    for (int k0 = 0; k0 < kvalid; k0 += kTK) {
        stage<T, kAAlongRows>(As, A, lda, ar0, ac0, k0, kvalid, amv);
        stage<T, kBAlongRows>(Bs, B, ldb, br0, bc0, k0, kvalid, bmv);
        __syncthreads();
        acc.step(As, Bs);
        __syncthreads();
    }
}

// in-LDS inverse of a lower-triangular tile (n <= 64): one thread per column
template <class T>
__device__ void tri_inverse_lds(T (*L)[kTM + kPad], T (*X)[kTM + kPad], int n) {
    const int c = threadIdx.x;
    if (c < 64) {
        for (int r = 0; r < 64; ++r) X[r][c] = T(0);
        if (c < n) {
            for (int r = c; r < n; ++r) {
                T acc = (r == c) ? T(1) : T(0);
                for (int k = c; k < r; ++k) acc -= L[r][k] * X[k][c];
                X[r][c] = acc / L[r][r];
            }
        }
    }
    __syncthreads();
}

template <class T>
__global__ void __launch_bounds__(kFT) k_factor_inverse(const int64_t* __restrict__ f_off,
                                                       const int64_t* __restrict__ qv,
                                                       const int64_t* __restrict__ ub_off,
                                                       T* __restrict__ Aall, T* __restrict__ Mall,
                                                       T* __restrict__ Dall, int32_t* __restrict__ shifts,
                                                       int32_t* __restrict__ fail) {
    __shared__ T Ld[kTM][kTM + kPad];
    __shared__ T Xd[kTM][kTM + kPad];
    __shared__ T As[kTK][kTM + kPad];
    __shared__ T Bs[kTK][kTN + kPad];
    __shared__ int bad;
    const int i = blockIdx.x;
    const int64_t q = qv[i];
    if (q == 0) return;
    T* A = Aall + f_off[i];   // original block, later X = L^{-1}
    T* W = Mall + f_off[i];   // factor workspace, later the inverse
    T* D = Dall + ub_off[i];
    const int tid = threadIdx.x;
    const int nt = (int)((q + kTM - 1) / kTM);
    for (int64_t r = tid; r < q; r += kFT) {
        T a = A[r * q + r];
        D[r] = (a > T(0) && isfinite(a)) ? T(1) / sqrt(a) : T(1);
    }
    __syncthreads();
    double eps = 0.0;
    int tries = 0;
    for (;;) {
        // W <- D A D + eps I
        for (int64_t e = tid; e < q * q; e += kFT) {
            int64_t r = e / q, c = e % q;
            W[e] = D[r] * A[e] * D[c] + ((r == c) ? T(eps) : T(0));
        }
        if (tid == 0) bad = 0;
        __syncthreads();
        // ---- 1. blocked Cholesky
        for (int kt = 0; kt < nt && !bad; ++kt) {
            const int64_t k0 = (int64_t)kt * kTM;
            const int kb = (int)((q - k0) < kTM ? (q - k0) : kTM);
            for (int e = tid; e < kTM * kTM; e += kFT) {
                int r = e / kTM, c = e % kTM;
                Ld[r][c] = (r < kb && c < kb) ? W[(k0 + r) * q + k0 + c] : T(0);
            }
            __syncthreads();
            for (int c = 0; c < kb; ++c) {
                T piv = Ld[c][c];
                if (!(piv > T(0)) || !isfinite(piv)) {
                    if (tid == 0) bad = 1;
                    __syncthreads();
                    break;
                }
                T lc = sqrt(piv);
                __syncthreads();
                if (tid == 0) Ld[c][c] = lc;
                for (int r = c + 1 + tid; r < kb; r += kFT) Ld[r][c] /= lc;
                __syncthreads();
                for (int e = tid; e < kTM * kTM; e += kFT) {
                    int r = e / kTM, s = e % kTM;
                    if (s > c && s <= r && r < kb) Ld[r][s] -= Ld[r][c] * Ld[s][c];
                }
                __syncthreads();
            }
            if (bad) break;
            for (int e = tid; e < kTM * kTM; e += kFT) {
                int r = e / kTM, c = e % kTM;
                if (r < kb && c <= r) W[(k0 + r) * q + k0 + c] = Ld[r][c];
            }
            tri_inverse_lds<T>(Ld, Xd, kb);
            // panel: P_it = A_it L_kk^{-T}, for every tile row below
            for (int it = kt + 1; it < nt; ++it) {
                const int64_t i0 = (int64_t)it * kTM;
                const int ib = (int)((q - i0) < kTM ? (q - i0) : kTM);
                TileAcc<T> acc;
                acc.zero();
                // B[k][n] = Xd[n][k]  (LDS source: stage from LDS by hand)
                for (int s0 = 0; s0 < kb; s0 += kTK) {
                    stage<T, false>(As, W, q, i0, k0, s0, kb, ib);
                    {
                        const int n = tid >> 2, k4 = (tid & 3) * 4;
                        for (int e2 = 0; e2 < 4; ++e2) {
                            const int kk = k4 + e2;
                            Bs[kk][n] = (s0 + kk < kb && n < kb) ? Xd[n][s0 + kk] : T(0);
                        }
                    }
                    __syncthreads();
                    acc.step(As, Bs);
                    __syncthreads();
                }
                acc.each([&](int r, int c, T v) {
                    if (r < ib && c < kb) W[(i0 + r) * q + k0 + c] = v;
                });
                __syncthreads();
            }
            // trailing update W_ij -= P_i P_j^T for kt < jt <= it
            for (int it = kt + 1; it < nt; ++it) {
                const int64_t i0 = (int64_t)it * kTM;
                const int ib = (int)((q - i0) < kTM ? (q - i0) : kTM);
                for (int jt = kt + 1; jt <= it; ++jt) {
                    const int64_t j0 = (int64_t)jt * kTM;
                    const int jb = (int)((q - j0) < kTM ? (q - j0) : kTM);
                    TileAcc<T> acc;
                    acc.zero();
                    tile_gemm<T, false, false>(acc, As, Bs, W, q, i0, k0, ib, W, q, j0, k0, jb, kb);
                    acc.each([&](int r, int c, T v) {
                        if (r < ib && c < jb) W[(i0 + r) * q + j0 + c] -= v;
                    });
                    __syncthreads();
                }
            }
        }
        __syncthreads();
        if (!bad) break;
        ++tries;
        if (tries > 12) {
            if (tid == 0) atomicAdd(fail, 1);
            return;
        }
        eps = (eps == 0.0) ? 10.0 * Unit<T>::u * (double)q : eps * 10.0;
    }
    if (tid == 0 && tries > 0) atomicAdd(shifts, 1);
    // ---- 2. X = L^{-1} into A (lower tiles)
    for (int kt = 0; kt < nt; ++kt) {
        const int64_t k0 = (int64_t)kt * kTM;
        const int kb = (int)((q - k0) < kTM ? (q - k0) : kTM);
        for (int e = tid; e < kTM * kTM; e += kFT) {
            int r = e / kTM, c = e % kTM;
            Ld[r][c] = (r < kb && c <= r) ? W[(k0 + r) * q + k0 + c] : T(0);
        }
        __syncthreads();
        tri_inverse_lds<T>(Ld, Xd, kb);
        for (int e = tid; e < kTM * kTM; e += kFT) {
            int r = e / kTM, c = e % kTM;
            if (r < kb && c < kb) A[(k0 + r) * q + k0 + c] = Xd[r][c];
        }
        __syncthreads();
    }
    for (int kt = 0; kt < nt; ++kt) {
        const int64_t k0 = (int64_t)kt * kTM;
        const int kb = (int)((q - k0) < kTM ? (q - k0) : kTM);
        for (int it = kt + 1; it < nt; ++it) {
            const int64_t i0 = (int64_t)it * kTM;
            const int ib = (int)((q - i0) < kTM ? (q - i0) : kTM);
            // S = sum_{jt=kt}^{it-1} L_{it,jt} X_{jt,kt}
            TileAcc<T> acc;
            acc.zero();
            const int kspan = (int)(i0 - k0);  // columns k0 .. i0-1 of L's row block it
            tile_gemm<T, false, true>(acc, As, Bs, W, q, i0, k0, ib, A, q, k0, k0, kb, kspan);
            acc.each([&](int r, int c, T v) {
                if (r < ib && c < kb) A[(i0 + r) * q + k0 + c] = v;
            });
            __syncthreads();
            // X_{it,kt} = -X_{it,it} S
            TileAcc<T> acc2;
            acc2.zero();
            tile_gemm<T, false, true>(acc2, As, Bs, A, q, i0, i0, ib, A, q, i0, k0, kb, ib);
            acc2.each([&](int r, int c, T v) {
                if (r < ib && c < kb) A[(i0 + r) * q + k0 + c] = -v;
            });
            __syncthreads();
        }
    }
    // ---- 3. W = D X^T X D (lower tiles computed, mirrored)
    for (int at = 0; at < nt; ++at) {
        const int64_t a0 = (int64_t)at * kTM;
        const int ab = (int)((q - a0) < kTM ? (q - a0) : kTM);
        for (int bt = 0; bt <= at; ++bt) {
            const int64_t b0 = (int64_t)bt * kTM;
            const int bb = (int)((q - b0) < kTM ? (q - b0) : kTM);
            TileAcc<T> acc;
            acc.zero();
            // sum over rows t >= a0 of X[t][a0+m] X[t][b0+n]
            tile_gemm<T, true, true>(acc, As, Bs, A, q, a0, a0, ab, A, q, a0, b0, bb, (int)(q - a0));
            acc.each([&](int r, int c, T v) {
                if (r < ab && c < bb) {
                    const int64_t gr = a0 + r, gc = b0 + c;
                    if (gc <= gr) {
                        T s = D[gr] * v * D[gc];
                        W[gr * q + gc] = s;
                        W[gc * q + gr] = s;
                    }
                }
            });
            __syncthreads();
        }
    }
}

}  // namespace

template <class T>
int factor_inverse(Handle& h, T* A, T* M, T* D, int32_t* flags) {
    KTimer kt_(h.stream, "k_factor_inverse");
    hipLaunchKernelGGL((k_factor_inverse<T>), dim3(h.geo.J), dim3(kFT), 0, h.stream, h.d_f_off, h.d_q,
                       h.d_ub_off, A, M, D, flags, flags + 1);
    kt_.stop();
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

template int factor_inverse<double>(Handle&, double*, double*, double*, int32_t*);
template int factor_inverse<float>(Handle&, float*, float*, float*, int32_t*);

}  // namespace rdd
