// 64x64 output tiles on CDNA matrix cores (v_mfma_*_16x16x4, wave64).
//
// A workgroup of 256 threads (4 waves in a 2x2 grid) owns a 64x64 output tile;
// each wave computes a 32x32 quarter as 2x2 blocks of 16x16.  Operands are
// staged k-major in LDS: As[k][m] (the A operand, m = output row) and
// Bs[k][n] (the B operand, n = output column), BK = 16 k-steps per stage.
// Lane layout of the 16x16x4 instructions: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; accumulator element i of lane l is D[row][l % 16] with
// row = l / 16 + 4 i for the FP64 instruction and row = 4 (l / 16) + i for the
// FP32 one (checked on gfx950 by an in-bounds probe).
#pragma once

#include <hip/hip_runtime.h>

namespace rdd {

template <class T>
struct Mfma;

template <>
struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int lane, int i) { return (lane >> 4) + 4 * i; }
};

template <>
struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int out_row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

constexpr int kTM = 64, kTN = 64, kTK = 16, kPad = 1;

template <class T>
struct TileAcc {
    typename Mfma<T>::acc_t c[2][2];
    __device__ __forceinline__ void zero() {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int i = 0; i < 4; ++i) c[a][b][i] = T(0);
    }
    // one BK stage from LDS
    __device__ __forceinline__ void step(const T (*As)[kTM + kPad], const T (*Bs)[kTN + kPad]) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int wm = wave >> 1, wn = wave & 1;
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < kTK; kk += 4) {
            T a0 = As[kk + lk][wm * 32 + lr];
            T a1 = As[kk + lk][wm * 32 + 16 + lr];
            T b0 = Bs[kk + lk][wn * 32 + lr];
            T b1 = Bs[kk + lk][wn * 32 + 16 + lr];
            c[0][0] = Mfma<T>::mma(a0, b0, c[0][0]);
            c[0][1] = Mfma<T>::mma(a0, b1, c[0][1]);
            c[1][0] = Mfma<T>::mma(a1, b0, c[1][0]);
            c[1][1] = Mfma<T>::mma(a1, b1, c[1][1]);
        }
    }
    // KS k-steps from LDS (As, Bs hold KS rows)
    template <int KS>
    __device__ __forceinline__ void step_k(const T (*As)[kTM + kPad], const T (*Bs)[kTN + kPad]) {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int wm = wave >> 1, wn = wave & 1;
        const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < KS; kk += 4) {
            T a0 = As[kk + lk][wm * 32 + lr];
            T a1 = As[kk + lk][wm * 32 + 16 + lr];
            T b0 = Bs[kk + lk][wn * 32 + lr];
            T b1 = Bs[kk + lk][wn * 32 + 16 + lr];
            c[0][0] = Mfma<T>::mma(a0, b0, c[0][0]);
            c[0][1] = Mfma<T>::mma(a0, b1, c[0][1]);
            c[1][0] = Mfma<T>::mma(a1, b0, c[1][0]);
            c[1][1] = Mfma<T>::mma(a1, b1, c[1][1]);
        }
    }
    // visit every accumulator element with its tile-local (row, col)
    template <class F>
    __device__ __forceinline__ void each(F f) const {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const int wm = wave >> 1, wn = wave & 1;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int i = 0; i < 4; ++i) {
                    int r = wm * 32 + a * 16 + Mfma<T>::out_row(lane, i);
                    int cc = wn * 32 + b * 16 + (lane & 15);
                    f(r, cc, c[a][b][i]);
                }
    }
};

constexpr int kBK = 32;  // k-steps per LDS stage of the tile products

// One kBK slice of a 64-wide operand, 8 elements per thread, held in
// registers between its global load and its LDS store (so the next slice is
// in flight while the current one is multiplied):
//  kAlongRows: element (kk, m) = src[(r0 + k0 + kk) * ld + c0 + m]
//  otherwise : element (kk, m) = src[(r0 + m) * ld + c0 + k0 + kk]
template <class T, bool kAlongRows>
__device__ __forceinline__ void fetch(T* reg, const T* src, int64_t ld, int64_t r0, int64_t c0, int k0,
                                      int kvalid, int mvalid) {
    const int t = threadIdx.x;
    if (kAlongRows) {
        const int m4 = (t & 15) * 4;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int kk = (t >> 4) + 16 * j;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m4 + e;
                reg[4 * j + e] = (k0 + kk < kvalid && m < mvalid) ? src[(r0 + k0 + kk) * ld + c0 + m] : T(0);
            }
        }
    } else {
        const int m = t >> 2, k8 = (t & 3) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int kk = k8 + e;
            reg[e] = (k0 + kk < kvalid && m < mvalid) ? src[(r0 + m) * ld + c0 + k0 + kk] : T(0);
        }
    }
}

template <class T, bool kAlongRows>
__device__ __forceinline__ void put(T (*S)[kTM + kPad], const T* reg) {
    const int t = threadIdx.x;
    if (kAlongRows) {
        const int m4 = (t & 15) * 4;
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) S[(t >> 4) + 16 * j][m4 + e] = reg[4 * j + e];
    } else {
        const int m = t >> 2, k8 = (t & 3) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) S[k8 + e][m] = reg[e];
    }
}

// acc += op(A) op(B) over K = kvalid, kBK k-steps per LDS stage (As, Bs hold
// kBK rows); the next stage is loaded while the current one is multiplied
template <class T, bool kAAlongRows, bool kBAlongRows>
__device__ void tile_gemm(TileAcc<T>& acc, T (*As)[kTM + kPad], T (*Bs)[kTN + kPad], const T* A,
                          int64_t lda, int64_t ar0, int64_t ac0, int amv, const T* B, int64_t ldb,
                          int64_t br0, int64_t bc0, int bmv, int kvalid) {
    T ra[8], rb[8];
    if (kvalid > 0) {
        fetch<T, kAAlongRows>(ra, A, lda, ar0, ac0, 0, kvalid, amv);
        fetch<T, kBAlongRows>(rb, B, ldb, br0, bc0, 0, kvalid, bmv);
    }
    for (int k0 = 0; k0 < kvalid; k0 += kBK) {
        put<T, kAAlongRows>(As, ra);
        put<T, kBAlongRows>(Bs, rb);
        __syncthreads();
        if (k0 + kBK < kvalid) {
            fetch<T, kAAlongRows>(ra, A, lda, ar0, ac0, k0 + kBK, kvalid, amv);
            fetch<T, kBAlongRows>(rb, B, ldb, br0, bc0, k0 + kBK, kvalid, bmv);
        }
        acc.template step_k<kBK>(As, Bs);
        __syncthreads();
    }
}

// value of v in lane l (l uniform), through the scalar unit
__device__ __forceinline__ double read_lane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

}  // namespace rdd
