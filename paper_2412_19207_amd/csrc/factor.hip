// Local inverses of the Schwarz blocks on matrix cores (paper Sec. 3: the
// local inverse A_i^{-1} of A_i = R_i H^T H R_i^T).
//
// With D = diag(A)^{-1/2} and the Cholesky factorisation D A D + eps I = L L^T,
//     A^{-1} = Y^T Y,   Y = L^{-1} D.
// The FP64 path stores W = Y^T Y itself as packed lower 64x64 tiles (read once
// per application); the mixed path stores Y in FP32 (Y^T Y stays positive
// semi-definite whatever the rounding of Y, so the FP32 operator is still a
// valid CG preconditioner, which a rounded W would not be).
//
// All blocks are factorised together, one tile per workgroup, in launches
// that follow the data dependences of the blocked algorithms:
//   Cholesky, for each panel step s:  diag(s)  : L_ss = chol(W_ss), L_ss^{-1}
//                                     panel(s) : L_as = W_as L_ss^{-T}
//                                     trail(s) : W_ab -= L_as L_bs^T (s < b <= a)
//   X = L^{-1}, by tile distance t:    X_ab = -L_aa^{-1} sum_{c=b}^{a-1} L_ac X_cb
//   Y = X D rounded to FP32 (mixed) or W = D X^T X D on matrix cores (FP64).
// A pivot that is not positive restarts that block with a diagonal shift
// eps = 10 u q, growing tenfold (the count is reported as `shifts`).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace rdd {

namespace {

constexpr int kFT = 256;  // threads

struct TileTask {
    int32_t blk, a, b, pad;
};

__device__ __forceinline__ int tile_dim(int64_t q, int t) {
    const int64_t r = q - (int64_t)t * kTM;
    return (int)(r < kTM ? r : kTM);
}

// D = diag(A)^{-1/2} (1 where the diagonal is not positive)
__global__ void k_equil(const int64_t* __restrict__ f_off, const int64_t* __restrict__ qv,
                        const int64_t* __restrict__ ub_off, const double* __restrict__ A,
                        double* __restrict__ D) {
    const int i = blockIdx.x;
    const int64_t q = qv[i];
    const double* Ai = A + f_off[i];
    for (int64_t r = threadIdx.x; r < q; r += blockDim.x) {
        const double a = Ai[r * q + r];
        D[ub_off[i] + r] = (a > 0.0 && isfinite(a)) ? 1.0 / sqrt(a) : 1.0;
    }
}

// W = D A D + eps_i I for the listed blocks (grid.y = list index)
__global__ void k_scale_shift(const int32_t* __restrict__ blks, const int64_t* __restrict__ f_off,
                              const int64_t* __restrict__ qv, const int64_t* __restrict__ ub_off,
                              const double* __restrict__ eps, const double* __restrict__ A,
                              const double* __restrict__ D, double* __restrict__ W,
                              int32_t* __restrict__ bad) {
    const int i = blks[blockIdx.y];
    const int64_t q = qv[i];
    const double* Ai = A + f_off[i];
    double* Wi = W + f_off[i];
    const double* Di = D + ub_off[i];
    const double e = eps[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) bad[i] = 0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < q * q;
         x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = x / q, c = x % q;
        Wi[x] = Di[r] * Ai[x] * Di[c] + (r == c ? e : 0.0);
    }
}

// L_ss = chol(W_ss) (written to W) and X_ss = L_ss^{-1} (written to Xd) for
// one diagonal tile, in one wave, in registers: lane r keeps row r of the
// tile.  Cholesky (right-looking): at column c the pivot and the scaled
// column entries are read from their lanes and every lane updates its row.
// Inverse (forward substitution on the identity, row-wise): at step c lane c
// scales its row of X by 1 / L_cc and every lane r > c subtracts L_rc times
// that row.  Beyond the block edge the tile is the identity during the
// factorisation and zero in the outputs.
__global__ void __launch_bounds__(64) k_chol_diag(const TileTask* __restrict__ tasks,
                                                  const int64_t* __restrict__ f_off,
                                                  const int64_t* __restrict__ qv,
                                                  const int64_t* __restrict__ xd_off,
                                                  double* __restrict__ Wall,
                                                  double* __restrict__ Xd,
                                                  int32_t* __restrict__ bad) {
    const TileTask tk = tasks[blockIdx.x];
    const int i = tk.blk, s = tk.a;
    if (bad[i]) return;
    const int64_t q = qv[i];
    double* W = Wall + f_off[i];
    const int64_t s0 = (int64_t)s * kTM;
    const int kb = tile_dim(q, s);
    const int r = threadIdx.x;
    double a[kTM];
#pragma unroll
    for (int c = 0; c < kTM; ++c)
        a[c] = (r < kb && c < kb) ? W[(s0 + r) * q + s0 + c] : (r == c ? 1.0 : 0.0);
    bool ok = true;
#pragma unroll
    for (int c = 0; c < kTM; ++c) {
        const double piv = read_lane(a[c], c);
        if (!(piv > 0.0) || !isfinite(piv)) {
            ok = false;  // uniform: every lane read the same pivot
            break;
        }
        const double lc = sqrt(piv);
        const double l = (r == c) ? lc : (r > c ? a[c] / lc : 0.0);
        a[c] = l;
#pragma unroll
        for (int t = c + 1; t < kTM; ++t) a[t] = fma(-l, read_lane(l, t), a[t]);
    }
    if (!ok) {
        if (r == 0) bad[i] = 1;
        return;
    }
#pragma unroll
    for (int c = 0; c < kTM; ++c)
        if (r < kb && c <= r) W[(s0 + r) * q + s0 + c] = a[c];
    double x[kTM];
#pragma unroll
    for (int t = 0; t < kTM; ++t) x[t] = (t == r) ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < kTM; ++c) {
        const double inv = 1.0 / read_lane(a[c], c);
#pragma unroll
        for (int t = 0; t <= c; ++t) x[t] = (r == c) ? x[t] * inv : x[t];
        const double lrc = (r > c) ? a[c] : 0.0;
#pragma unroll
        for (int t = 0; t <= c; ++t) x[t] = fma(-lrc, read_lane(x[t], c), x[t]);
    }
    double* X = Xd + xd_off[i] + (int64_t)s * kTM * kTM;
#pragma unroll
    for (int t = 0; t < kTM; ++t) X[r * kTM + t] = (r < kb && t < kb) ? x[t] : 0.0;
}

// L_as = W_as X_ss^T  (a > s)
__global__ void __launch_bounds__(kFT) k_chol_panel(const TileTask* __restrict__ tasks,
                                                    const int64_t* __restrict__ f_off,
                                                    const int64_t* __restrict__ qv,
                                                    const int64_t* __restrict__ xd_off,
                                                    double* __restrict__ Wall,
                                                    const double* __restrict__ Xd,
                                                    const int32_t* __restrict__ bad) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const TileTask tk = tasks[blockIdx.x];
    const int i = tk.blk, a = tk.a, s = tk.b;
    if (bad[i]) return;
    const int64_t q = qv[i];
    double* W = Wall + f_off[i];
    const int64_t a0 = (int64_t)a * kTM, s0 = (int64_t)s * kTM;
    const int ab = tile_dim(q, a), kb = tile_dim(q, s);
    const double* X = Xd + xd_off[i] + (int64_t)s * kTM * kTM;
    TileAcc<double> acc;
    acc.zero();
    tile_gemm<double, false, false>(acc, As, Bs, W, q, a0, s0, ab, X, kTM, 0, 0, kb, kb);
    acc.each([&](int r, int c, double v) {
        if (r < ab && c < kb) W[(a0 + r) * q + s0 + c] = v;
    });
}

// W_ab -= L_as L_bs^T  (s < b <= a)
__global__ void __launch_bounds__(kFT) k_chol_trail(const TileTask* __restrict__ tasks, int s,
                                                    const int64_t* __restrict__ f_off,
                                                    const int64_t* __restrict__ qv,
                                                    double* __restrict__ Wall,
                                                    const int32_t* __restrict__ bad) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const TileTask tk = tasks[blockIdx.x];
    const int i = tk.blk, a = tk.a, b = tk.b;
    if (bad[i]) return;
    const int64_t q = qv[i];
    double* W = Wall + f_off[i];
    const int64_t a0 = (int64_t)a * kTM, b0 = (int64_t)b * kTM, s0 = (int64_t)s * kTM;
    const int ab = tile_dim(q, a), bb = tile_dim(q, b), kb = tile_dim(q, s);
    TileAcc<double> acc;
    acc.zero();
    tile_gemm<double, false, false>(acc, As, Bs, W, q, a0, s0, ab, W, q, b0, s0, bb, kb);
    acc.each([&](int r, int c, double v) {
        if (r < ab && c < bb) W[(a0 + r) * q + b0 + c] -= v;
    });
}

// X_aa = Xd[a] (full tile, zeros above the diagonal) into the X storage
__global__ void k_place_diag(const TileTask* __restrict__ tasks, const int64_t* __restrict__ f_off,
                             const int64_t* __restrict__ qv, const int64_t* __restrict__ xd_off,
                             const double* __restrict__ Xd, double* __restrict__ Xall) {
    const TileTask tk = tasks[blockIdx.x];
    const int i = tk.blk, a = tk.a;
    const int64_t q = qv[i];
    const int64_t a0 = (int64_t)a * kTM;
    const int ab = tile_dim(q, a);
    const double* src = Xd + xd_off[i] + (int64_t)a * kTM * kTM;
    double* X = Xall + f_off[i];
    for (int e = threadIdx.x; e < kTM * kTM; e += blockDim.x) {
        const int r = e / kTM, c = e % kTM;
        if (r < ab && c < ab) X[(a0 + r) * q + a0 + c] = src[e];
    }
}

// X_ab = -X_aa sum_{c=b}^{a-1} L_ac X_cb  (a > b; X_cb known for c < a)
__global__ void __launch_bounds__(kFT) k_inv_off(const TileTask* __restrict__ tasks,
                                                 const int64_t* __restrict__ f_off,
                                                 const int64_t* __restrict__ qv,
                                                 const double* __restrict__ Lall,
                                                 double* __restrict__ Xall) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const TileTask tk = tasks[blockIdx.x];
    const int i = tk.blk, a = tk.a, b = tk.b;
    const int64_t q = qv[i];
    const double* L = Lall + f_off[i];
    double* X = Xall + f_off[i];
    const int64_t a0 = (int64_t)a * kTM, b0 = (int64_t)b * kTM;
    const int ab = tile_dim(q, a), bb = tile_dim(q, b);
    TileAcc<double> acc;
    acc.zero();
    tile_gemm<double, false, true>(acc, As, Bs, L, q, a0, b0, ab, X, q, b0, b0, bb, (int)(a0 - b0));
    acc.each([&](int r, int c, double v) {
        if (r < ab && c < bb) X[(a0 + r) * q + b0 + c] = v;
    });
    __syncthreads();
    TileAcc<double> acc2;
    acc2.zero();
    tile_gemm<double, false, true>(acc2, As, Bs, X, q, a0, a0, ab, X, q, a0, b0, bb, ab);
    acc2.each([&](int r, int c, double v) {
        if (r < ab && c < bb) X[(a0 + r) * q + b0 + c] = -v;
    });
}

// packed tile (a, b) of Y = X D, zero-padded to 64 x 64
template <class T>
__global__ void k_make_Y(const TileTask* __restrict__ tasks, const int64_t* __restrict__ f_off,
                         const int64_t* __restrict__ qv, const int64_t* __restrict__ ub_off,
                         const int64_t* __restrict__ t_off, const double* __restrict__ Xall,
                         const double* __restrict__ Dall, T* __restrict__ Y) {
    const TileTask tk = tasks[blockIdx.x];
    const int i = tk.blk, a = tk.a, b = tk.b;
    const int64_t q = qv[i];
    const int64_t a0 = (int64_t)a * kTM, b0 = (int64_t)b * kTM;
    const int ab = tile_dim(q, a), bb = tile_dim(q, b);
    const double* X = Xall + f_off[i];
    const double* D = Dall + ub_off[i];
    T* out = Y + t_off[i] + ((int64_t)a * (a + 1) / 2 + b) * kTM * kTM;
    for (int e = threadIdx.x; e < kTM * kTM; e += blockDim.x) {
        const int r = e / kTM, c = e % kTM;
        double v = 0.0;
        if (r < ab && c < bb && (a > b || c <= r)) v = X[(a0 + r) * q + b0 + c] * D[b0 + c];
        out[e] = (T)v;
    }
}


// packed tile (a, b), b <= a, of W = A^{-1} = D X^T X D: sum over the rows t >= a0
// of X[t][a0 + r] X[t][b0 + c] (X is lower triangular), scaled by D on both
// sides, in FP64; a diagonal tile is written whole and exactly symmetric, as T
template <class T>
__global__ void __launch_bounds__(kFT) k_make_W(const TileTask* __restrict__ tasks,
                                                const int64_t* __restrict__ f_off,
                                                const int64_t* __restrict__ qv,
                                                const int64_t* __restrict__ ub_off,
                                                const int64_t* __restrict__ t_off,
                                                const double* __restrict__ Xall,
                                                const double* __restrict__ Dall,
                                                T* __restrict__ Wt) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    __shared__ double Cs[kTM][kTM + kPad];
    const TileTask tk = tasks[blockIdx.x];
    const int i = tk.blk, a = tk.a, b = tk.b;
    const int64_t q = qv[i];
    const int64_t a0 = (int64_t)a * kTM, b0 = (int64_t)b * kTM;
    const int ab = tile_dim(q, a), bb = tile_dim(q, b);
    const double* X = Xall + f_off[i];
    const double* D = Dall + ub_off[i];
    T* out = Wt + t_off[i] + ((int64_t)a * (a + 1) / 2 + b) * kTM * kTM;
    TileAcc<double> acc;
    acc.zero();
    tile_gemm<double, true, true>(acc, As, Bs, X, q, a0, a0, ab, X, q, a0, b0, bb, (int)(q - a0));
    acc.each([&](int r, int c, double v) {
        Cs[r][c] = (r < ab && c < bb) ? D[a0 + r] * v * D[b0 + c] : 0.0;
    });
    __syncthreads();
    for (int e = threadIdx.x; e < kTM * kTM; e += kFT) {
        const int r = e / kTM, c = e % kTM;
        out[e] = (T)((a == b && c > r) ? Cs[c][r] : Cs[r][c]);
    }
}

}  // namespace

// Tile counts and packed offsets of every block (host tables and device copy).
int plan_tiles(Handle& h) {
    const int J = h.geo.J;
    h.nt.assign(J, 0);
    h.t_off.assign(J + 1, 0);
    for (int i = 0; i < J; ++i) {
        const int64_t nt = (h.q[i] + kTM - 1) / kTM;
        h.nt[i] = (int32_t)nt;
        h.t_off[i + 1] = h.t_off[i] + nt * (nt + 1) / 2 * kTM * kTM;
    }
    h.tile_elems = h.t_off[J];
    RDD_TRY(dev_alloc(h, &h.d_t_off, (size_t)J + 1));
    RDD_TRY(upload(h, h.d_t_off, h.t_off.data(), sizeof(int64_t) * (J + 1)));
    return RANN_OK;
}

namespace {

struct Launch {
    int64_t off, cnt;
};

int upload_tasks(Handle& h, const std::vector<TileTask>& v, TileTask** d) {
    RDD_TRY(dev_alloc(h, d, v.size()));
    if (!v.empty())
        RDD_TRY(upload(h, *d, v.data(), sizeof(TileTask) * v.size()));
    return RANN_OK;
}

}  // namespace

// A (q x q per block, FP64, row-major) -> packed tiles of Y = L^{-1} D into
// h.d_M64 or h.d_M32.  A is left unchanged until the factorisations succeed
// and is then overwritten with X = L^{-1}.  Synchronous.
int factor_tiles(Handle& h, double* A, double* W) {
    const int J = h.geo.J;
    KTimer kt_(h.stream, "k_factor");
    int ntmax = 0;
    for (int i = 0; i < J; ++i) ntmax = std::max(ntmax, h.nt[i]);
    std::vector<int64_t> xd_off(J + 1, 0);
    for (int i = 0; i < J; ++i) xd_off[i + 1] = xd_off[i] + (int64_t)h.nt[i] * kTM * kTM;
    double *d_D = nullptr, *d_Xd = nullptr, *d_eps = nullptr;
    int64_t* d_xd_off = nullptr;
    int32_t *d_bad = nullptr, *d_blks = nullptr;
    RDD_TRY(dev_alloc(h, &d_D, (size_t)h.ub_total));
    RDD_TRY(dev_alloc(h, &d_Xd, (size_t)xd_off[J]));
    RDD_TRY(dev_alloc(h, &d_eps, (size_t)J));
    RDD_TRY(dev_alloc(h, &d_xd_off, (size_t)J + 1));
    RDD_TRY(dev_alloc(h, &d_bad, (size_t)J));
    RDD_TRY(dev_alloc(h, &d_blks, (size_t)J));
    RDD_TRY(upload(h, d_xd_off, xd_off.data(), sizeof(int64_t) * (J + 1)));
    hipLaunchKernelGGL(k_equil, dim3(J), dim3(256), 0, h.stream, h.d_f_off, h.d_q, h.d_ub_off, A, d_D);
    RDD_HIP(hipGetLastError());

    std::vector<double> eps(J, 0.0);
    std::vector<int32_t> active;
    for (int i = 0; i < J; ++i)
        if (h.q[i] > 0) active.push_back(i);
    std::vector<int32_t> bad(J, 0);
    h.shifts = 0;
    std::vector<TileTask*> task_bufs;
    int tries = 0;
    while (!active.empty()) {
        // task lists of the Cholesky launches for the active blocks
        std::vector<TileTask> tasks;
        std::vector<Launch> diag(ntmax), panel(ntmax), trail(ntmax);
        for (int s = 0; s < ntmax; ++s) {
            diag[s].off = (int64_t)tasks.size();
            for (int i : active)
                if (h.nt[i] > s) tasks.push_back({i, s, s, 0});
            diag[s].cnt = (int64_t)tasks.size() - diag[s].off;
            panel[s].off = (int64_t)tasks.size();
            for (int i : active)
                for (int a = s + 1; a < h.nt[i]; ++a) tasks.push_back({i, a, s, 0});
            panel[s].cnt = (int64_t)tasks.size() - panel[s].off;
            trail[s].off = (int64_t)tasks.size();
            for (int i : active)
                for (int a = s + 1; a < h.nt[i]; ++a)
                    for (int b = s + 1; b <= a; ++b) tasks.push_back({i, a, b, 0});
            trail[s].cnt = (int64_t)tasks.size() - trail[s].off;
        }
        TileTask* d_tasks = nullptr;
        RDD_TRY(upload_tasks(h, tasks, &d_tasks));
        task_bufs.push_back(d_tasks);
        RDD_TRY(upload(h, d_eps, eps.data(), sizeof(double) * J));
        RDD_TRY(upload(h, d_blks, active.data(), sizeof(int32_t) * active.size()));
        hipLaunchKernelGGL(k_scale_shift, dim3(64, (unsigned)active.size()), dim3(256), 0, h.stream,
                           d_blks, h.d_f_off, h.d_q, h.d_ub_off, d_eps, A, d_D, W, d_bad);
        RDD_HIP(hipGetLastError());
        for (int s = 0; s < ntmax; ++s) {
            if (diag[s].cnt)
                hipLaunchKernelGGL(k_chol_diag, dim3((unsigned)diag[s].cnt), dim3(64), 0, h.stream,
                                   d_tasks + diag[s].off, h.d_f_off, h.d_q, d_xd_off, W, d_Xd, d_bad);
            if (panel[s].cnt)
                hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)panel[s].cnt), dim3(kFT), 0, h.stream,
                                   d_tasks + panel[s].off, h.d_f_off, h.d_q, d_xd_off, W, d_Xd, d_bad);
            if (trail[s].cnt)
                hipLaunchKernelGGL(k_chol_trail, dim3((unsigned)trail[s].cnt), dim3(kFT), 0, h.stream,
                                   d_tasks + trail[s].off, s, h.d_f_off, h.d_q, W, d_bad);
            RDD_HIP(hipGetLastError());
        }
        RDD_TRY(download(h, bad.data(), d_bad, sizeof(int32_t) * J));
        RDD_HIP(hipStreamSynchronize(h.stream));
        std::vector<int32_t> again;
        for (int i : active)
            if (bad[i]) again.push_back(i);
        if (again.empty()) break;
        if (++tries > 12) {
            set_error("a local Schwarz block is not positive definite even after diagonal shifts");
            return RANN_EBREAKDOWN;
        }
        for (int i : again) {
            if (eps[i] == 0.0) ++h.shifts;
            eps[i] = (eps[i] == 0.0) ? 10.0 * DBL_EPSILON * (double)h.q[i] : eps[i] * 10.0;
        }
        active.swap(again);
    }
    // X = L^{-1} into A, by tile distance
    {
        std::vector<TileTask> tasks;
        std::vector<Launch> dist(ntmax);
        for (int i = 0; i < J; ++i)
            for (int a = 0; a < h.nt[i]; ++a) tasks.push_back({i, a, a, 0});
        const int64_t ndiag = (int64_t)tasks.size();
        for (int t = 1; t < ntmax; ++t) {
            dist[t].off = (int64_t)tasks.size();
            for (int i = 0; i < J; ++i)
                for (int b = 0; b + t < h.nt[i]; ++b) tasks.push_back({i, b + t, b, 0});
            dist[t].cnt = (int64_t)tasks.size() - dist[t].off;
        }
        TileTask* d_tasks = nullptr;
        RDD_TRY(upload_tasks(h, tasks, &d_tasks));
        task_bufs.push_back(d_tasks);
        if (ndiag)
            hipLaunchKernelGGL(k_place_diag, dim3((unsigned)ndiag), dim3(256), 0, h.stream, d_tasks,
                               h.d_f_off, h.d_q, d_xd_off, d_Xd, A);
        for (int t = 1; t < ntmax; ++t)
            if (dist[t].cnt)
                hipLaunchKernelGGL(k_inv_off, dim3((unsigned)dist[t].cnt), dim3(kFT), 0, h.stream,
                                   d_tasks + dist[t].off, h.d_f_off, h.d_q, W, A);
        RDD_HIP(hipGetLastError());
    }
    // Y = X D (mixed, FP32; with W = Y^T Y in FP32 as well for blocks of at
    // most 6 tiles) or W = Y^T Y (FP64) in packed lower tiles
    {
        std::vector<TileTask> tasks;
        for (int i = 0; i < J; ++i)
            for (int a = 0; a < h.nt[i]; ++a)
                for (int b = 0; b <= a; ++b) tasks.push_back({i, a, b, 0});
        TileTask* d_tasks = nullptr;
        RDD_TRY(upload_tasks(h, tasks, &d_tasks));
        task_bufs.push_back(d_tasks);
        if (!tasks.empty()) {
            if (h.precision == RANN_MIXED) {
                hipLaunchKernelGGL(k_make_Y<float>, dim3((unsigned)tasks.size()), dim3(256), 0,
                                   h.stream, d_tasks, h.d_f_off, h.d_q, h.d_ub_off, h.d_t_off, A,
                                   d_D, h.d_M32);
                if (h.d_W32)
                    hipLaunchKernelGGL(k_make_W<float>, dim3((unsigned)tasks.size()), dim3(kFT), 0, h.stream,
                                       d_tasks, h.d_f_off, h.d_q, h.d_ub_off, h.d_t_off, A, d_D, h.d_W32);
            } else {
                hipLaunchKernelGGL(k_make_W<double>, dim3((unsigned)tasks.size()), dim3(kFT), 0, h.stream,
                                   d_tasks, h.d_f_off, h.d_q, h.d_ub_off, h.d_t_off, A, d_D, h.d_M64);
            }
        }
        RDD_HIP(hipGetLastError());
    }
    RDD_HIP(hipStreamSynchronize(h.stream));
    kt_.stop();
    for (TileTask* p : task_bufs) dev_free(h, p);
    dev_free(h, d_D);
    dev_free(h, d_Xd);
    dev_free(h, d_eps);
    dev_free(h, d_xd_off);
    dev_free(h, d_bad);
    dev_free(h, d_blks);
    return RANN_OK;
}

}  // namespace rdd
