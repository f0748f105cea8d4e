// The iteration: products with H and H^T, Krylov recurrences, true residual,
// adjoint and probe evaluation (paper Sec. 2 normal equations, Sec. 3
// preconditioned CG / GMRES, Sec. 5 stopping rule).
//
// Vectors are FP64, (rows, k) row-major with the right-hand side fastest.
// All reductions are two-stage with a fixed number of workgroups and a fixed
// order, so results are bitwise reproducible (no floating-point atomics).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "cg_step.h"
#include "common.h"

namespace rdd {

namespace {

constexpr int kDotBlocks = 240;
constexpr int kChunkRows = 128;

__global__ void k_HTy_reduce(int64_t P, int k, const int32_t* __restrict__ col_sub,
                             const int64_t* __restrict__ col_off,
                             const int64_t* __restrict__ chunk_off,
                             const int64_t* __restrict__ part_off, const double* __restrict__ part,
                             double* __restrict__ x) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= P * k) return;
    const int64_t g = idx / k;
    const int t = (int)(idx % k);
    const int j = col_sub[g];
    const int64_t c = g - col_off[j];
    double s = 0.0;
    for (int64_t ch = chunk_off[j]; ch < chunk_off[j + 1]; ++ch) s += part[(part_off[ch] + c) * k + t];
    x[idx] = s;
}

// ------------------------------------------------------------------ reductions
// Sum over the 256 / k threads x = ro k + t that share t (k a power of two up to
// 64): a butterfly over the lanes of each wave, then the four waves through
// LDS (sh: 4 k doubles).  The result is returned to threads t < k.
__device__ inline double wave_block_sum(double v, int k, double* sh) {
    for (int off = 32; off >= k; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63;
    if (lane < k) sh[(threadIdx.x >> 6) * k + lane] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x < k) r = (sh[threadIdx.x] + sh[k + threadIdx.x]) + (sh[2 * k + threadIdx.x] + sh[3 * k + threadIdx.x]);
    return r;
}
__device__ inline bool pow2_upto64(int k) { return k <= 64 && (k & (k - 1)) == 0; }

// partial[b * k + t] = sum over this block's rows of a[row, t] * b[row, t]
__global__ void __launch_bounds__(256) k_dot_part(int64_t rows, int k, const double* __restrict__ a,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ partial) {
    __shared__ double s[256];
    const int per = 256 / k;  // rows per step (k <= 256)
    const int t = threadIdx.x % k, ro = threadIdx.x / k;
    double acc = 0.0;
    if (ro < per) {
        for (int64_t r = (int64_t)blockIdx.x * per + ro; r < rows; r += (int64_t)gridDim.x * per)
            acc = fma(a[r * k + t], b[r * k + t], acc);
    }
    if (pow2_upto64(k)) {
        const double tot = wave_block_sum(acc, k, s);
        if (threadIdx.x < k) partial[blockIdx.x * k + threadIdx.x] = tot;
        return;
    }
    s[threadIdx.x] = (ro < per) ? acc : 0.0;
    __syncthreads();
    if (threadIdx.x < k) {
        double tot = 0.0;
        for (int q = 0; q < per; ++q) tot += s[q * k + threadIdx.x];
        partial[blockIdx.x * k + threadIdx.x] = tot;
    }
}

// out[t] = sum over the nb partials; per = 256 / k threads share each t (fixed order)
__global__ void __launch_bounds__(256) k_dot_fin(int k, int nb, const double* __restrict__ partial,
                                                 double* __restrict__ out) {
    __shared__ double s[256];
    const int per = 256 / k;
    const int t = threadIdx.x % k, ro = threadIdx.x / k;
    double acc = 0.0;
    if (ro < per)
        for (int b = ro; b < nb; b += per) acc += partial[b * k + t];
    if (pow2_upto64(k)) {
        const double tot = wave_block_sum(acc, k, s);
        if (threadIdx.x < k) out[threadIdx.x] = tot;
        return;
    }
    s[threadIdx.x] = (ro < per) ? acc : 0.0;
    __syncthreads();
    if (threadIdx.x < k) {
        double tot = 0.0;
        for (int q = 0; q < per; ++q) tot += s[q * k + threadIdx.x];
        out[threadIdx.x] = tot;
    }
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ c) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < n) c[idx] = a[idx] - b[idx];
}

__global__ void k_scale_rows(int64_t row0, int64_t rows, int k, double f, const double* __restrict__ in,
                             double* __restrict__ out) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= rows * k) return;
    out[row0 * k + idx] = f * in[row0 * k + idx];
}

__global__ void k_add(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] += a[i];
}

__global__ void k_copy(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < n) b[idx] = a[idx];
}

__global__ void k_nan_check(int64_t n, const double* __restrict__ a, int32_t* __restrict__ flag) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < n && !isfinite(a[idx])) flag[0] = 1;
}

// ------------------------------------------------------------------ GMRES pieces
// h[i][t] for i < nv: dots of w with V_i (V stored (restart+1) x P x k)
__global__ void __launch_bounds__(256) k_mdot_part(int64_t P, int k, int nv, const double* __restrict__ V,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ partial) {
    // blockIdx.y = basis vector index
    __shared__ double s[256];
    const int i = blockIdx.y;
    const int per = 256 / k;
    const int t = threadIdx.x % k, ro = threadIdx.x / k;
    const double* Vi = V + (int64_t)i * P * k;
    double acc = 0.0;
    if (ro < per)
        for (int64_t r = (int64_t)blockIdx.x * per + ro; r < P; r += (int64_t)gridDim.x * per)
            acc = fma(Vi[r * k + t], w[r * k + t], acc);
    s[threadIdx.x] = (ro < per) ? acc : 0.0;
    __syncthreads();
    if (threadIdx.x < k) {
        double tot = 0.0;
        for (int q = 0; q < per; ++q) tot += s[q * k + threadIdx.x];
        partial[((int64_t)i * gridDim.x + blockIdx.x) * k + threadIdx.x] = tot;
    }
    (void)nv;
}

__global__ void k_mdot_fin(int k, int nv, int nb, const double* __restrict__ partial,
                           double* __restrict__ out) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nv * k) return;
    int i = idx / k, t = idx % k;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[((int64_t)i * nb + b) * k + t];
    out[idx] = s;
}

// w -= sum_i h[i][t] V_i
__global__ void k_mgs_update(int64_t P, int k, int nv, const double* __restrict__ V,
                             const double* __restrict__ h, double* __restrict__ w) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= P * k) return;
    const int t = (int)(idx % k);
    double acc = w[idx];
    for (int i = 0; i < nv; ++i) acc -= h[i * k + t] * V[(int64_t)i * P * k + idx];
    w[idx] = acc;
}

// v_{j+1} = w / ||w||
__global__ void k_normalize(int64_t P, int k, const double* __restrict__ nrm2, const double* __restrict__ w,
                            double* __restrict__ v) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= P * k) return;
    const double n = sqrt(nrm2[idx % k]);
    v[idx] = (n > 0.0) ? w[idx] / n : 0.0;
}

// Givens update of column j of the Hessenberg matrix (per RHS, one thread each)
// Hs: (restart+1) x restart x k column-major per RHS: Hs[(i * restart + col) * k + t]
__global__ void k_givens(int k, int j, int restart, const double* __restrict__ hcol1,
                         const double* __restrict__ hcol2, const double* __restrict__ wnorm2,
                         double* __restrict__ Hs, double* __restrict__ cs, double* __restrict__ sn,
                         double* __restrict__ g, double* __restrict__ res,
                         const int32_t* __restrict__ active) {
    int t = threadIdx.x;
    if (t >= k || !active[t]) return;
    // column entries h[0..j] from the two Gram-Schmidt passes, h[j+1] = ||w||
    double col[130];
    for (int i = 0; i <= j; ++i) col[i] = hcol1[i * k + t] + hcol2[i * k + t];
    col[j + 1] = sqrt(wnorm2[t]);
    for (int i = 0; i < j; ++i) {
        double c = cs[i * k + t], s = sn[i * k + t];
        double a = c * col[i] + s * col[i + 1];
        col[i + 1] = -s * col[i] + c * col[i + 1];
        col[i] = a;
    }
    double den = hypot(col[j], col[j + 1]);
    double c = den > 0.0 ? col[j] / den : 1.0, s = den > 0.0 ? col[j + 1] / den : 0.0;
    cs[j * k + t] = c;
    sn[j * k + t] = s;
    col[j] = den;
    col[j + 1] = 0.0;
    for (int i = 0; i <= j; ++i) Hs[((int64_t)i * restart + j) * k + t] = col[i];
    double gj = g[j * k + t];
    g[(j + 1) * k + t] = -s * gj;
    g[j * k + t] = c * gj;
    res[t] = fabs(-s * gj);
}

// y = R^{-1} g (back substitution) per RHS; x += V y
__global__ void k_gmres_solve(int k, int jn, int restart, const double* __restrict__ Hs,
                              const double* __restrict__ g, double* __restrict__ y,
                              const int32_t* __restrict__ nused) {
    int t = threadIdx.x;
    if (t >= k) return;
    int n = nused[t] < jn ? nused[t] : jn;
    for (int i = n - 1; i >= 0; --i) {
        double s = g[i * k + t];
        for (int q = i + 1; q < n; ++q) s -= Hs[((int64_t)i * restart + q) * k + t] * y[q * k + t];
        double d = Hs[((int64_t)i * restart + i) * k + t];
        y[i * k + t] = d != 0.0 ? s / d : 0.0;
    }
    for (int i = n; i < restart; ++i) y[i * k + t] = 0.0;
}

__global__ void k_gmres_update(int64_t P, int k, int jn, const double* __restrict__ V,
                               const double* __restrict__ y, double* __restrict__ x) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= P * k) return;
    const int t = (int)(idx % k);
    double acc = x[idx];
    for (int i = 0; i < jn; ++i) acc += y[i * k + t] * V[(int64_t)i * P * k + idx];
    x[idx] = acc;
}

__global__ void k_gmres_init(int k, const double* __restrict__ nrm2, double* __restrict__ g,
                             int restart, int32_t* __restrict__ nused) {
    int t = threadIdx.x;
    if (t >= k) return;
    for (int i = 0; i <= restart; ++i) g[i * k + t] = 0.0;
    g[t] = sqrt(nrm2[t]);
    nused[t] = 0;
}

__global__ void k_gmres_count(int k, int j, const int32_t* __restrict__ active, int32_t* __restrict__ nused,
                              int32_t* __restrict__ iters) {
    int t = threadIdx.x;
    if (t >= k || !active[t]) return;
    nused[t] = j + 1;
    iters[t] += 1;
}

__global__ void k_gmres_deactivate(int k, double tol, const double* __restrict__ res,
                                   const double* __restrict__ mbn, int32_t* __restrict__ active) {
    int t = threadIdx.x;
    if (t >= k || !active[t]) return;
    if (res[t] <= tol * mbn[t]) active[t] = 0;
}

// ------------------------------------------------------------------ probes
// value of each (probe, subdomain) pair: P0 * sum_f c_f tanh(z_f)
// val[pair] = P0 sum_f c_f tanh(z_f): 16 pairs per workgroup, 16 lanes per
// pair each summing every 16th feature, lanes meeting by shuffles
template <int KB>
__global__ void __launch_bounds__(256) k_eval_pairs(Geo g, int64_t pairs, const int32_t* __restrict__ pair_sub,
                                                    const double* __restrict__ rec,
                                                    const int32_t* __restrict__ m,
                                                    const int64_t* __restrict__ m_off,
                                                    const double* __restrict__ Rf,
                                                    const double* __restrict__ bf,
                                                    const double* __restrict__ cf, int k, int k0,
                                                    double* __restrict__ val) {
    const int64_t pid = blockIdx.x * 16LL + (threadIdx.x >> 4);
    const int fl = threadIdx.x & 15;
    const bool live = pid < pairs;
    const int j = live ? pair_sub[pid] : 0;
    const double* rr = rec + (live ? pid : 0) * kPairRec;
    double xt[kMaxDim];
    for (int i = 0; i < kMaxDim; ++i) xt[i] = rr[kRecX + i];
    double acc[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) acc[t] = 0.0;
    const int mj = live ? m[j] : 0;
    for (int f = fl; f < mj; f += 16) {
        const int64_t gf = m_off[j] + f;
        double z = bf[gf];
        for (int i = 0; i < g.d; ++i) z = fma(Rf[gf * 4 + i], xt[i], z);
        const double th = tanh(z);
#pragma unroll
        for (int t = 0; t < KB; ++t) acc[t] = fma(th, cf[gf * k + k0 + t], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < KB; ++t)
        for (int off = 1; off < 16; off <<= 1) acc[t] += __shfl_xor(acc[t], off);
    if (live && fl == 0) {
        const double P0 = rr[kRecP0];
#pragma unroll
        for (int t = 0; t < KB; ++t) val[pid * k + k0 + t] = P0 * acc[t];
    }
}

__global__ void k_point_sum(int64_t n, int k, const int64_t* __restrict__ cover_off,
                            const int64_t* __restrict__ cover, const double* __restrict__ val,
                            double* __restrict__ U) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * k) return;
    const int64_t r = idx / k;
    const int t = (int)(idx % k);
    double s = 0.0;
    for (int64_t c = cover_off[r]; c < cover_off[r + 1]; ++c) s += val[cover[c] * k + t];
    U[idx] = s;
}

// transpose: dc_j[f] = sum over probe pairs of j of P0 tanh(z_f) dU[row].
// Workgroup (j, 64-feature group, pair slice z): thread (f, lane pl) sums the
// pairs pl, pl + 4, ... of the slice; the 4 lanes meet in LDS.  With several
// slices the partial sums go to part[z] and k_eval_T_sum adds them in order.
template <int KB>
__global__ void __launch_bounds__(256) k_eval_T(Geo g, const int64_t* __restrict__ row_off,
                                                const int32_t* __restrict__ rows,
                                                const double* __restrict__ rec,
                                                const int32_t* __restrict__ m,
                                                const int64_t* __restrict__ m_off,
                                                const double* __restrict__ Rf,
                                                const double* __restrict__ bf,
                                                const double* __restrict__ dU, int k, int k0,
                                                int64_t sum_m, double* __restrict__ dc) {
    __shared__ double red[4][64];
    const int j = blockIdx.x;
    const int f = blockIdx.y * 64 + (threadIdx.x & 63);
    const int pl = threadIdx.x >> 6;
    const bool live = f < m[j];
    const int64_t gf = m_off[j] + (live ? f : 0);
    const int64_t p0 = row_off[j], np = row_off[j + 1] - p0;
    const int64_t s_lo = p0 + np * blockIdx.z / gridDim.z, s_hi = p0 + np * (blockIdx.z + 1) / gridDim.z;
    double R[kMaxDim];
    for (int i = 0; i < kMaxDim; ++i) R[i] = Rf[gf * 4 + i];
    const double b = bf[gf];
    double acc[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) acc[t] = 0.0;
    if (live) {
        for (int64_t pid = s_lo + pl; pid < s_hi; pid += 4) {
            const double* rr = rec + pid * kPairRec;
            double z = b;
            for (int i = 0; i < g.d; ++i) z = fma(R[i], rr[kRecX + i], z);
            const double w = rr[kRecP0] * tanh(z);
            const double* du = dU + (int64_t)rows[pid] * k + k0;
#pragma unroll
            for (int t = 0; t < KB; ++t) acc[t] = fma(w, du[t], acc[t]);
        }
    }
    double* out = dc + (int64_t)blockIdx.z * sum_m * k;
#pragma unroll
    for (int t = 0; t < KB; ++t) {
        red[pl][threadIdx.x & 63] = acc[t];
        __syncthreads();
        if (pl == 0 && live)
            out[gf * k + k0 + t] = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                                   (red[2][threadIdx.x] + red[3][threadIdx.x]);
        __syncthreads();
    }
}

// dc = sum over the nz pair slices of part[z], in slice order
__global__ void k_eval_T_sum(int64_t n, int nz, const double* __restrict__ part, double* __restrict__ dc) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n) return;
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * n + idx];
    dc[idx] = s;
}

// c_j = V_j W_j (raw-neuron coefficients) and its transpose: 16 outputs per
// workgroup, 16 lanes per output each summing every 16th term, lanes meeting
// by shuffles
__global__ void __launch_bounds__(256) k_coeffs(int64_t sum_m, int k, const int32_t* __restrict__ feat_sub,
                                                const int64_t* __restrict__ m_off, const int32_t* __restrict__ p,
                                                const int64_t* __restrict__ v_off,
                                                const int64_t* __restrict__ col_off,
                                                const double* __restrict__ V, const double* __restrict__ W,
                                                double* __restrict__ c) {
    const int64_t idx = blockIdx.x * 16LL + (threadIdx.x >> 4);
    const int ql = threadIdx.x & 15;
    const bool live = idx < sum_m * k;
    double s = 0.0;
    if (live) {
        const int64_t gf = idx / k;
        const int t = (int)(idx % k);
        const int j = feat_sub[gf];
        const int64_t f = gf - m_off[j];
        const int pj = p[j];
        const double* Vr = V + v_off[j] + f * pj;
        const double* Wj = W + col_off[j] * k + t;
        for (int q = ql; q < pj; q += 16) s = fma(Vr[q], Wj[(int64_t)q * k], s);
    }
    for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off);
    if (live && ql == 0) c[idx] = s;
}

__global__ void __launch_bounds__(256) k_coeffs_T(int64_t P, int k, const int32_t* __restrict__ col_sub,
                                                  const int64_t* __restrict__ m_off, const int32_t* __restrict__ m,
                                                  const int32_t* __restrict__ p, const int64_t* __restrict__ v_off,
                                                  const int64_t* __restrict__ col_off,
                                                  const double* __restrict__ V, const double* __restrict__ dc,
                                                  double* __restrict__ dW) {
    const int64_t idx = blockIdx.x * 16LL + (threadIdx.x >> 4);
    const int fl = threadIdx.x & 15;
    const bool live = idx < P * k;
    double s = 0.0;
    if (live) {
        const int64_t gcol = idx / k;
        const int t = (int)(idx % k);
        const int j = col_sub[gcol];
        const int64_t q = gcol - col_off[j];
        const int pj = p[j];
        const double* Vj = V + v_off[j];
        const double* dcj = dc + m_off[j] * k + t;
        for (int f = fl; f < m[j]; f += 16) s = fma(Vj[(int64_t)f * pj + q], dcj[(int64_t)f * k], s);
    }
    for (int off = 1; off < 16; off <<= 1) s += __shfl_xor(s, off);
    if (live && fl == 0) dW[idx] = s;
}

// ------------------------------------------------------------------ fused CG pieces
// The element-wise kernels run red_grid(P k) workgroups over a grid stride that
// is a multiple of k, so every thread keeps one right-hand side.  Producers of
// dot products write per-workgroup partial sums; each consumer workgroup adds
// them itself in a fixed order (no second launch, no cross-workgroup sync).

constexpr int kRedMax = 240;
// workgroups of an element-wise kernel over n entries: about 4 entries per
// thread, at most kRedMax (each consumer adds every partial)
inline int red_grid(int64_t n) {
    const int64_t g = (n + 1023) / 1024;
    return (int)(g < 32 ? 32 : g > kRedMax ? kRedMax : g);
}

__device__ inline int64_t rhs_stride(int k) { return ((int64_t)gridDim.x * 256 / k) * k; }

// Per-workgroup partial sums by right-hand side, fixed-order tree.  The grid
// stride is a multiple of k, so thread x of block b always handles RHS
// t = (b * 256 + x) % k; threads are grouped by that t.
__device__ void block_partial_by_rhs(double val, int k, double* sh, double* out, int base_override = -1) {
    if (k == 1) {  // a butterfly over each wave, then the four waves
        double w = val;
        for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = w;
        __syncthreads();
        if (threadIdx.x == 0) out[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        __syncthreads();
        return;
    }
    sh[threadIdx.x] = val;
    __syncthreads();
    // general k: thread x with e = x belongs to t(e) = (base + e) % k; sum the
    // entries of each t along e = e0, e0 + k, ... with a pairwise tree
    const int base = base_override >= 0 ? base_override : (int)(((int64_t)blockIdx.x * 256) % k);
    const int groups = (256 + k - 1) / k;  // entries per t (at most)
    for (int st = 1; st < groups; st <<= 1) {
        const int e = threadIdx.x;
        // e is the first entry of a pair at this level when its index along
        // its t-chain is a multiple of 2 st
        const int t = (base + e) % k;
        int e0 = (t - base) % k;
        if (e0 < 0) e0 += k;
        const int idx = (e - e0) / k;
        if ((idx % (2 * st)) == 0 && e + st * k < 256) sh[e] += sh[e + st * k];
        __syncthreads();
    }
    if (threadIdx.x < k) {
        const int t = threadIdx.x;
        int e0 = (t - base) % k;
        if (e0 < 0) e0 += k;
        out[blockIdx.x * k + t] = (e0 < 256) ? sh[e0] : 0.0;
    }
    __syncthreads();
}

// res[t] = sum over the nparts partials part[b * k + t], for t < k
__device__ inline void sum_partials(const double* part, int nparts, int k, double* res, double* sh) {
    sum_partials_kb(part, nparts, k, 0, k, res, sh);
}

// Element-wise loop over idx = i0, i0 + stride, ... < n, four entries per
// round so that their loads are in flight together.
#define RDD_EW_LOOP(i0, stride, n, BODY)                                               \
    for (int64_t base_ = (i0); base_ < (n); base_ += 4 * (stride)) {                   \
        _Pragma("unroll") for (int u_ = 0; u_ < 4; ++u_) {                             \
            const int64_t idx = base_ + u_ * (stride);                                 \
            if (idx < (n)) { BODY }                                                    \
        }                                                                              \
    }

// alpha = rho / <p, s> (from nA partials); x += alpha p; r -= alpha s; partials of <r, r>.
// The operands of each thread's first four entries are loaded before the
// partials are summed (their loads do not wait for alpha).
__global__ void __launch_bounds__(256) k_cg_xr2(int64_t P, int k, int nA, const double* __restrict__ partA,
                                                const double* __restrict__ rho_in,
                                                const int32_t* __restrict__ active_in,
                                                const double* __restrict__ p,
                                                const double* __restrict__ s, double* __restrict__ x,
                                                double* __restrict__ r, double* __restrict__ partB,
                                                int32_t* __restrict__ flags) {
    __shared__ double sh[256];
    __shared__ double al[256];
    const int64_t stride = rhs_stride(k);
    const int64_t i0 = blockIdx.x * 256LL + threadIdx.x;
    const int64_t n = P * k;
    const bool live = i0 < stride;
    double pv[4], sv[4], xv[4], rv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t idx = i0 + u * stride;
        const int64_t ic = (live && idx < n) ? idx : 0;
        pv[u] = p[ic];
        sv[u] = s[ic];
        xv[u] = x[ic];
        rv[u] = r[ic];
    }
    sum_partials(partA, nA, k, al, sh);
    if (threadIdx.x < k) {
        const int t = threadIdx.x;
        double a = 0.0;
        if (active_in[t]) {
            const double pS = al[t];
            if (!(pS > 0.0)) {
                if (blockIdx.x == 0) flags[0] = 1;
            } else {
                a = rho_in[t] / pS;
            }
            if (!isfinite(pS) && blockIdx.x == 0) flags[1] = 1;
        }
        al[t] = a;
    }
    __syncthreads();
    double acc = 0.0;
    if (live) {
        const double a = al[i0 % k];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t idx = i0 + u * stride;
            if (idx < n) {
                x[idx] = fma(a, pv[u], xv[u]);
                const double rn = fma(-a, sv[u], rv[u]);
                r[idx] = rn;
                acc = fma(rn, rn, acc);
            }
        }
        RDD_EW_LOOP(i0 + 4 * stride, stride, n, {
            x[idx] = fma(a, p[idx], x[idx]);
            const double rn = fma(-a, s[idx], r[idx]);
            r[idx] = rn;
            acc = fma(rn, rn, acc);
        })
    }
    block_partial_by_rhs(acc, k, sh, partB);
}

// z = sum of the weighted local solutions (gather form of the Schwarz sum) and
// partials of <r, z>; without a preconditioner z = r
__global__ void __launch_bounds__(256) k_gather_dot(int64_t P, int k, int identity,
                                                    const int64_t* __restrict__ gat_off,
                                                    const int64_t* __restrict__ gat,
                                                    const double* __restrict__ gat_w,
                                                    const double* __restrict__ u,
                                                    const double* __restrict__ r, double* __restrict__ z,
                                                    double* __restrict__ partC) {
    __shared__ double sh[256];
    const int64_t stride = rhs_stride(k);
    const int64_t i0 = blockIdx.x * 256LL + threadIdx.x;
    const int64_t n = P * k;
    double acc = 0.0;
    if (i0 < stride) {
        RDD_EW_LOOP(i0, stride, n, {
            double zv;
            if (identity) {
                zv = r[idx];
            } else {
                const int64_t g = idx / k;
                const int t = (int)(idx % k);
                zv = 0.0;
                const int64_t e1 = gat_off[g + 1];
                // 12 entries per round (a column of a 2D full stencil has up to 9),
                // so that their loads are in flight together
                for (int64_t e0 = gat_off[g]; e0 < e1; e0 += 12) {
                    int64_t gi[12];
                    double wv[12];
                    _Pragma("unroll") for (int v = 0; v < 12; ++v) {
                        gi[v] = (e0 + v < e1) ? gat[e0 + v] : -1;
                        wv[v] = (e0 + v < e1) ? gat_w[e0 + v] : 0.0;
                    }
                    _Pragma("unroll") for (int v = 0; v < 12; ++v) if (gi[v] >= 0) zv += wv[v] * u[gi[v] * k + t];
                }
            }
            z[idx] = zv;
            acc = fma(r[idx], zv, acc);
        })
    }
    block_partial_by_rhs(acc, k, sh, partC);
}

// The Schwarz sum by subdomain: the p_j k entries of z that belong to subdomain
// j are the weighted sum of contiguous segments of the block results, one per
// block that uses j (in block order, as the gather lists add them).
// Task (j, y) of J Y (tasks numbered by XCD, xcd_task) takes the entries
// [y E, (y + 1) E) of subdomain j with E = 4 L, L = (256 / k) k: thread x < L
// the entries y E + x + L v, v < 4, all of right-hand side x % k.  With part,
// workgroup b's partials of <r, z> go to part[b k + t].
__global__ void __launch_bounds__(256) k_gather_seg(int k, int Y, const int32_t* __restrict__ pv,
                                                    const int64_t* __restrict__ col_off,
                                                    const int64_t* __restrict__ seg_off,
                                                    const int64_t* __restrict__ seg_src,
                                                    const double* __restrict__ seg_w,
                                                    const double* __restrict__ u, const double* __restrict__ r,
                                                    double* __restrict__ z, double* __restrict__ part) {
    constexpr int kSB = 9;  // segments per round (a 2D full-stencil subdomain lies in 9 blocks)
    __shared__ double sh[256];
    const int wb = xcd_task(blockIdx.x, gridDim.x);
    const int j = wb / Y, y = wb % Y;
    const int L = (256 / k) * k;
    const int64_t n = (int64_t)pv[j] * k;
    const int64_t s0 = seg_off[j], s1 = seg_off[j + 1];
    const int64_t zb = col_off[j] * k;
    double acc = 0.0;
    if (threadIdx.x < L) {
        const int64_t e0 = (int64_t)y * 4 * L + threadIdx.x;
        double zv[4] = {0.0, 0.0, 0.0, 0.0};
        // the loads of a round's segments are all in flight together; the sums
        // keep the segment order
        for (int64_t q0 = s0; q0 < s1; q0 += kSB) {
            const int nq = (int)((s1 - q0 < kSB) ? (s1 - q0) : kSB);
            double w[kSB], uv[kSB][4];
#pragma unroll
            for (int i = 0; i < kSB; ++i) {
                const double* us = u + ((i < nq) ? seg_src[q0 + i] : 0) * k;
                w[i] = (i < nq) ? seg_w[q0 + i] : 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t e = e0 + (int64_t)L * v;
                    uv[i][v] = (i < nq && e < n) ? us[e] : 0.0;
                }
            }
#pragma unroll
            for (int i = 0; i < kSB; ++i)
                if (i < nq)
#pragma unroll
                    for (int v = 0; v < 4; ++v) zv[v] += w[i] * uv[i][v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t e = e0 + (int64_t)L * v;
            if (e < n) {
                z[zb + e] = zv[v];
                if (part) acc = fma(r[zb + e], zv[v], acc);
            }
        }
    }
    if (part) block_partial_by_rhs(acc, k, sh, part, 0);
}

// beta = <r,z> / rho, rho and activity update (workgroup 0 writes the state of
// the next iteration into the other buffer), p = z + beta p.  The state and
// the operands of each thread's first four entries are loaded before the
// partials are summed.
__global__ void __launch_bounds__(256) k_cg_p2(int64_t P, int k, int nB, int nC, const double* __restrict__ partB,
                                               const double* __restrict__ partC,
                                               const double* __restrict__ bn2,
                                               const double* __restrict__ tol2,
                                               const double* __restrict__ rho_in,
                                               double* __restrict__ rho_out,
                                               const int32_t* __restrict__ active_in,
                                               int32_t* __restrict__ active_out,
                                               int32_t* __restrict__ iters, double* __restrict__ rres,
                                               const double* __restrict__ z, double* __restrict__ p) {
    __shared__ double sh[256];
    __shared__ double rr[256];
    __shared__ double rz[256];
    const int64_t stride = rhs_stride(k);
    const int64_t i0 = blockIdx.x * 256LL + threadIdx.x;
    const int64_t n = P * k;
    const bool live = i0 < stride;
    double pv[4], zv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t idx = i0 + u * stride;
        const int64_t ic = (live && idx < n) ? idx : 0;
        pv[u] = p[ic];
        zv[u] = z[ic];
    }
    const int tl = threadIdx.x < k ? (int)threadIdx.x : 0;
    const int act_l = active_in[tl];
    const double rho_l = rho_in[tl], tol2_l = tol2[tl], bn2_l = bn2[tl];
    sum_partials(partB, nB, k, rr, sh);
    sum_partials(partC, nC, k, rz, sh);
    if (threadIdx.x < k) {
        const int t = threadIdx.x;
        const double b = act_l ? rz[t] / rho_l : 0.0;
        if (blockIdx.x == 0) {
            rho_out[t] = act_l ? rz[t] : rho_l;
            active_out[t] = (act_l && !(rr[t] <= tol2_l * bn2_l)) ? 1 : 0;
            if (act_l) {
                iters[t] += 1;
                rres[t] = sqrt(rr[t] / bn2_l);
            }
        }
        rz[t] = act_l ? b : 0.0;  // reuse as beta
        rr[t] = act_l ? 1.0 : 0.0;  // reuse as the activity
    }
    __syncthreads();
    if (live) {
        const int t = (int)(i0 % k);
        if (rr[t] != 0.0) {
            const double b = rz[t];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t idx = i0 + u * stride;
                if (idx < n) p[idx] = fma(b, pv[u], zv[u]);
            }
            RDD_EW_LOOP(i0 + 4 * stride, stride, n, { p[idx] = fma(b, p[idx], z[idx]); })
        }
    }
}

#undef RDD_EW_LOOP

inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

inline int kb_for(int rem) {
    return rem >= 32 ? 32 : rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
}

}  // namespace

// ------------------------------------------------------------------ launchers
static int gather_rows(const Handle& h, int k) {
    int pmax = 1;
    for (int pj : h.p) pmax = std::max(pmax, pj);
    const int64_t E = 4LL * ((256 / k) * k);
    return (int)std::max<int64_t>(1, ((int64_t)pmax * k + E - 1) / E);
}

int gather_parts(const Handle& h, int k) { return h.geo.J * gather_rows(h, k); }

int launch_gather(Handle& h, const ApplyPlan& pl, const double* ub, const double* r, int k, double* z,
                  double* part) {
    if (k < 1 || k > 256) return RANN_EINVAL;
    const int Y = gather_rows(h, k);
    hipLaunchKernelGGL(k_gather_seg, dim3((unsigned)(h.geo.J * Y)), dim3(256), 0, h.stream, k, Y, h.d_p,
                       h.d_col_off, pl.d_seg_off, pl.d_seg_src, pl.d_seg_w, ub, r, z, part);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

int launch_Hx_pairs(Handle& h, const double* x, int k, double* y, double* tpair);
int launch_HTy_part(Handle& h, const double* y, int k, double* part);

// per-pair scratch of H x, grown on demand (kept apart from the Krylov workspace)
static int ensure_tpair(Handle& h, int k) {
    const size_t need = (size_t)std::max<int64_t>(h.pts.pairs, 1) * k;
    if (h.tpair_elems >= need) return RANN_OK;
    if (h.d_tpair) dev_free(h, h.d_tpair);
    h.d_tpair = nullptr;
    h.tpair_elems = 0;
    RDD_TRY(dev_alloc(h, &h.d_tpair, need));
    h.tpair_elems = need;
    return RANN_OK;
}

int launch_Hx(Handle& h, const double* x, int k, double* y, bool) {
    RDD_TRY(ensure_tpair(h, k));
    return launch_Hx_pairs(h, x, k, y, h.d_tpair);
}

int launch_HTy(Handle& h, const double* y, int k, double* x, double* part) {
    RDD_TRY(launch_HTy_part(h, y, k, part));
    hipLaunchKernelGGL(k_HTy_reduce, dim3(grid_for(h.P * k)), dim3(256), 0, h.stream, h.P, k,
                       h.d_col_sub, h.d_col_off, h.d_chunk_off, h.d_part_off, part, x);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

namespace {

struct Scratch {
    double* base = nullptr;
    size_t used = 0;  // doubles
    double* take(size_t n) {
        double* p = base + used;
        used += (n + 31) & ~size_t(31);
        return p;
    }
};

int dot(Handle& h, int64_t rows, int k, const double* a, const double* b, double* partial, double* out) {
    hipLaunchKernelGGL(k_dot_part, dim3(kDotBlocks), dim3(256), 0, h.stream, rows, k, a, b, partial);
    hipLaunchKernelGGL(k_dot_fin, dim3(1), dim3(256), 0, h.stream, k, kDotBlocks, partial, out);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

// s = H^T H x through the assembled normal matrix
int normal_op(Handle& h, const double* x, int k, double* y, double* part, double* s) {
    (void)y;
    (void)part;
    return launch_normal(h, x, k, s, nullptr);
}

// s = H^T (H x) from the rows of H (y: N k, part: part_total k scratch); the
// residuals that decide convergence use this form, so the assembled normal
// matrix only drives the corrections (iterative refinement)
int exact_normal_op(Handle& h, const double* x, int k, double* y, double* part, double* s) {
    RDD_TRY(launch_Hx(h, x, k, y, false));
    RDD_TRY(launch_HTy(h, y, k, s, part));
    return RANN_OK;
}

// r = H^T (Fs - H W) from the rows of H when the rows' right-hand side Fs is
// known (its rounding scales with the least-squares residual, not with H W),
// else r = rhs - H^T (H W) (the adjoint); y: N k scratch, s: P k scratch
int ls_residual(Handle& h, const double* Fs, const double* rhs, const double* W, int k, double* y,
                double* part, double* s, double* r) {
    const int64_t Pk = h.P * k, Nk = h.N * k;
    RDD_TRY(launch_Hx(h, W, k, y, false));
    if (Fs) {
        hipLaunchKernelGGL(k_sub, dim3(grid_for(Nk)), dim3(256), 0, h.stream, Nk, Fs, y, y);
        RDD_TRY(launch_HTy(h, y, k, r, part));
    } else {
        RDD_TRY(launch_HTy(h, y, k, s, part));
        hipLaunchKernelGGL(k_sub, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, rhs, s, r);
    }
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace

int scale_boundary(Handle& h, const double* F, int k, double* Fs, double factor) {
    const int64_t ni = h.n_int * k, nb = h.n_bnd * k;
    hipLaunchKernelGGL(k_copy, dim3(grid_for(ni)), dim3(256), 0, h.stream, ni, F, Fs);
    if (nb > 0)
        hipLaunchKernelGGL(k_scale_rows, dim3(grid_for(nb)), dim3(256), 0, h.stream, h.n_int, h.n_bnd,
                           k, factor, F, Fs);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

// ||H^T (Fs - H W)|| and ||H^T Fs|| per RHS (host outputs)
int true_residual(Handle& h, const double* Fs, const double* W, int k, double* out_host,
                  double* rhs_norm_host) {
    // own scratch: callers inside a Krylov loop hold pointers into the main workspace
    const size_t need = (size_t)h.N * k * 2 + (size_t)h.P * k * 2 + (size_t)h.part_total * k +
                        (size_t)kDotBlocks * k + 4 * (size_t)k + 256;
    if (h.ws2_bytes < need * sizeof(double)) {
        if (h.ws2) dev_free(h, h.ws2);
        h.ws2 = nullptr;
        h.ws2_bytes = 0;
        double* p2 = nullptr;
        RDD_TRY(dev_alloc(h, &p2, need));
        h.ws2 = p2;
        h.ws2_bytes = need * sizeof(double);
    }
    Scratch sc{static_cast<double*>(h.ws2), 0};
    double* y = sc.take((size_t)h.N * k);
    double* y2 = sc.take((size_t)h.N * k);
    double* r = sc.take((size_t)h.P * k);
    double* g = sc.take((size_t)h.P * k);
    double* part = sc.take((size_t)h.part_total * k);
    double* dp = sc.take((size_t)kDotBlocks * k);
    double* o1 = sc.take(k);
    double* o2 = sc.take(k);
    RDD_TRY(launch_Hx(h, W, k, y, false));
    hipLaunchKernelGGL(k_sub, dim3(grid_for(h.N * k)), dim3(256), 0, h.stream, h.N * k, Fs, y, y2);
    RDD_TRY(launch_HTy(h, y2, k, r, part));
    RDD_TRY(launch_HTy(h, Fs, k, g, part));
    RDD_TRY(dot(h, h.P, k, r, r, dp, o1));
    RDD_TRY(dot(h, h.P, k, g, g, dp, o2));
    std::vector<double> a(k), b(k);
    RDD_TRY(download(h, a.data(), o1, sizeof(double) * k));
    RDD_TRY(download(h, b.data(), o2, sizeof(double) * k));
    RDD_HIP(hipStreamSynchronize(h.stream));
    for (int t = 0; t < k; ++t) {
        out_host[t] = std::sqrt(a[t]);
        if (rhs_norm_host) rhs_norm_host[t] = std::sqrt(b[t]);
    }
    return RANN_OK;
}

// Preconditioned CG on H^T H W = rhs (rhs = H^T Fs, or dW for the adjoint).
// Fs may be null (adjoint): then only the recurrence residual is checked.
static int cg_core(Handle& h, const double* rhs, const double* Fs, int k, const double* W0,
                   const rann_dd_solve_opts& o, double* Wout, std::vector<int>& iters_out,
                   std::vector<double>& res_out, int* status) {
    const size_t P = (size_t)h.P, N = (size_t)h.N;
    const size_t need = P * k * 6 + N * k + (size_t)h.part_total * k + (size_t)(2 * h.ub_total + 2 * h.slot_total) * k +
                        (size_t)kDotBlocks * k + (size_t)(kRedMax + std::max(kRedMax, gather_parts(h, k))) * k +
                        (size_t)h.n_slab_tasks * k + 24 * (size_t)k + 2048;
    RDD_TRY(ensure_ws(h, need * sizeof(double)));
    Scratch sc{static_cast<double*>(h.ws), 0};
    // the iterate lives in the workspace (so that a captured check window does
    // not depend on the caller's buffer) and is copied out at the end
    double* W = sc.take(P * k);
    double* r = sc.take(P * k);
    double* z = sc.take(P * k);
    double* pbuf[2];  // the direction, double-buffered (see the loop)
    pbuf[0] = sc.take(P * k);
    pbuf[1] = sc.take(P * k);
    int pc = 0;
    double* s = sc.take(P * k);
    double* y = sc.take(N * k);
    double* part = sc.take((size_t)h.part_total * k);
    double* ub = sc.take((size_t)(2 * h.ub_total + 2 * h.slot_total) * k);
    double* dp = sc.take((size_t)kDotBlocks * k);
    double* rho = sc.take(k);
    double* pS = sc.take(k);
    double* alpha = sc.take(k);
    double* beta = sc.take(k);
    double* rz = sc.take(k);
    double* rr = sc.take(k);
    double* bn2 = sc.take(k);
    double* tol2v = sc.take(k);
    double* rhoB = sc.take(2 * (size_t)k);       // rho, double-buffered
    double* partA = sc.take((size_t)std::max<int64_t>(1, h.n_slab_tasks) * k);
    double* partB = sc.take((size_t)kRedMax * k);
    const int nC = (h.precond == RANN_PRECOND_NONE) ? 0 : gather_parts(h, k);  // 0: rgrid partials
    double* partC = sc.take((size_t)std::max(kRedMax, nC) * k);
    // the state the host reads after each window, in one block (one copy):
    // recurrence residuals (k doubles), activity (2 k int32, double-buffered),
    // iteration counts (k int32), flags (4 int32)
    const size_t stat_doubles = 3 * (size_t)k + 4;
    double* stat_dev = sc.take(stat_doubles);
    double* rres = stat_dev;
    int32_t* activeB = reinterpret_cast<int32_t*>(stat_dev + k);
    int32_t* iters = reinterpret_cast<int32_t*>(stat_dev + 2 * (size_t)k);
    int32_t* flags = reinterpret_cast<int32_t*>(stat_dev + 3 * (size_t)k);
    (void)rho; (void)pS; (void)alpha; (void)beta; (void)rz; (void)rr;
    int par = 0;
    int32_t* active = activeB;  // current buffer, follows par
    const int64_t Pk = (int64_t)P * k;
    // workgroups of the element-wise kernels
    const unsigned rgrid = (unsigned)std::min(red_grid(Pk), std::max(32, (int)h.tune.red_cap));
    const int nCp = nC > 0 ? nC : (int)rgrid;  // partials of <r, z>
    const int nA = normal_parts(h, k);          // partials of <p, s>

    RDD_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t) * 4, h.stream));
    RDD_HIP(hipMemsetAsync(iters, 0, sizeof(int32_t) * k, h.stream));
    RDD_TRY(dot(h, P, k, rhs, rhs, dp, bn2));
    hipLaunchKernelGGL(k_nan_check, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, rhs, flags + 1);
    // x0, r0 = rhs - A x0
    if (W0) {
        hipLaunchKernelGGL(k_copy, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, W0, W);
        RDD_TRY(normal_op(h, W, k, y, part, s));
        hipLaunchKernelGGL(k_sub, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, rhs, s, r);
    } else {
        RDD_HIP(hipMemsetAsync(W, 0, sizeof(double) * Pk, h.stream));
        hipLaunchKernelGGL(k_copy, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, rhs, r);
    }
    std::vector<double> bn2h(k), tmp(k);
    std::vector<int32_t> act(k, 1), ith(k, 0);
    RDD_TRY(download(h, bn2h.data(), bn2, sizeof(double) * k));
    RDD_HIP(hipStreamSynchronize(h.stream));
    for (int t = 0; t < k; ++t)
        if (!(bn2h[t] > 0.0)) bn2h[t] = 1.0;  // zero right-hand side: solution 0
    RDD_TRY(upload(h, bn2, bn2h.data(), sizeof(double) * k));

    auto restart = [&]() -> int {
        RDD_TRY(launch_precond(h, r, k, z, ub));
        hipLaunchKernelGGL(k_copy, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, z, pbuf[pc]);
        RDD_TRY(dot(h, P, k, r, z, dp, rhoB + (size_t)par * k));
        return RANN_OK;
    };
    RDD_TRY(upload(h, active, act.data(), sizeof(int32_t) * k));
    std::vector<double> tol2h(k, o.tol * o.tol);
    RDD_TRY(upload(h, tol2v, tol2h.data(), sizeof(double) * k));
    RDD_TRY(restart());
    int it = 0;
    const int every = std::max(1, o.check_every);
    std::vector<double> tres(k);
    int replacements = 0, stalls = 0;
    double best_true = 1e300;
    *status = RANN_OK;
    const int ident = (h.precond == RANN_PRECOND_NONE) ? 1 : 0;
    // the launches of iteration q of a check window of nq iterations (device
    // work only, so that a window can be captured into a graph)
    auto launch_iter = [&](int q, int nq) -> int {
        double* rho_in = rhoB + (size_t)par * k;
        double* rho_out = rhoB + (size_t)(par ^ 1) * k;
        int32_t* act_in = activeB + (size_t)par * k;
        int32_t* act_out = activeB + (size_t)(par ^ 1) * k;
        // s = H^T H p (assembled normal matrix) and partials of <p, s>.
        // Inside a check window the previous iteration's direction update
        // p = z + beta p and its bookkeeping ride on this product (into
        // the other direction buffer); the window's last iteration does
        // them itself, so the host always sees a finished iteration.
        if (q > 0) {
            const size_t pq = (size_t)(par ^ 1) * k;  // the previous iteration's state
            const PUpd pu{pbuf[pc], z, pbuf[pc ^ 1], partB, partC, (int)rgrid, nCp, bn2, tol2v,
                          rhoB + pq, rho_in, activeB + pq, act_in, iters, rres};
            RDD_TRY(launch_normal(h, pbuf[pc], k, s, partA, &pu));
            pc ^= 1;
        } else {
            RDD_TRY(launch_normal(h, pbuf[pc], k, s, partA));
        }
        double* p = pbuf[pc];
        hipLaunchKernelGGL(k_cg_xr2, dim3(rgrid), dim3(256), 0, h.stream, (int64_t)P, k, nA, partA, rho_in,
                           act_in, p, s, W, r, partB, flags);
        // z = M^{-1} r and partials of <r, z>
        if (!ident) {
            RDD_TRY(launch_precond_local(h, h.ap, r, k, ub));
            RDD_TRY(launch_gather(h, h.ap, ub, r, k, z, partC));
        } else {
            hipLaunchKernelGGL(k_gather_dot, dim3(rgrid), dim3(256), 0, h.stream, (int64_t)P, k, ident,
                               h.ap.d_gat_off, h.ap.d_gat, h.ap.d_gat_w, ub, r, z, partC);
        }
        if (q + 1 == nq)
            hipLaunchKernelGGL(k_cg_p2, dim3(rgrid), dim3(256), 0, h.stream, (int64_t)P, k, (int)rgrid, nCp, partB,
                               partC, bn2, tol2v, rho_in, rho_out, act_in, act_out, iters, rres, z, p);
        par ^= 1;
        return RANN_OK;
    };
    int window = 0;
    // Window lengths: every iterations, shortened near the end to the
    // iterations that the slowest active right-hand side still needs at the
    // rate of its last window (plus one), so that few iterations run past
    // convergence; windows shorter than every run eagerly.
    std::vector<double> stat(stat_doubles), rprev(k, -1.0);
    int next_nq = every, nq_prev = 0;
    while (true) {
        const int nq = std::min(next_nq, o.maxiter - it);
        // with the kernel timers on, one window in four runs eagerly with its
        // timers; the others run without timers (from the graph when allowed),
        // so that the timers' events do not slow the timed solve down
        const bool sampled = ktime_enabled() && (window++ % 4 == 0);
        KTimeOff quiet_window(!sampled);
        // a full window replays a captured graph of its launches when the
        // handle allows it: the launches depend only on the workspace, the
        // sizes, the launch parameters and the parities of the two double
        // buffers at the window's start
        hipGraphExec_t ex = nullptr;
        if (!sampled && h.tune.use_graph && !h.graph_broken && nq == every && nq > 0) {
            uint64_t key = 1469598103934665603ULL;
            const uint64_t parts[] = {(uint64_t)(uintptr_t)h.ws, (uint64_t)k, (uint64_t)nq, (uint64_t)par,
                                      (uint64_t)pc, (uint64_t)h.tune.tile_grid, (uint64_t)rgrid, (uint64_t)P};
            for (uint64_t v : parts) key = (key ^ v) * 1099511628211ULL;
            for (auto& g : h.cg_graph)
                if (g.exec && g.key == key) ex = g.exec;
            if (!ex) {
                const int par0 = par, pc0 = pc;
                KTimeOff no_timers;
                int rc = RANN_OK;
                hipGraph_t graph = nullptr;
                // captured on a private stream (the handle's may be the null
                // stream, which cannot be captured); replayed on the handle's
                if (!h.cap_stream && hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking) != hipSuccess)
                    h.cap_stream = nullptr;
                const hipStream_t own = h.stream;
                if (h.cap_stream && hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                    h.stream = h.cap_stream;
                    for (int q = 0; q < nq && rc == RANN_OK; ++q) rc = launch_iter(q, nq);
                    h.stream = own;
                    const hipError_t e = hipStreamEndCapture(h.cap_stream, &graph);
                    if (rc == RANN_OK && e == hipSuccess && graph &&
                        hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess)
                        ex = nullptr;
                    if (graph) (void)hipGraphDestroy(graph);
                }
                h.stream = own;
                par = par0;  // the captured launches have not run
                pc = pc0;
                if (ex) {
                    auto& slot = h.cg_graph[h.cg_graph_next];
                    h.cg_graph_next = (h.cg_graph_next + 1) % 4;
                    if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
                    slot.exec = ex;
                    slot.key = key;
                } else {
                    h.graph_broken = 1;  // eager launches from now on
                    (void)hipGetLastError();
                }
            }
        }
        if (ex) {
            RDD_HIP(hipGraphLaunch(ex, h.stream));
            // the state of the double buffers after the window's iterations
            par ^= (nq & 1);
            pc ^= ((nq - 1) & 1);
        } else {
            for (int q = 0; q < nq; ++q) RDD_TRY(launch_iter(q, nq));
        }
        it += nq;
        active = activeB + (size_t)par * k;
        RDD_HIP(hipGetLastError());
        RDD_TRY(download(h, stat.data(), stat_dev, sizeof(double) * stat_doubles));
        RDD_HIP(hipStreamSynchronize(h.stream));
        const int32_t* act_now = reinterpret_cast<const int32_t*>(stat.data() + k) + (size_t)par * k;
        std::copy(act_now, act_now + k, act.begin());
        const int32_t* fl = reinterpret_cast<const int32_t*>(stat.data() + 3 * (size_t)k);
        {
            int need = 0;
            bool known = nq_prev > 0;
            for (int t = 0; t < k && known; ++t) {
                if (!act[t]) continue;
                const double now = stat[t], before = rprev[t], tl = std::sqrt(tol2h[t]);
                if (!(tl > 0.0 && now > tl && before > now)) {
                    known = false;
                    break;
                }
                const double rate = std::log(now / before) / nq_prev;  // per iteration, < 0
                const double rem = std::ceil(std::log(tl / now) / rate);
                if (!(rem < every)) {
                    known = false;
                    break;
                }
                need = std::max(need, (int)rem);
            }
            next_nq = known ? std::max(1, std::min(every, need + 1)) : every;
            for (int t = 0; t < k; ++t) rprev[t] = stat[t];
            nq_prev = nq;
        }
        if (fl[1]) {
            set_error("NaN or Inf in the Krylov iteration");
            return RANN_ENAN;
        }
        if (fl[0]) {
            set_error("CG breakdown: <p, H^T H p> <= 0");
            return RANN_EBREAKDOWN;
        }
        bool any = false;
        for (int t = 0; t < k; ++t) any |= act[t] != 0;
        if (!any) {
            if (Fs == nullptr) break;
            // confirm on the true FP64 normal residual recomputed from scratch; a
            // right-hand side that fails it resumes its recurrence with a tighter
            // recurrence threshold, or restarts from the true residual when the
            // recurrence has drifted far from it
            RDD_TRY(true_residual(h, Fs, W, k, tres.data(), tmp.data()));
            std::vector<double> rrh(k);
            RDD_TRY(download(h, rrh.data(), rres, sizeof(double) * k));
            bool again = false, drift = false;
            for (int t = 0; t < k; ++t) {
                double relr = tmp[t] > 0 ? tres[t] / tmp[t] : 0.0;
                if (relr > o.tol) {
                    act[t] = 1;
                    again = true;
                    tol2h[t] *= 0.01;
                    if (relr > 1e3 * std::max(rrh[t], 1e-300)) drift = true;
                }
            }
            bool floor_hit = false;
            for (int t = 0; t < k; ++t) floor_hit |= tol2h[t] < 1e-60;
            // stagnation: the true residual stopped improving at the FP64 floor
            double worst = 0.0;
            for (int t = 0; t < k; ++t) worst = std::max(worst, tmp[t] > 0 ? tres[t] / tmp[t] : 0.0);
            if (worst < 0.9 * best_true) {
                best_true = worst;
                stalls = 0;
            } else {
                ++stalls;
                // no progress since the last check: restart from the true
                // residual (a step of iterative refinement on H^T H through the
                // rows of H) before counting it as the floor
                drift = again;
            }
            if (!again || it >= o.maxiter || replacements > 20 || floor_hit || stalls >= 4) {
                if (again) *status = RANN_ENOTCONV;
                break;
            }
            RDD_TRY(upload(h, tol2v, tol2h.data(), sizeof(double) * k));
            RDD_TRY(upload(h, active, act.data(), sizeof(int32_t) * k));
            if (drift) {
                ++replacements;
                RDD_TRY(launch_Hx(h, W, k, y, false));
                hipLaunchKernelGGL(k_sub, dim3(grid_for((int64_t)N * k)), dim3(256), 0, h.stream,
                                   (int64_t)N * k, Fs, y, y);
                RDD_TRY(launch_HTy(h, y, k, r, part));
                RDD_TRY(restart());
            }
            continue;
        }
        if (it >= o.maxiter) {
            *status = RANN_ENOTCONV;
            break;
        }
    }
    hipLaunchKernelGGL(k_copy, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, W, Wout);
    RDD_TRY(download(h, ith.data(), iters, sizeof(int32_t) * k));
    std::vector<double> rrh(k);
    RDD_TRY(download(h, rrh.data(), rres, sizeof(double) * k));
    RDD_HIP(hipStreamSynchronize(h.stream));
    iters_out.assign(ith.begin(), ith.end());
    res_out = rrh;
    return RANN_OK;
}

namespace {
// x[i] = a pseudo-random value in [-1, 1) from a 64-bit mix of i (SplitMix64)
__global__ void k_fill_mix(int64_t n, double* __restrict__ x) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}
}  // namespace

// Time of `iters` CG iterations with k right-hand sides under the handle's
// current launch parameters (tolerance 0, a fixed pseudo-random right-hand
// side; rhs and W: P k device scratch); the first run (graph capture, caches)
// is not timed.
int time_cg_iterations(Handle& h, int k, int iters, double* rhs, double* W, double* us_per_iter) {
    const int64_t Pk = h.P * (int64_t)k;
    hipLaunchKernelGGL(k_fill_mix, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, rhs);
    RDD_HIP(hipGetLastError());
    rann_dd_solve_opts o{0.0, iters, RANN_METHOD_CG, 0, std::min(10, iters)};
    std::vector<int> its;
    std::vector<double> res;
    int status = 0;
    RDD_TRY(cg_core(h, rhs, nullptr, k, nullptr, o, W, its, res, &status));
    hipEvent_t a, b;
    RDD_HIP(hipEventCreate(&a));
    RDD_HIP(hipEventCreate(&b));
    (void)hipEventRecord(a, h.stream);
    const int rc = cg_core(h, rhs, nullptr, k, nullptr, o, W, its, res, &status);
    (void)hipEventRecord(b, h.stream);
    float ms = 0.0f;
    const hipError_t e = hipEventSynchronize(b);
    if (e == hipSuccess) (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    RDD_TRY(rc);
    RDD_HIP(e);
    *us_per_iter = 1e3 * (double)ms / iters;
    return RANN_OK;
}

int krylov_cg(Handle& h, const double* Fs, int k, const double* W0, const rann_dd_solve_opts& o,
              double* W, rann_dd_stats* st, int* status) {
    double* rhs = nullptr;
    double* part = nullptr;
    RDD_TRY(dev_alloc(h, &rhs, (size_t)h.P * k));
    RDD_TRY(dev_alloc(h, &part, (size_t)h.part_total * k));
    RDD_TRY(launch_HTy(h, Fs, k, rhs, part));
    std::vector<int> iters;
    std::vector<double> rres;
    int rc = cg_core(h, rhs, Fs, k, W0, o, W, iters, rres, status);
    dev_free(h, part);
    if (rc < 0) {
        dev_free(h, rhs);
        return rc;
    }
    dev_free(h, rhs);
    if (st) {
        std::vector<double> tres(k), bn(k);
        RDD_TRY(true_residual(h, Fs, W, k, tres.data(), bn.data()));
        st->iterations = 0;
        st->converged = 0;
        st->max_rel_residual = 0.0;
        for (int t = 0; t < k; ++t) {
            double rel = bn[t] > 0 ? tres[t] / bn[t] : 0.0;
            st->iterations = std::max(st->iterations, iters[t]);
            st->converged += rel <= o.tol ? 1 : 0;
            st->max_rel_residual = std::max(st->max_rel_residual, rel);
            if (st->rel_residual) st->rel_residual[t] = rel;
            if (st->rhs_iterations) st->rhs_iterations[t] = iters[t];
        }
        st->shifts = h.shifts;
    }
    return RANN_OK;
}

int adjoint_cg(Handle& h, const double* dW, int k, const rann_dd_solve_opts& o, double* z,
               rann_dd_stats* st, int* status) {
    std::vector<int> iters;
    std::vector<double> rres;
    RDD_TRY(cg_core(h, dW, nullptr, k, nullptr, o, z, iters, rres, status));
    if (st) {
        st->iterations = 0;
        st->converged = 0;
        st->max_rel_residual = 0.0;
        for (int t = 0; t < k; ++t) {
            st->iterations = std::max(st->iterations, iters[t]);
            st->converged += rres[t] <= o.tol ? 1 : 0;
            st->max_rel_residual = std::max(st->max_rel_residual, rres[t]);
            if (st->rel_residual) st->rel_residual[t] = rres[t];
            if (st->rhs_iterations) st->rhs_iterations[t] = iters[t];
        }
        st->shifts = h.shifts;
    }
    return RANN_OK;
}

// Left-preconditioned GMRES(restart): minimise ||M^{-1}(rhs - H^T H W)|| per RHS.
static int gmres_core(Handle& h, const double* rhs, const double* Fs, int k, const double* W0,
                      const rann_dd_solve_opts& o, double* W, std::vector<int>& iters_out,
                      int* status) {
    const int m = std::max(1, std::min(o.restart, 128));
    const size_t P = (size_t)h.P, N = (size_t)h.N;
    const size_t need = P * k * (m + 1) + P * k * 3 + N * k + (size_t)h.part_total * k +
                        (size_t)(2 * h.ub_total + 2 * h.slot_total) * k + (size_t)kDotBlocks * k * (m + 1) +
                        (size_t)k * ((m + 1) * m + 6 * (m + 1) + 16) + 1024;
    RDD_TRY(ensure_ws(h, need * sizeof(double)));
    Scratch sc{static_cast<double*>(h.ws), 0};
    double* V = sc.take(P * k * (m + 1));
    double* w = sc.take(P * k);
    double* s = sc.take(P * k);
    double* t0 = sc.take(P * k);
    double* y = sc.take(N * k);
    double* part = sc.take((size_t)h.part_total * k);
    double* ub = sc.take((size_t)(2 * h.ub_total + 2 * h.slot_total) * k);
    double* dp = sc.take((size_t)kDotBlocks * k * (m + 1));
    double* Hs = sc.take((size_t)k * (m + 1) * m);
    double* h1 = sc.take((size_t)k * (m + 1));
    double* h2 = sc.take((size_t)k * (m + 1));
    double* cs = sc.take((size_t)k * (m + 1));
    double* sn = sc.take((size_t)k * (m + 1));
    double* g = sc.take((size_t)k * (m + 1));
    double* yv = sc.take((size_t)k * (m + 1));
    double* nrm = sc.take(k);
    double* res = sc.take(k);
    double* mbn = sc.take(k);
    int32_t* active = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* nused = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* iters = reinterpret_cast<int32_t*>(sc.take(k));
    const int64_t Pk = (int64_t)P * k;
    RDD_HIP(hipMemsetAsync(iters, 0, sizeof(int32_t) * k, h.stream));
    if (W0) {
        hipLaunchKernelGGL(k_copy, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, W0, W);
    } else {
        RDD_HIP(hipMemsetAsync(W, 0, sizeof(double) * Pk, h.stream));
    }
    // right preconditioning: GMRES on A M^{-1}, W = W0 + M^{-1} (V y), residuals
    // unpreconditioned; left: GMRES on M^{-1} A with preconditioned residuals
    const bool right = (o.method == RANN_METHOD_GMRES_RIGHT);
    // ||M^{-1} rhs|| (left) or ||rhs|| (right)
    if (right)
        hipLaunchKernelGGL(k_copy, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, rhs, w);
    else
        RDD_TRY(launch_precond(h, rhs, k, w, ub));
    RDD_TRY(dot(h, P, k, w, w, dp, nrm));
    std::vector<double> mb(k);
    RDD_TRY(download(h, mb.data(), nrm, sizeof(double) * k));
    RDD_HIP(hipStreamSynchronize(h.stream));
    for (int t = 0; t < k; ++t) mb[t] = mb[t] > 0 ? std::sqrt(mb[t]) : 1.0;
    RDD_TRY(upload(h, mbn, mb.data(), sizeof(double) * k));
    double tol_p = o.tol;
    int it = 0, cycles = 0;
    std::vector<int32_t> act(k, 1);
    std::vector<double> tres(k), bn(k), rh(k);
    *status = RANN_OK;
    while (true) {
        // r = M^{-1}(rhs - A W) (left) or rhs - A W (right), A applied through the rows of H
        if (right) {
            RDD_TRY(ls_residual(h, Fs, rhs, W, k, y, part, s, w));
        } else {
            RDD_TRY(ls_residual(h, Fs, rhs, W, k, y, part, s, t0));
            RDD_TRY(launch_precond(h, t0, k, w, ub));
        }
        RDD_TRY(dot(h, P, k, w, w, dp, nrm));
        hipLaunchKernelGGL(k_normalize, dim3(grid_for(Pk)), dim3(256), 0, h.stream, (int64_t)P, k, nrm,
                           w, V);
        hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(256), 0, h.stream, k, nrm, g, m, nused);
        // active: those whose preconditioned residual is above tol_p
        RDD_TRY(download(h, rh.data(), nrm, sizeof(double) * k));
        RDD_HIP(hipStreamSynchronize(h.stream));
        bool any = false;
        for (int t = 0; t < k; ++t) {
            act[t] = (std::sqrt(rh[t]) > tol_p * mb[t]) ? 1 : 0;
            any |= act[t] != 0;
        }
        RDD_TRY(upload(h, active, act.data(), sizeof(int32_t) * k));
        int jn = 0;
        if (any) {
            for (int j = 0; j < m && it < o.maxiter; ++j, ++it) {
                double* vj = V + (size_t)j * P * k;
                if (right) {
                    RDD_TRY(launch_precond(h, vj, k, t0, ub));
                    RDD_TRY(normal_op(h, t0, k, y, part, w));
                } else {
                    RDD_TRY(normal_op(h, vj, k, y, part, s));
                    RDD_TRY(launch_precond(h, s, k, w, ub));
                }
                // classical Gram-Schmidt, twice
                hipLaunchKernelGGL(k_mdot_part, dim3(kDotBlocks, j + 1), dim3(256), 0, h.stream,
                                   (int64_t)P, k, j + 1, V, w, dp);
                hipLaunchKernelGGL(k_mdot_fin, dim3((unsigned)(((j + 1) * k + 255) / 256)), dim3(256), 0,
                                   h.stream, k, j + 1, kDotBlocks, dp, h1);
                hipLaunchKernelGGL(k_mgs_update, dim3(grid_for(Pk)), dim3(256), 0, h.stream, (int64_t)P,
                                   k, j + 1, V, h1, w);
                hipLaunchKernelGGL(k_mdot_part, dim3(kDotBlocks, j + 1), dim3(256), 0, h.stream,
                                   (int64_t)P, k, j + 1, V, w, dp);
                hipLaunchKernelGGL(k_mdot_fin, dim3((unsigned)(((j + 1) * k + 255) / 256)), dim3(256), 0,
                                   h.stream, k, j + 1, kDotBlocks, dp, h2);
                hipLaunchKernelGGL(k_mgs_update, dim3(grid_for(Pk)), dim3(256), 0, h.stream, (int64_t)P,
                                   k, j + 1, V, h2, w);
                RDD_TRY(dot(h, P, k, w, w, dp, nrm));
                hipLaunchKernelGGL(k_normalize, dim3(grid_for(Pk)), dim3(256), 0, h.stream, (int64_t)P, k,
                                   nrm, w, V + (size_t)(j + 1) * P * k);
                hipLaunchKernelGGL(k_givens, dim3(1), dim3(256), 0, h.stream, k, j, m, h1, h2, nrm, Hs,
                                   cs, sn, g, res, active);
                hipLaunchKernelGGL(k_gmres_count, dim3(1), dim3(256), 0, h.stream, k, j, active, nused,
                                   iters);
                hipLaunchKernelGGL(k_gmres_deactivate, dim3(1), dim3(256), 0, h.stream, k, tol_p, res, mbn,
                                   active);
                jn = j + 1;
                if ((j + 1) % std::max(1, o.check_every) == 0) {
                    RDD_TRY(download(h, act.data(), active, sizeof(int32_t) * k));
                    RDD_HIP(hipStreamSynchronize(h.stream));
                    bool a2 = false;
                    for (int t = 0; t < k; ++t) a2 |= act[t] != 0;
                    if (!a2) break;
                }
            }
            hipLaunchKernelGGL(k_gmres_solve, dim3(1), dim3(256), 0, h.stream, k, jn, m, Hs, g, yv, nused);
            if (right) {
                // W += M^{-1} (V y)
                RDD_HIP(hipMemsetAsync(t0, 0, sizeof(double) * Pk, h.stream));
                hipLaunchKernelGGL(k_gmres_update, dim3(grid_for(Pk)), dim3(256), 0, h.stream, (int64_t)P,
                                   k, jn, V, yv, t0);
                RDD_TRY(launch_precond(h, t0, k, w, ub));
                hipLaunchKernelGGL(k_add, dim3(grid_for(Pk)), dim3(256), 0, h.stream, Pk, w, W);
            } else {
                hipLaunchKernelGGL(k_gmres_update, dim3(grid_for(Pk)), dim3(256), 0, h.stream, (int64_t)P,
                                   k, jn, V, yv, W);
            }
            RDD_HIP(hipGetLastError());
        }
        ++cycles;
        // convergence on the true normal residual
        if (Fs) {
            RDD_TRY(true_residual(h, Fs, W, k, tres.data(), bn.data()));
            bool ok = true;
            for (int t = 0; t < k; ++t) ok &= (bn[t] > 0 ? tres[t] / bn[t] : 0.0) <= o.tol;
            if (ok) break;
            if (!any) tol_p *= 0.1;  // preconditioned residual met but true residual not yet
        } else if (!any) {
            break;
        }
        if (it >= o.maxiter || cycles > 10000 || tol_p < 1e-30) {
            *status = RANN_ENOTCONV;
            break;
        }
    }
    std::vector<int32_t> ith(k);
    RDD_TRY(download(h, ith.data(), iters, sizeof(int32_t) * k));
    RDD_HIP(hipStreamSynchronize(h.stream));
    iters_out.assign(ith.begin(), ith.end());
    return RANN_OK;
}

int krylov_gmres(Handle& h, const double* Fs, int k, const double* W0, const rann_dd_solve_opts& o,
                 double* W, rann_dd_stats* st, int* status) {
    double* rhs = nullptr;
    double* part = nullptr;
    RDD_TRY(dev_alloc(h, &rhs, (size_t)h.P * k));
    RDD_TRY(dev_alloc(h, &part, (size_t)h.part_total * k));
    RDD_TRY(launch_HTy(h, Fs, k, rhs, part));
    dev_free(h, part);
    std::vector<int> iters;
    int rc = gmres_core(h, rhs, Fs, k, W0, o, W, iters, status);
    dev_free(h, rhs);
    RDD_TRY(rc);
    if (st) {
        std::vector<double> tres(k), bn(k);
        RDD_TRY(true_residual(h, Fs, W, k, tres.data(), bn.data()));
        st->iterations = 0;
        st->converged = 0;
        st->max_rel_residual = 0.0;
        for (int t = 0; t < k; ++t) {
            double rel = bn[t] > 0 ? tres[t] / bn[t] : 0.0;
            st->iterations = std::max(st->iterations, iters[t]);
            st->converged += rel <= o.tol ? 1 : 0;
            st->max_rel_residual = std::max(st->max_rel_residual, rel);
            if (st->rel_residual) st->rel_residual[t] = rel;
            if (st->rhs_iterations) st->rhs_iterations[t] = iters[t];
        }
        st->shifts = h.shifts;
    }
    return RANN_OK;
}

int adjoint_gmres(Handle& h, const double* dW, int k, const rann_dd_solve_opts& o, double* z,
                  rann_dd_stats* st, int* status) {
    std::vector<int> iters;
    RDD_TRY(gmres_core(h, dW, nullptr, k, nullptr, o, z, iters, status));
    if (st) {
        st->iterations = 0;
        for (int t = 0; t < k; ++t) {
            st->iterations = std::max(st->iterations, iters[t]);
            if (st->rhs_iterations) st->rhs_iterations[t] = iters[t];
        }
        st->converged = k;
        st->max_rel_residual = 0.0;
        st->shifts = h.shifts;
    }
    return RANN_OK;
}

// ------------------------------------------------------------------ CGS and BiCG
// Conjugate gradients squared (Sonneveld) and biconjugate gradients (Fletcher),
// the Krylov variants of the paper's Table 1b that also take the
// non-symmetric SAS and RAS preconditioners (Sec. 5, Example 1).  Vectors are
// (P, k) with the right-hand side fastest; every per-RHS scalar stays on the
// device and inactive right-hand sides are frozen by the element-wise kernels.
namespace {

// partial[b][t] of <a, b> and, at partial + nb k, of <c, d>
__global__ void __launch_bounds__(256) k_dot2_part(int64_t rows, int k, const double* __restrict__ a,
                                                   const double* __restrict__ b, const double* __restrict__ c,
                                                   const double* __restrict__ d, double* __restrict__ partial) {
    __shared__ double s1[256], s2[256];
    const int per = 256 / k;
    const int t = threadIdx.x % k, ro = threadIdx.x / k;
    double acc1 = 0.0, acc2 = 0.0;
    if (ro < per) {
        for (int64_t r = (int64_t)blockIdx.x * per + ro; r < rows; r += (int64_t)gridDim.x * per) {
            acc1 = fma(a[r * k + t], b[r * k + t], acc1);
            acc2 = fma(c[r * k + t], d[r * k + t], acc2);
        }
    }
    if (pow2_upto64(k)) {
        const double t1 = wave_block_sum(acc1, k, s1);
        const double t2 = wave_block_sum(acc2, k, s2);
        if (threadIdx.x < k) {
            partial[blockIdx.x * k + threadIdx.x] = t1;
            partial[((int64_t)gridDim.x + blockIdx.x) * k + threadIdx.x] = t2;
        }
        return;
    }
    s1[threadIdx.x] = (ro < per) ? acc1 : 0.0;
    s2[threadIdx.x] = (ro < per) ? acc2 : 0.0;
    __syncthreads();
    if (threadIdx.x < k) {
        double t1 = 0.0, t2 = 0.0;
        for (int q = 0; q < per; ++q) {
            t1 += s1[q * k + threadIdx.x];
            t2 += s2[q * k + threadIdx.x];
        }
        partial[blockIdx.x * k + threadIdx.x] = t1;
        partial[((int64_t)gridDim.x + blockIdx.x) * k + threadIdx.x] = t2;
    }
}

// (re)start: right-hand sides with go[t] set become active with a fresh
// direction; the others keep their state
__global__ void k_lz_start(int k, const int32_t* __restrict__ go, int32_t* __restrict__ active,
                           int32_t* __restrict__ first, int32_t* __restrict__ brk, int32_t* __restrict__ cyc) {
    const int t = threadIdx.x;
    if (t >= k || !go[t]) return;
    active[t] = 1;
    first[t] = 1;
    brk[t] = 0;
    cyc[t] = 0;
}

// alpha = rho / sigma; a zero or non-finite step is a breakdown: the right-hand
// side stops and the host restarts it from its true residual
__global__ void k_lz_alpha(int k, const double* __restrict__ rho, const double* __restrict__ sigma,
                           int32_t* __restrict__ active, int32_t* __restrict__ brk, double* __restrict__ alpha) {
    const int t = threadIdx.x;
    if (t >= k || !active[t]) return;
    const double a = rho[t] / sigma[t];
    if (rho[t] == 0.0 || sigma[t] == 0.0 || !isfinite(a)) {
        active[t] = 0;
        brk[t] = 1;
        alpha[t] = 0.0;
        return;
    }
    alpha[t] = a;
}

// per right-hand side after an iteration: count it, record the recurrence
// residual, stop when it meets the threshold, shift rho (rho_next: the new
// <r~, r> of CGS; BiCG recomputes rho at the top of its iteration).  With
// cap > 0 a cycle ends after cap iterations (brk set: restart, not converged).
__global__ void k_lz_fin(int k, int cap, const double* __restrict__ rr, const double* __restrict__ bn2,
                         const double* __restrict__ tol2, double* __restrict__ rho,
                         double* __restrict__ rho_old, const double* __restrict__ rho_next,
                         int32_t* __restrict__ first, int32_t* __restrict__ active, int32_t* __restrict__ brk,
                         int32_t* __restrict__ cyc, int32_t* __restrict__ iters, double* __restrict__ rres,
                         int32_t* __restrict__ flags) {
    const int t = threadIdx.x;
    if (t >= k || !active[t]) return;
    iters[t] += 1;
    cyc[t] += 1;
    if (!isfinite(rr[t])) flags[1] = 1;
    rres[t] = sqrt(rr[t] / bn2[t]);
    rho_old[t] = rho[t];
    if (rho_next) rho[t] = rho_next[t];
    first[t] = 0;
    if (rr[t] <= tol2[t] * bn2[t]) {
        active[t] = 0;
    } else if (cap > 0 && cyc[t] >= cap) {
        active[t] = 0;
        brk[t] = 1;
    }
}

// CGS directions: u = r + beta q, pd = u + beta (q + beta pd), beta = rho /
// rho_old; on a (re)start u = pd = r
__global__ void k_cgs_dir(int64_t n, int k, const double* __restrict__ rho, const double* __restrict__ rho_old,
                          const int32_t* __restrict__ first, const int32_t* __restrict__ active,
                          const double* __restrict__ r, const double* __restrict__ q, double* __restrict__ u,
                          double* __restrict__ pd) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = (int)(i % k);
    if (!active[t]) return;
    if (first[t]) {
        u[i] = r[i];
        pd[i] = r[i];
        return;
    }
    const double beta = rho[t] / rho_old[t];
    const double uu = fma(beta, q[i], r[i]);
    u[i] = uu;
    pd[i] = fma(beta, fma(beta, pd[i], q[i]), uu);
}

// q = u - alpha v, w = u + q
__global__ void k_cgs_q(int64_t n, int k, const double* __restrict__ alpha, const int32_t* __restrict__ active,
                        const double* __restrict__ u, const double* __restrict__ v, double* __restrict__ q,
                        double* __restrict__ w) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = (int)(i % k);
    if (!active[t]) return;
    const double qq = fma(-alpha[t], v[i], u[i]);
    q[i] = qq;
    w[i] = u[i] + qq;
}

// x += alpha dx, r -= alpha dr and, when rt is given, rt -= alpha drt
__global__ void k_lz_xr(int64_t n, int k, const double* __restrict__ alpha, const int32_t* __restrict__ active,
                        const double* __restrict__ dx, const double* __restrict__ dr,
                        const double* __restrict__ drt, double* __restrict__ x, double* __restrict__ r,
                        double* __restrict__ rt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = (int)(i % k);
    if (!active[t]) return;
    const double a = alpha[t];
    x[i] = fma(a, dx[i], x[i]);
    r[i] = fma(-a, dr[i], r[i]);
    if (rt) rt[i] = fma(-a, drt[i], rt[i]);
}

// BiCG directions: pd = z + beta pd, pt = zt + beta pt (beta = 0 on a restart)
__global__ void k_bicg_dir(int64_t n, int k, const double* __restrict__ rho, const double* __restrict__ rho_old,
                           const int32_t* __restrict__ first, const int32_t* __restrict__ active,
                           const double* __restrict__ z, const double* __restrict__ zt, double* __restrict__ pd,
                           double* __restrict__ pt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = (int)(i % k);
    if (!active[t]) return;
    if (first[t]) {
        pd[i] = z[i];
        pt[i] = zt[i];
        return;
    }
    const double beta = rho[t] / rho_old[t];
    pd[i] = fma(beta, pd[i], z[i]);
    pt[i] = fma(beta, pt[i], zt[i]);
}

}  // namespace

// CGS or BiCG on H^T H W = rhs.  The recurrences run on the assembled normal
// matrix; when every right-hand side has met the threshold on its recurrence
// residual (or broken down), the FP64 residual is recomputed from the rows of
// H and the right-hand sides that fail it restart from it (shadow r~ = r): the
// outer loop of the oracle.
//
// Mixed precision: the FP32 local solves make M^{-1} inexact, and these
// recurrences, unlike CG's, then lose their (bi)orthogonality and can diverge
// once the residual has fallen a few orders below its start.  So each cycle is
// an iterative-refinement step: it stops when its recurrence residual has
// dropped 1e4-fold (or meets tol) or after o.restart iterations, and the next
// cycle restarts from the FP64 residual.
int krylov_lanczos(Handle& h, const double* rhs, const double* Fs, int k, const double* W0,
                   const rann_dd_solve_opts& o, double* W, rann_dd_stats* st, int* status) {
    const bool cgs = (o.method == RANN_METHOD_CGS);
    const size_t P = (size_t)h.P, N = (size_t)h.N;
    const size_t need = P * k * 11 + k + N * k + (size_t)h.part_total * k +
                        (size_t)(2 * h.ub_total + 2 * h.slot_total) * k + 2 * (size_t)kDotBlocks * k +
                        40 * (size_t)k + 2048;
    RDD_TRY(ensure_ws(h, need * sizeof(double)));
    Scratch sc{static_cast<double*>(h.ws), 0};
    double* r = sc.take(P * k);
    double* rt = sc.take(P * k);
    double* v1 = sc.take(P * k);  // CGS: u      BiCG: z
    double* v2 = sc.take(P * k);  // CGS: pd     BiCG: zt
    double* v3 = sc.take(P * k);  // CGS: q      BiCG: pd
    double* v4 = sc.take(P * k);  // CGS: ph     BiCG: pt
    double* v5 = sc.take(P * k);  // CGS: vh     BiCG: q
    double* v6 = sc.take(P * k);  // CGS: w      BiCG: qt
    double* v7 = sc.take((P + 1) * k);  // CGS: uh     BiCG: M^{-T} scratch ((P + 1) k)
    double* v8 = sc.take(P * k);  // CGS: A uh
    double* y = sc.take(N * k);
    double* part = sc.take((size_t)h.part_total * k);
    double* ub = sc.take((size_t)(2 * h.ub_total + 2 * h.slot_total) * k);
    double* dp = sc.take(2 * (size_t)kDotBlocks * k);
    double* rho = sc.take(k);
    double* rho_old = sc.take(k);
    double* rho_next = sc.take(k);
    double* sigma = sc.take(k);
    double* alpha = sc.take(k);
    double* rr = sc.take(k);
    double* bn2 = sc.take(k);
    double* tol2v = sc.take(k);
    double* rres = sc.take(k);
    int32_t* active = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* first = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* brk = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* go = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* iters = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* cyc = reinterpret_cast<int32_t*>(sc.take(k));
    int32_t* flags = reinterpret_cast<int32_t*>(sc.take(4));
    const int64_t Pk = (int64_t)P * k;
    const dim3 eg(grid_for(Pk)), b256(256);
    const bool mixed = (h.precision == RANN_MIXED);
    const int cap = (mixed && o.restart > 0) ? o.restart : 0;
    const double red2 = mixed ? 1e-8 : 0.0;  // squared per-cycle reduction

    RDD_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t) * 4, h.stream));
    RDD_HIP(hipMemsetAsync(iters, 0, sizeof(int32_t) * k, h.stream));
    RDD_HIP(hipMemsetAsync(active, 0, sizeof(int32_t) * k, h.stream));
    RDD_HIP(hipMemsetAsync(rres, 0, sizeof(double) * k, h.stream));
    RDD_TRY(dot(h, P, k, rhs, rhs, dp, bn2));
    hipLaunchKernelGGL(k_nan_check, eg, b256, 0, h.stream, Pk, rhs, flags + 1);
    if (W0)
        hipLaunchKernelGGL(k_copy, eg, b256, 0, h.stream, Pk, W0, W);
    else
        RDD_HIP(hipMemsetAsync(W, 0, sizeof(double) * Pk, h.stream));
    std::vector<double> bn2h(k), tol2h(k, o.tol * o.tol);
    RDD_TRY(download(h, bn2h.data(), bn2, sizeof(double) * k));
    RDD_HIP(hipStreamSynchronize(h.stream));
    for (int t = 0; t < k; ++t)
        if (!(bn2h[t] > 0.0)) bn2h[t] = 1.0;  // zero right-hand side: solution 0
    RDD_TRY(upload(h, bn2, bn2h.data(), sizeof(double) * k));
    RDD_TRY(upload(h, tol2v, tol2h.data(), sizeof(double) * k));

    // r = rhs - H^T H W from the rows of H, r~ = r; ||r||^2 and, for CGS, rho = <r~, r>
    std::vector<int32_t> goh(k, 1), act(k), brkh(k);
    std::vector<double> rrh(k);
    auto residual = [&]() -> int {
        RDD_TRY(ls_residual(h, Fs, rhs, W, k, y, part, v8, r));
        hipLaunchKernelGGL(k_copy, eg, b256, 0, h.stream, Pk, r, rt);
        hipLaunchKernelGGL(k_dot2_part, dim3(kDotBlocks), b256, 0, h.stream, (int64_t)P, k, r, r, rt, r, dp);
        hipLaunchKernelGGL(k_dot_fin, dim3(1), b256, 0, h.stream, k, kDotBlocks, dp, rr);
        hipLaunchKernelGGL(k_dot_fin, dim3(1), b256, 0, h.stream, k, kDotBlocks, dp + (size_t)kDotBlocks * k, rho);
        RDD_HIP(hipGetLastError());
        RDD_TRY(download(h, rrh.data(), rr, sizeof(double) * k));
        RDD_HIP(hipStreamSynchronize(h.stream));
        return RANN_OK;
    };
    // per-cycle recurrence thresholds (relative to ||rhs||^2)
    std::vector<double> thr(k);
    auto thresholds = [&]() -> int {
        for (int t = 0; t < k; ++t) thr[t] = std::max(tol2h[t], red2 * rrh[t] / bn2h[t]);
        return upload(h, tol2v, thr.data(), sizeof(double) * k);
    };
    RDD_TRY(residual());
    for (int t = 0; t < k; ++t) goh[t] = (rrh[t] > tol2h[t] * bn2h[t]) ? 1 : 0;
    RDD_TRY(thresholds());
    RDD_TRY(upload(h, go, goh.data(), sizeof(int32_t) * k));
    hipLaunchKernelGGL(k_lz_start, dim3(1), b256, 0, h.stream, k, go, active, first, brk, cyc);

    int it = 0, restarts = 0, stalls = 0;
    const int every = std::max(1, o.check_every);
    double best_true = 1e300;
    std::vector<double> tres(k), tbn(k);
    std::vector<int> gaps(k, 0);
    *status = RANN_OK;
    while (true) {
        for (int q = 0; q < every && it < o.maxiter; ++q, ++it) {
            if (cgs) {
                double *u = v1, *pd = v2, *qv = v3, *ph = v4, *vh = v5, *w = v6, *uh = v7, *s = v8;
                hipLaunchKernelGGL(k_cgs_dir, eg, b256, 0, h.stream, Pk, k, rho, rho_old, first, active, r, qv, u,
                                   pd);
                RDD_TRY(launch_precond(h, pd, k, ph, ub));
                RDD_TRY(normal_op(h, ph, k, y, part, vh));
                RDD_TRY(dot(h, P, k, rt, vh, dp, sigma));
                hipLaunchKernelGGL(k_lz_alpha, dim3(1), b256, 0, h.stream, k, rho, sigma, active, brk, alpha);
                hipLaunchKernelGGL(k_cgs_q, eg, b256, 0, h.stream, Pk, k, alpha, active, u, vh, qv, w);
                RDD_TRY(launch_precond(h, w, k, uh, ub));
                RDD_TRY(normal_op(h, uh, k, y, part, s));
                hipLaunchKernelGGL(k_lz_xr, eg, b256, 0, h.stream, Pk, k, alpha, active, uh, s,
                                   (const double*)nullptr, W, r, (double*)nullptr);
                hipLaunchKernelGGL(k_dot2_part, dim3(kDotBlocks), b256, 0, h.stream, (int64_t)P, k, r, r, rt, r,
                                   dp);
                hipLaunchKernelGGL(k_dot_fin, dim3(1), b256, 0, h.stream, k, kDotBlocks, dp, rr);
                hipLaunchKernelGGL(k_dot_fin, dim3(1), b256, 0, h.stream, k, kDotBlocks,
                                   dp + (size_t)kDotBlocks * k, rho_next);
                hipLaunchKernelGGL(k_lz_fin, dim3(1), b256, 0, h.stream, k, cap, rr, bn2, tol2v, rho, rho_old,
                                   rho_next, first, active, brk, cyc, iters, rres, flags);
            } else {
                double *z = v1, *zt = v2, *pd = v3, *pt = v4, *qv = v5, *qt = v6, *tmp = v7;
                RDD_TRY(launch_precond(h, r, k, z, ub));
                RDD_TRY(launch_precond_T(h, rt, k, zt, ub, tmp));
                RDD_TRY(dot(h, P, k, z, rt, dp, rho));
                hipLaunchKernelGGL(k_bicg_dir, eg, b256, 0, h.stream, Pk, k, rho, rho_old, first, active, z, zt,
                                   pd, pt);
                RDD_TRY(normal_op(h, pd, k, y, part, qv));
                RDD_TRY(normal_op(h, pt, k, y, part, qt));
                RDD_TRY(dot(h, P, k, pt, qv, dp, sigma));
                hipLaunchKernelGGL(k_lz_alpha, dim3(1), b256, 0, h.stream, k, rho, sigma, active, brk, alpha);
                hipLaunchKernelGGL(k_lz_xr, eg, b256, 0, h.stream, Pk, k, alpha, active, pd, qv, qt, W, r, rt);
                RDD_TRY(dot(h, P, k, r, r, dp, rr));
                hipLaunchKernelGGL(k_lz_fin, dim3(1), b256, 0, h.stream, k, cap, rr, bn2, tol2v, rho, rho_old,
                                   (const double*)nullptr, first, active, brk, cyc, iters, rres, flags);
            }
        }
        RDD_HIP(hipGetLastError());
        int32_t fl[4];
        RDD_TRY(download(h, act.data(), active, sizeof(int32_t) * k));
        RDD_TRY(download(h, brkh.data(), brk, sizeof(int32_t) * k));
        RDD_TRY(download(h, fl, flags, sizeof(fl)));
        RDD_HIP(hipStreamSynchronize(h.stream));
        if (fl[1]) {
            set_error("NaN or Inf in the Krylov iteration");
            return RANN_ENAN;
        }
        bool any = false;
        for (int t = 0; t < k; ++t) any |= act[t] != 0;
        if (any) {
            if (it >= o.maxiter) {
                *status = RANN_ENOTCONV;
                break;
            }
            continue;
        }
        // every right-hand side stopped: confirm on the recomputed residual
        // (forward: ||H^T (Fs - H W)|| / ||H^T Fs||; adjoint: ||rhs - H^T H W|| / ||rhs||)
        RDD_TRY(residual());
        if (Fs) RDD_TRY(true_residual(h, Fs, W, k, tres.data(), tbn.data()));
        bool again = false;
        double worst = 0.0;
        for (int t = 0; t < k; ++t) {
            const double rel = Fs ? (tbn[t] > 0 ? tres[t] / tbn[t] : 0.0) : std::sqrt(rrh[t] / bn2h[t]);
            worst = std::max(worst, rel);
            goh[t] = rel > o.tol ? 1 : 0;
            if (goh[t]) {
                again = true;
                // the recurrence met tol, the true residual did not.  The
                // restart from the true residual removes the gap that the
                // recurrence accumulated (large intermediate updates drift off
                // through the assembled normal matrix); a gap that comes back
                // on the next cycle is the floor: tighten from then on
                if (!brkh[t] && thr[t] <= tol2h[t] && gaps[t]++ > 0) tol2h[t] *= 0.01;
            }
        }
        if (worst < 0.9 * best_true) {
            best_true = worst;
            stalls = 0;
        } else {
            ++stalls;
        }
        bool floor_hit = false;
        for (int t = 0; t < k; ++t) floor_hit |= tol2h[t] < 1e-60;
        if (!again || it >= o.maxiter || restarts > (mixed ? 1000 : 50) || floor_hit || stalls >= 4) {
            if (again) *status = RANN_ENOTCONV;
            break;
        }
        ++restarts;
        RDD_TRY(thresholds());
        RDD_TRY(upload(h, go, goh.data(), sizeof(int32_t) * k));
        hipLaunchKernelGGL(k_lz_start, dim3(1), b256, 0, h.stream, k, go, active, first, brk, cyc);
    }
    std::vector<int32_t> ith(k);
    std::vector<double> rres_h(k);
    RDD_TRY(download(h, ith.data(), iters, sizeof(int32_t) * k));
    RDD_TRY(download(h, rres_h.data(), rres, sizeof(double) * k));
    RDD_HIP(hipStreamSynchronize(h.stream));
    if (st) {
        if (Fs) {
            RDD_TRY(true_residual(h, Fs, W, k, tres.data(), tbn.data()));
        } else {
            RDD_TRY(residual());
            for (int t = 0; t < k; ++t) {
                tres[t] = std::sqrt(rrh[t]);
                tbn[t] = std::sqrt(bn2h[t]);
            }
        }
        st->iterations = 0;
        st->converged = 0;
        st->max_rel_residual = 0.0;
        for (int t = 0; t < k; ++t) {
            const double rel = tbn[t] > 0 ? tres[t] / tbn[t] : 0.0;
            st->iterations = std::max(st->iterations, ith[t]);
            st->converged += rel <= o.tol ? 1 : 0;
            st->max_rel_residual = std::max(st->max_rel_residual, rel);
            if (st->rel_residual) st->rel_residual[t] = rel;
            if (st->rhs_iterations) st->rhs_iterations[t] = ith[t];
        }
        st->shifts = h.shifts;
    }
    return RANN_OK;
}

// ------------------------------------------------------------------ probes
int coeffs_raw(Handle& h, const double* W, int k, double* c, bool transpose) {
    if (k >= 8) return coeffs_batched(h, W, k, c, transpose);  // batched right-hand sides: matrix cores
    if (!transpose) {
        hipLaunchKernelGGL(k_coeffs, dim3((unsigned)((h.sum_m * k + 15) / 16)), dim3(256), 0, h.stream, h.sum_m, k,
                           h.d_feat_sub, h.d_m_off, h.d_p, h.d_v_off, h.d_col_off, h.d_V, W, c);
    } else {
        hipLaunchKernelGGL(k_coeffs_T, dim3((unsigned)((h.P * k + 15) / 16)), dim3(256), 0, h.stream, h.P, k,
                           h.d_col_sub, h.d_m_off, h.d_m, h.d_p, h.d_v_off, h.d_col_off, h.d_V, W, c);
    }
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

int eval_points(Handle& h, const double* Xq, int64_t M, const double* Lq, const double* W, int k,
                double* U, bool transpose) {
    PointSet ps;
    size_t mark = h.allocs.size();
    auto cleanup = [&]() {
        // free every allocation made for this probe set
        std::vector<void*> mine(h.allocs.begin() + mark, h.allocs.end());
        for (void* p : mine) dev_free(h, p);
    };
    int rc = bin_points(h, Xq, M, ps);
    if (rc == RANN_OK)
        rc = pair_records(h, Xq, 0, nullptr, nullptr, nullptr, nullptr, M, 1.0, true, Lq, ps);
    double* cf = nullptr;
    double* val = nullptr;
    if (rc == RANN_OK) rc = dev_alloc(h, &cf, (size_t)h.sum_m * k);
    if (rc == RANN_OK && !transpose) rc = dev_alloc(h, &val, (size_t)ps.pairs * k);
    if (rc == RANN_OK && (h.deep.n > 0 || k >= 8)) {
        // several hidden layers, or batched right-hand sides: the explicit
        // probe values (once) times the coefficients on the matrix cores
        if (!transpose) {
            rc = coeffs_raw(h, W, k, cf, false);
            if (rc == RANN_OK) rc = eval_explicit(h, ps, cf, k, val, false);
            if (rc == RANN_OK)
                hipLaunchKernelGGL(k_point_sum, dim3(grid_for(M * k)), dim3(256), 0, h.stream, M, k,
                                   ps.d_cover_off, ps.d_cover, val, U);
        } else {
            rc = eval_explicit(h, ps, W, k, cf, true);
            if (rc == RANN_OK) rc = coeffs_raw(h, cf, k, U, true);
        }
    } else if (rc == RANN_OK && !transpose) {
        rc = coeffs_raw(h, W, k, cf, false);
        for (int k0 = 0; rc == RANN_OK && k0 < k;) {
            int kb = kb_for(k - k0);
#define RDD_EV(KBV)                                                                                    \
    hipLaunchKernelGGL((k_eval_pairs<KBV>), dim3((unsigned)((ps.pairs + 15) / 16)), dim3(256), 0, h.stream, h.geo, \
                       ps.pairs, ps.d_pair_sub, ps.d_rec, h.d_m, h.d_m_off, h.d_Rf, h.d_bf, cf, k, k0, \
                       val)
            switch (kb) {
                case 32: RDD_EV(32); break;
                case 16: RDD_EV(16); break;
                case 8: RDD_EV(8); break;
                case 4: RDD_EV(4); break;
                case 2: RDD_EV(2); break;
                default: RDD_EV(1); break;
            }
#undef RDD_EV
            k0 += kb;
        }
        hipLaunchKernelGGL(k_point_sum, dim3(grid_for(M * k)), dim3(256), 0, h.stream, M, k,
                           ps.d_cover_off, ps.d_cover, val, U);
    } else if (rc == RANN_OK) {
        // U holds dW (output), W holds dU (input) in the transposed call.
        // Pair slices per subdomain so that about 1024 workgroups run.
        int max_m = 0;
        for (int j = 0; j < h.geo.J; ++j) max_m = std::max(max_m, h.m[j]);
        const int fgroups = (max_m + 63) / 64;
        const int nz = std::max(1, std::min(16, 1024 / std::max(1, h.geo.J * fgroups)));
        double* cpart = cf;
        if (nz > 1) rc = dev_alloc(h, &cpart, (size_t)nz * h.sum_m * k);
        for (int k0 = 0; rc == RANN_OK && k0 < k;) {
            int kb = kb_for(k - k0);
#define RDD_ET(KBV)                                                                                    \
    hipLaunchKernelGGL((k_eval_T<KBV>), dim3(h.geo.J, fgroups, nz), dim3(256), 0, h.stream, h.geo,      \
                       ps.d_row_off, ps.d_rows, ps.d_rec, h.d_m, h.d_m_off, h.d_Rf, h.d_bf, W, k, k0, \
                       (int64_t)h.sum_m, cpart)
            switch (kb) {
                case 32: RDD_ET(32); break;
                case 16: RDD_ET(16); break;
                case 8: RDD_ET(8); break;
                case 4: RDD_ET(4); break;
                case 2: RDD_ET(2); break;
                default: RDD_ET(1); break;
            }
#undef RDD_ET
            k0 += kb;
        }
        if (rc == RANN_OK && nz > 1)
            hipLaunchKernelGGL(k_eval_T_sum, dim3(grid_for(h.sum_m * k)), dim3(256), 0, h.stream,
                               (int64_t)h.sum_m * k, nz, cpart, cf);
        if (rc == RANN_OK) rc = coeffs_raw(h, cf, k, U, true);
    }
    if (rc == RANN_OK) {
        hipError_t e = hipStreamSynchronize(h.stream);
        if (e != hipSuccess) {
            set_error(std::string("eval: ") + hipGetErrorString(e));
            rc = RANN_EDEVICE;
        }
    }
    cleanup();
    return rc;
}

}  // namespace rdd
