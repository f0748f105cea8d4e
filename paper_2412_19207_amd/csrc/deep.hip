// Subdomain networks with several fixed hidden layers (paper eq. (net)):
// Phi_j = f^{n-1} o ... o f^1 with f^i(y) = tanh(R_i y + b_i), every R_i, b_i
// fixed, R_1 acting on the normalised input.
//
// The inner layers are carried per (point, subdomain) pair in forward mode:
// value, first and pure second derivatives in x (k_deep_chain, one pair per
// 64-lane row of a workgroup, the layer weights read k-major so that the lanes
// of a wave read consecutive words).  What the last layer needs from them is
// reduced to a few vectors of the last inner width w per pair:
//   C0 = z (the last inner output), C1 = sum_q (P1_q d_q z + P2_q d_qq z),
//   C_{2+q} = d_q z,
// because with a_f = R_f . z + b_f, t = tanh a_f and s = 1 - t^2 the chain rule
// gives d_q phi_f = s R_f . d_q z and d_qq phi_f = s R_f . d_qq z
// - 2 t s (R_f . d_q z)^2, so that the operator row entry of feature f with the
// pair coefficients P0, P1, P2 is
//   t (P0 - 2 s sum_q P2_q (R_f . C_{2+q})^2) + s (R_f . C1).
// The contractions with R_j are FP64 matrix-core products over K = w
// (k_deep_rows; the value matrix of the PCA and the probe values take C0 only,
// k_deep_values).  The explicit rows then multiply V_j like any other batched
// product (k_seg_gemm), which also serves the explicit probe evaluation and
// its transpose (eval_explicit, for layered networks and for batched
// right-hand sides of one-layer networks).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace rdd {

namespace {

// forward-mode channels of a layer's output: 0 the value, 1 + 2q its first and
// 2 + 2q its pure second derivative in x_q
constexpr int kCh = 2 * kMaxDim + 1;

// weights of every subdomain's inner layers, k-major: layer i of subdomain j
// at inner[j * stride + lo[i]]: R_i^T (w_{i-1} x w_i) then b_i (w_i)
__global__ void k_pack_inner(DeepNet D, const double* __restrict__ Rin, const double* __restrict__ bin,
                             double* __restrict__ out) {
    const int j = blockIdx.x;
    int64_t rin = 0, bo = 0;
    for (int i = 0; i < D.n; ++i) {
        rin += (int64_t)D.w[i] * D.w[i + 1];
        bo += D.w[i + 1];
    }
    const double* Rj = Rin + (int64_t)j * rin;
    const double* bj = bin + (int64_t)j * bo;
    double* oj = out + (int64_t)j * D.stride;
    for (int i = 0; i < D.n; ++i) {
        const int wi = D.w[i], wo = D.w[i + 1];
        for (int e = threadIdx.x; e < wi * wo; e += blockDim.x) {
            const int k = e / wo, o = e % wo;
            oj[D.lo[i] + e] = Rj[(int64_t)o * wi + k];
        }
        for (int e = threadIdx.x; e < wo; e += blockDim.x) oj[D.lo[i] + wi * wo + e] = bj[e];
        Rj += (int64_t)wi * wo;
        bj += wo;
    }
}

// Inner layers of subdomain j at its pairs blockIdx.y * 4 .. + 3 (one per
// 64-lane row).  kRows: the channels C0, C1, C_{2+q} of every pair
// (row stride (2 + d) w); otherwise C0 alone (row stride w).
template <bool kRows>
__global__ void __launch_bounds__(256) k_deep_chain(Geo g, DeepNet D, const int64_t* __restrict__ row_off,
                                                    const double* __restrict__ rec,
                                                    const double* __restrict__ inner, double* __restrict__ C) {
    __shared__ double act[2][4][kCh][64];
    const int j = blockIdx.x;
    const int64_t n = row_off[j + 1] - row_off[j];
    if ((int64_t)blockIdx.y * 4 >= n) return;  // uniform over the workgroup
    const int slot = threadIdx.x >> 6, o = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.y * 4 + slot;
    const bool live = i < n;
    const int d = g.d;
    const int nch = kRows ? 1 + 2 * d : 1;
    const double* rr = rec + (row_off[j] + (live ? i : 0)) * kPairRec;
    if (o < d) {
        act[0][slot][0][o] = rr[kRecX + o];
        if (kRows)
            for (int q = 0; q < d; ++q) {
                act[0][slot][1 + 2 * q][o] = (q == o) ? g.inv_sigma[q] : 0.0;
                act[0][slot][2 + 2 * q][o] = 0.0;
            }
    }
    __syncthreads();
    const double* Wj = inner + (int64_t)j * D.stride;
    int cur = 0;
    for (int L = 0; L < D.n; ++L) {
        const int win = D.w[L], wout = D.w[L + 1];
        const double* WT = Wj + D.lo[L];
        if (o < wout) {
            double a[kCh];
            a[0] = WT[win * wout + o];
#pragma unroll
            for (int c = 1; c < kCh; ++c) a[c] = 0.0;
            for (int k = 0; k < win; ++k) {
                const double wk = WT[k * wout + o];
#pragma unroll
                for (int c = 0; c < kCh; ++c)
                    if (c < nch) a[c] = fma(wk, act[cur][slot][c][k], a[c]);
            }
            const double t = tanh(a[0]);
            act[cur ^ 1][slot][0][o] = t;
            if (kRows) {
                const double s = 1.0 - t * t;
#pragma unroll
                for (int q = 0; q < kMaxDim; ++q)
                    if (q < d) {
                        const double da = a[1 + 2 * q];
                        act[cur ^ 1][slot][1 + 2 * q][o] = s * da;
                        act[cur ^ 1][slot][2 + 2 * q][o] = s * a[2 + 2 * q] - 2.0 * t * s * da * da;
                    }
            }
        }
        __syncthreads();
        cur ^= 1;
    }
    const int wl = D.w[D.n];
    if (live && o < wl) {
        double* out = C + (row_off[j] + i) * (int64_t)(kRows ? (2 + d) * wl : wl);
        out[o] = act[cur][slot][0][o];
        if (kRows) {
            double u = 0.0;
            for (int q = 0; q < d; ++q) {
                u = fma(rr[kRecP1 + q], act[cur][slot][1 + 2 * q][o], u);
                u = fma(rr[kRecP2 + q], act[cur][slot][2 + 2 * q][o], u);
            }
            out[wl + o] = u;
            for (int q = 0; q < d; ++q) out[(2 + q) * wl + o] = act[cur][slot][1 + 2 * q][o];
        }
    }
}

struct DeepTile { int j, tm, tn, pad; };

// out_j[i][f] = rec_i[slot] tanh(R_f . C0_i + b_f), row-major n_j x m_j at
// out_off[j]: the value matrix Psi_j (slot = window) or the probe values
// (slot = L w_j)
__global__ void __launch_bounds__(256) k_deep_values(const DeepTile* __restrict__ tiles, int wl,
                                                     const int64_t* __restrict__ row_off,
                                                     const double* __restrict__ rec, int slot,
                                                     const int32_t* __restrict__ m,
                                                     const int64_t* __restrict__ m_off,
                                                     const double* __restrict__ Rl,
                                                     const double* __restrict__ bf,
                                                     const double* __restrict__ C0,
                                                     const int64_t* __restrict__ out_off, double* __restrict__ out) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const DeepTile t = tiles[blockIdx.x];
    const int j = t.j, mj = m[j];
    const int64_t n = row_off[j + 1] - row_off[j];
    const int64_t r0 = (int64_t)t.tm * kTM;
    const int f0 = t.tn * kTN;
    TileAcc<double> acc;
    acc.zero();
    tile_gemm<double, false, false>(acc, As, Bs, C0 + row_off[j] * wl, wl, r0, 0, (int)std::min<int64_t>(64, n - r0),
                                    Rl + m_off[j] * wl, wl, f0, 0, std::min(64, mj - f0), wl);
    acc.each([&](int r, int c, double v) {
        const int64_t row = r0 + r;
        const int f = f0 + c;
        if (row < n && f < mj)
            out[out_off[j] + row * mj + f] = rec[(row_off[j] + row) * kPairRec + slot] * tanh(v + bf[m_off[j] + f]);
    });
}

// Ahat_j[i][f] = A[L w_j phi_f](x_i) (interior) or lambda_B (L w_j phi_f)(x_i)
// (boundary; P1 = P2 = 0 there), row-major n_j x m_j at a_off[j], from the
// channels C (row stride (2 + d) wl)
__global__ void __launch_bounds__(256) k_deep_rows(const DeepTile* __restrict__ tiles, int d, int wl,
                                                   const int64_t* __restrict__ row_off,
                                                   const double* __restrict__ rec,
                                                   const int32_t* __restrict__ m,
                                                   const int64_t* __restrict__ m_off,
                                                   const double* __restrict__ Rl, const double* __restrict__ bf,
                                                   const double* __restrict__ C,
                                                   const int64_t* __restrict__ a_off, double* __restrict__ Ahat) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const DeepTile t = tiles[blockIdx.x];
    const int j = t.j, mj = m[j];
    const int64_t n = row_off[j + 1] - row_off[j];
    const int64_t r0 = (int64_t)t.tm * kTM;
    const int f0 = t.tn * kTN;
    const int ld = (2 + d) * wl;
    const double* Cj = C + row_off[j] * ld;
    const double* Rj = Rl + m_off[j] * wl;
    const int amv = (int)std::min<int64_t>(64, n - r0), bmv = std::min(64, mj - f0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    auto row_of = [&](int a, int i) { return wm * 32 + a * 16 + Mfma<double>::out_row(lane, i); };
    auto col_of = [&](int b) { return wn * 32 + b * 16 + (lane & 15); };
    TileAcc<double> acc;
    double th[2][2][4], sq[2][2][4];
    // pre-activations: t = tanh(R_f . z + b_f)
    acc.zero();
    tile_gemm<double, false, false>(acc, As, Bs, Cj, ld, r0, 0, amv, Rj, wl, f0, 0, bmv, wl);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int f = f0 + col_of(b);
            const double bb = (f < mj) ? bf[m_off[j] + f] : 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                th[a][b][i] = tanh(acc.c[a][b][i] + bb);
                sq[a][b][i] = 0.0;
            }
        }
    // sum_q P2_q (R_f . d_q z)^2
    for (int q = 0; q < d; ++q) {
        acc.zero();
        tile_gemm<double, false, false>(acc, As, Bs, Cj, ld, r0, (2 + q) * wl, amv, Rj, wl, f0, 0, bmv, wl);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = r0 + row_of(a, i);
                const double p2 = (row < n) ? rec[(row_off[j] + row) * kPairRec + kRecP2 + q] : 0.0;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double g = acc.c[a][b][i];
                    sq[a][b][i] = fma(p2 * g, g, sq[a][b][i]);
                }
            }
    }
    // R_f . C1 and the row entry
    acc.zero();
    tile_gemm<double, false, false>(acc, As, Bs, Cj, ld, r0, wl, amv, Rj, wl, f0, 0, bmv, wl);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = r0 + row_of(a, i);
            if (row >= n) continue;
            const double P0 = rec[(row_off[j] + row) * kPairRec + kRecP0];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int f = f0 + col_of(b);
                if (f >= mj) continue;
                const double tt = th[a][b][i], s = 1.0 - tt * tt;
                Ahat[a_off[j] + row * mj + f] = tt * (P0 - 2.0 * s * sq[a][b][i]) + s * acc.c[a][b][i];
            }
        }
}

// A batch of row-major products C_s = op(A_s) B_s: op(A_s) M x K (A_s stored
// M x K, or K x M when kAT), B_s K x N, C_s M x N; an FP32 copy of C when C32
struct SegDesc {
    int64_t a, b, c;
    int M, K, N, lda, ldb, ldc;
};

template <bool kAT>
__global__ void __launch_bounds__(256) k_seg_gemm(const DeepTile* __restrict__ tiles, const SegDesc* __restrict__ sd,
                                                  const double* __restrict__ A, const double* __restrict__ B,
                                                  double* __restrict__ Cout, float* __restrict__ C32) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const DeepTile t = tiles[blockIdx.x];
    const SegDesc s = sd[t.j];
    const int r0 = t.tm * kTM, c0 = t.tn * kTN;
    TileAcc<double> acc;
    acc.zero();
    if (kAT)
        tile_gemm<double, true, true>(acc, As, Bs, A + s.a, s.lda, 0, r0, std::min(64, s.M - r0), B + s.b, s.ldb, 0,
                                      c0, std::min(64, s.N - c0), s.K);
    else
        tile_gemm<double, false, true>(acc, As, Bs, A + s.a, s.lda, r0, 0, std::min(64, s.M - r0), B + s.b, s.ldb,
                                       0, c0, std::min(64, s.N - c0), s.K);
    acc.each([&](int r, int c, double v) {
        const int gr = r0 + r, gc = c0 + c;
        if (gr < s.M && gc < s.N) {
            const int64_t e = s.c + (int64_t)gr * s.ldc + gc;
            Cout[e] = v;
            if (C32) C32[e] = (float)v;
        }
    });
}

__global__ void k_gather_pairs(int64_t pairs, int k, const int32_t* __restrict__ rows, const double* __restrict__ src,
                               double* __restrict__ dst) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= pairs * k) return;
    const int64_t pid = e / k;
    dst[e] = src[(int64_t)rows[pid] * k + (e % k)];
}

unsigned grid1(int64_t n) { return (unsigned)((n + 255) / 256); }

int launch_seg(Handle& h, const std::vector<SegDesc>& segs, bool at, const double* A, const double* B, double* C,
               float* C32) {
    std::vector<DeepTile> tiles;
    for (int s = 0; s < (int)segs.size(); ++s) {
        const int nm = (segs[s].M + kTM - 1) / kTM, nn = (segs[s].N + kTN - 1) / kTN;
        if (segs[s].K <= 0) continue;
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b < nn; ++b) tiles.push_back({s, a, b, 0});
    }
    if (tiles.empty()) return RANN_OK;
    DeepTile* d_t = nullptr;
    SegDesc* d_s = nullptr;
    RDD_TRY(dev_alloc(h, &d_t, tiles.size()));
    RDD_TRY(dev_alloc(h, &d_s, segs.size()));
    RDD_TRY(upload(h, d_t, tiles.data(), sizeof(DeepTile) * tiles.size()));
    RDD_TRY(upload(h, d_s, segs.data(), sizeof(SegDesc) * segs.size()));
    if (at)
        hipLaunchKernelGGL(k_seg_gemm<true>, dim3((unsigned)tiles.size()), dim3(256), 0, h.stream, d_t, d_s, A, B, C,
                           C32);
    else
        hipLaunchKernelGGL(k_seg_gemm<false>, dim3((unsigned)tiles.size()), dim3(256), 0, h.stream, d_t, d_s, A, B, C,
                           C32);
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, d_t);
    dev_free(h, d_s);
    return RANN_OK;
}

// tiles over the n_j x m_j value or row matrices of a point set
std::vector<DeepTile> feature_tiles(const Handle& h, const PointSet& ps) {
    std::vector<DeepTile> tiles;
    for (int j = 0; j < h.geo.J; ++j) {
        const int64_t n = ps.row_off[j + 1] - ps.row_off[j];
        const int nm = (int)((n + kTM - 1) / kTM), nn = (h.m[j] + kTN - 1) / kTN;
        for (int a = 0; a < nm; ++a)
            for (int b = 0; b < nn; ++b) tiles.push_back({j, a, b, 0});
    }
    return tiles;
}

int64_t max_rows(const Handle& h, const PointSet& ps) {
    int64_t mx = 0;
    for (int j = 0; j < h.geo.J; ++j) mx = std::max(mx, ps.row_off[j + 1] - ps.row_off[j]);
    return mx;
}

}  // namespace

int deep_setup(Handle& h, const rann_dd_desc* ds) {
    DeepNet& D = h.deep;
    D = DeepNet{};
    if (ds->n_inner == 0) return RANN_OK;
    if (ds->n_inner < 0 || ds->n_inner > kMaxInner) {
        set_error("n_inner must be 0..3");
        return RANN_EINVAL;
    }
    if (!ds->R_inner || !ds->b_inner) {
        set_error("R_inner and b_inner are required when n_inner > 0");
        return RANN_EINVAL;
    }
    D.n = ds->n_inner;
    D.w[0] = h.geo.d;
    int off = 0;
    for (int i = 0; i < D.n; ++i) {
        const int w = ds->inner_w[i];
        if (w < 1 || w > kMaxInnerWidth) {
            set_error("inner widths must be 1..64");
            return RANN_EINVAL;
        }
        D.w[i + 1] = w;
        D.lo[i] = off;
        off += D.w[i] * w + w;
    }
    D.stride = off;
    const int J = h.geo.J;
    RDD_TRY(dev_alloc(h, &h.d_inner, (size_t)J * D.stride));
    hipLaunchKernelGGL(k_pack_inner, dim3(J), dim3(256), 0, h.stream, D, ds->R_inner, ds->b_inner, h.d_inner);
    RDD_HIP(hipGetLastError());
    const int wl = D.w[D.n];
    RDD_TRY(dev_alloc(h, &h.d_Rl, (size_t)h.sum_m * wl));
    RDD_HIP(hipMemcpyAsync(h.d_Rl, ds->R, sizeof(double) * h.sum_m * wl, hipMemcpyDeviceToDevice, h.stream));
    return RANN_OK;
}

int deep_values(Handle& h, const PointSet& ps, int slot, const int64_t* d_out_off, double* out) {
    const DeepNet& D = h.deep;
    const int wl = D.w[D.n];
    const int64_t mx = max_rows(h, ps);
    if (mx == 0) return RANN_OK;
    double* C0 = nullptr;
    RDD_TRY(dev_alloc(h, &C0, (size_t)ps.pairs * wl));
    KTimer kt_(h.stream, "k_deep_values");
    hipLaunchKernelGGL(k_deep_chain<false>, dim3(h.geo.J, (unsigned)((mx + 3) / 4)), dim3(256), 0, h.stream, h.geo,
                       D, ps.d_row_off, ps.d_rec, h.d_inner, C0);
    RDD_HIP(hipGetLastError());
    std::vector<DeepTile> tiles = feature_tiles(h, ps);
    DeepTile* d_t = nullptr;
    RDD_TRY(dev_alloc(h, &d_t, tiles.size()));
    RDD_TRY(upload(h, d_t, tiles.data(), sizeof(DeepTile) * tiles.size()));
    hipLaunchKernelGGL(k_deep_values, dim3((unsigned)tiles.size()), dim3(256), 0, h.stream, d_t, wl,
                       ps.d_row_off, ps.d_rec, slot, h.d_m, h.d_m_off, h.d_Rl, h.d_bf, C0, d_out_off, out);
    RDD_HIP(hipGetLastError());
    kt_.stop();
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, d_t);
    dev_free(h, C0);
    return RANN_OK;
}

int deep_feature_rows(Handle& h) {
    const DeepNet& D = h.deep;
    const int wl = D.w[D.n], d = h.geo.d, J = h.geo.J;
    const PointSet& ps = h.pts;
    const int64_t mx = max_rows(h, ps);
    if (mx == 0) return RANN_OK;
    double* C = nullptr;
    RDD_TRY(dev_alloc(h, &C, (size_t)ps.pairs * (2 + d) * wl));
    KTimer kt_(h.stream, "k_deep_rows");
    hipLaunchKernelGGL(k_deep_chain<true>, dim3(J, (unsigned)((mx + 3) / 4)), dim3(256), 0, h.stream, h.geo, D,
                       ps.d_row_off, ps.d_rec, h.d_inner, C);
    RDD_HIP(hipGetLastError());
    std::vector<int64_t> a_off(J + 1, 0);
    for (int j = 0; j < J; ++j) a_off[j + 1] = a_off[j] + (ps.row_off[j + 1] - ps.row_off[j]) * h.m[j];
    int64_t* d_a_off = nullptr;
    double* Ahat = nullptr;
    RDD_TRY(dev_alloc(h, &d_a_off, (size_t)J + 1));
    RDD_TRY(dev_alloc(h, &Ahat, (size_t)std::max<int64_t>(1, a_off[J])));
    RDD_TRY(upload(h, d_a_off, a_off.data(), sizeof(int64_t) * (J + 1)));
    std::vector<DeepTile> tiles = feature_tiles(h, ps);
    DeepTile* d_t = nullptr;
    RDD_TRY(dev_alloc(h, &d_t, tiles.size()));
    RDD_TRY(upload(h, d_t, tiles.data(), sizeof(DeepTile) * tiles.size()));
    hipLaunchKernelGGL(k_deep_rows, dim3((unsigned)tiles.size()), dim3(256), 0, h.stream, d_t, d, wl,
                       ps.d_row_off, ps.d_rec, h.d_m, h.d_m_off, h.d_Rl, h.d_bf, C, d_a_off, Ahat);
    RDD_HIP(hipGetLastError());
    kt_.stop();
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, d_t);
    dev_free(h, C);
    // H_j = Ahat_j V_j (and its FP32 copy when the mixed path keeps one)
    std::vector<SegDesc> segs(J);
    for (int j = 0; j < J; ++j) {
        const int64_t n = ps.row_off[j + 1] - ps.row_off[j];
        segs[j] = SegDesc{a_off[j], h.v_off[j], h.h_off[j], (int)n, h.m[j], h.p[j], h.m[j], h.p[j], h.p[j]};
    }
    KTimer kt2_(h.stream, "k_seg_gemm");
    RDD_TRY(launch_seg(h, segs, false, Ahat, h.d_V, h.d_H, h.d_H32));
    kt2_.stop();
    dev_free(h, Ahat);
    dev_free(h, d_a_off);
    return RANN_OK;
}

int coeffs_batched(Handle& h, const double* x, int k, double* y, bool transpose) {
    const int J = h.geo.J;
    std::vector<SegDesc> segs(J);
    bool empty = false;
    for (int j = 0; j < J; ++j) {
        empty |= h.p[j] == 0;
        if (!transpose)  // c_j (m_j x k) = V_j (m_j x p_j) W_j (p_j x k)
            segs[j] = SegDesc{h.v_off[j], h.col_off[j] * k, h.m_off[j] * k, h.m[j], h.p[j], k, h.p[j], k, k};
        else  // W_j (p_j x k) = V_j^T c_j, V_j read as stored (m_j x p_j)
            segs[j] = SegDesc{h.v_off[j], h.m_off[j] * k, h.col_off[j] * k, h.p[j], h.m[j], k, h.p[j], k, k};
    }
    if (empty && !transpose) RDD_HIP(hipMemsetAsync(y, 0, sizeof(double) * h.sum_m * k, h.stream));
    return launch_seg(h, segs, transpose, h.d_V, x, y, nullptr);
}

int eval_explicit(Handle& h, const PointSet& ps, const double* x, int k, double* y, bool transpose) {
    const int J = h.geo.J;
    std::vector<int64_t> t_off(J + 1, 0);
    for (int j = 0; j < J; ++j) t_off[j + 1] = t_off[j] + (ps.row_off[j + 1] - ps.row_off[j]) * h.m[j];
    int64_t* d_t_off = nullptr;
    double* T = nullptr;
    RDD_TRY(dev_alloc(h, &d_t_off, (size_t)J + 1));
    RDD_TRY(dev_alloc(h, &T, (size_t)std::max<int64_t>(1, t_off[J])));
    RDD_TRY(upload(h, d_t_off, t_off.data(), sizeof(int64_t) * (J + 1)));
    // T_j[i][f] = L(x_i) w_j(x_i) phi_f(x_i) at the probe pairs
    RDD_TRY(values_matrix(h, ps, kRecP0, d_t_off, T));
    std::vector<SegDesc> segs(J);
    int rc = RANN_OK;
    if (!transpose) {
        // per-pair values y[pair][t] = T_j[pair] . x_j[:, t] (x: raw coefficients, sum_m x k)
        for (int j = 0; j < J; ++j) {
            const int64_t n = ps.row_off[j + 1] - ps.row_off[j];
            segs[j] = SegDesc{t_off[j], h.m_off[j] * k, ps.row_off[j] * k, (int)n, h.m[j], k, h.m[j], k, k};
        }
        rc = launch_seg(h, segs, false, T, x, y, nullptr);
    } else {
        // y[f][t] = sum over the pairs of j of T_j[pair][f] x[row(pair)][t] (x: per point, M x k)
        double* xg = nullptr;
        rc = dev_alloc(h, &xg, (size_t)std::max<int64_t>(1, ps.pairs * k));
        if (rc == RANN_OK && ps.pairs > 0) {
            hipLaunchKernelGGL(k_gather_pairs, dim3(grid1(ps.pairs * k)), dim3(256), 0, h.stream, ps.pairs, k,
                               ps.d_rows, x, xg);
            if (hipGetLastError() != hipSuccess) {
                set_error("k_gather_pairs launch failed");
                rc = RANN_EDEVICE;
            }
        }
        if (rc == RANN_OK) {
            for (int j = 0; j < J; ++j) {
                const int64_t n = ps.row_off[j + 1] - ps.row_off[j];
                segs[j] = SegDesc{t_off[j], ps.row_off[j] * k, h.m_off[j] * k, h.m[j], (int)n, k, h.m[j], k, k};
            }
            // rows of subdomains without probe pairs stay zero
            RDD_HIP(hipMemsetAsync(y, 0, sizeof(double) * h.sum_m * k, h.stream));
            rc = launch_seg(h, segs, true, T, xg, y, nullptr);
        }
        if (xg) dev_free(h, xg);
    }
    dev_free(h, T);
    dev_free(h, d_t_off);
    return rc;
}

}  // namespace rdd
