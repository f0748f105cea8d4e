// Matrix-core GEMMs of the set-up phase.
//
//  * k_psi, k_pca_gram: G_j = Psi_j^T Psi_j, Psi_j[i,k] = w_j(x_i) tanh(z_k(x_i)),
//                  the value matrix of the PCA step (paper Sec. 4); Psi is
//                  evaluated once into scratch memory, then multiplied by tiles.
//  * k_feat_rows : H_j = A_j V_j with A_j[i,k] = A[L w_j phi_k](x_i) generated
//                  in the GEMM prologue from the pair coefficients (eqs. (sum),
//                  (system_new)) and the tanh values the PCA's value matrices
//                  kept (computed again when the PCA did not run); FP64
//                  output plus an FP32 copy in the mixed path.
//                  (Networks with several hidden layers take deep.hip instead,
//                  for both products.)
//  * k_local_gram: Gram blocks G_jk = H_j^T H_k over the rows the two supports
//                  share, the pieces of the Schwarz blocks A_i = R_i H^T H R_i^T
//                  (Sec. 3); FP64, or FP32 with FP32 accumulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "mfma.h"

namespace rdd {

namespace {

struct GramTile { int j, tm, tn, pad; };

__device__ __forceinline__ double feature_z(const double* Rk, double bk, const double* xt, int d) {
    double z = bk;
    for (int i = 0; i < d; ++i) z = fma(Rk[i], xt[i], z);
    return z;
}

// Psi_j[i][f] = rec_i[slot] tanh(z_f(x_i)), row-major n_j x m_j, for the 16
// pair rows of workgroup (j, chunk); each value is computed once.  slot: the
// window (value matrix of the PCA) or L w_j (probe values).  With T, the
// tanh values themselves too (kept for the operator rows).
__global__ void __launch_bounds__(256) k_psi(Geo g, const int64_t* __restrict__ row_off,
                                             const double* __restrict__ rec, int slot, const int32_t* __restrict__ m,
                                             const int64_t* __restrict__ m_off, const double* __restrict__ Rf,
                                             const double* __restrict__ bf, const int64_t* __restrict__ psi_off,
                                             double* __restrict__ Psi, double* __restrict__ T) {
    const int j = blockIdx.x, mj = m[j];
    const int64_t n = row_off[j + 1] - row_off[j];
    const int64_t r0 = (int64_t)blockIdx.y * 16;
    if (r0 >= n) return;
    const double* rj = rec + row_off[j] * kPairRec;
    double* out = Psi + psi_off[j];
    for (int e = threadIdx.x; e < 16 * mj; e += 256) {
        const int64_t i = r0 + e / mj;
        const int f = e % mj;
        if (i < n) {
            double xt[kMaxDim] = {0, 0, 0, 0};
            for (int q = 0; q < g.d; ++q) xt[q] = rj[i * kPairRec + kRecX + q];
            const double w = rj[i * kPairRec + slot];
            const int64_t gf = m_off[j] + f;
            const double th = tanh(feature_z(Rf + gf * 4, bf[gf], xt, g.d));
            out[i * mj + f] = w * th;
            if (T) T[psi_off[j] + i * mj + f] = th;
        }
    }
}

// tile (a, b), b <= a, of G_j = Psi_j^T Psi_j (both triangles written)
__global__ void __launch_bounds__(256) k_pca_gram(const GramTile* __restrict__ tiles,
                                                  const int64_t* __restrict__ row_off,
                                                  const int32_t* __restrict__ m,
                                                  const int64_t* __restrict__ psi_off,
                                                  const double* __restrict__ Psi,
                                                  const int64_t* __restrict__ g_off,
                                                  double* __restrict__ G) {
    __shared__ double As[kBK][kTM + kPad];
    __shared__ double Bs[kBK][kTN + kPad];
    const GramTile t = tiles[blockIdx.x];
    const int j = t.j, mj = m[j];
    const int n = (int)(row_off[j + 1] - row_off[j]);
    const double* Pj = Psi + psi_off[j];
    const int64_t a0 = (int64_t)t.tm * kTM, b0 = (int64_t)t.tn * kTN;
    const int av = (int)((mj - a0) < kTM ? (mj - a0) : kTM), bv = (int)((mj - b0) < kTN ? (mj - b0) : kTN);
    TileAcc<double> acc;
    acc.zero();
    tile_gemm<double, true, true>(acc, As, Bs, Pj, mj, 0, a0, av, Pj, mj, 0, b0, bv, n);
    const bool diag = (t.tm == t.tn);
    double* Gj = G + g_off[j];
    acc.each([&](int r, int c, double v) {
        const int64_t gr = a0 + r, gc = b0 + c;
        if (gr < mj && gc < mj) {
            if (!diag || gr >= gc) {
                Gj[gr * mj + gc] = v;
                Gj[gc * mj + gr] = v;
            }
        }
    });
}

__global__ void __launch_bounds__(256) k_feat_rows(Geo g, const GramTile* __restrict__ tiles,
                                                   const int64_t* __restrict__ row_off,
                                                   const double* __restrict__ rec,
                                                   const int32_t* __restrict__ m,
                                                   const int64_t* __restrict__ m_off,
                                                   const double* __restrict__ Rf,
                                                   const double* __restrict__ bf,
                                                   const int32_t* __restrict__ p,
                                                   const int64_t* __restrict__ v_off,
                                                   const double* __restrict__ V,
                                                   const int64_t* __restrict__ h_off,
                                                   double* __restrict__ H, float* __restrict__ H32,
                                                   const double* __restrict__ T,
                                                   const int64_t* __restrict__ t_off) {
    __shared__ double As[kTK][kTM + kPad];
    __shared__ double Bs[kTK][kTN + kPad];
    const GramTile t = tiles[blockIdx.x];
    const int j = t.j, mj = m[j], pj = p[j];
    const int64_t n = row_off[j + 1] - row_off[j];
    const int mm = threadIdx.x & 63, kq = threadIdx.x >> 6;
    const int64_t row = (int64_t)t.tm * kTM + mm;
    // pair coefficients of this thread's row, kept in registers over the K loop
    double xt[kMaxDim] = {0, 0, 0, 0}, P0 = 0.0, P1[kMaxDim] = {0, 0, 0, 0},
           P2[kMaxDim] = {0, 0, 0, 0};
    const bool rv = row < n;
    if (rv) {
        const double* rr = rec + (row_off[j] + row) * kPairRec;
        for (int q = 0; q < g.d; ++q) {
            xt[q] = rr[kRecX + q];
            P1[q] = rr[kRecP1 + q];
            P2[q] = rr[kRecP2 + q];
        }
        P0 = rr[kRecP0];
    }
    const int bk = threadIdx.x >> 4, bc4 = (threadIdx.x & 15) * 4;
    const double* Vj = V + v_off[j];
    TileAcc<double> acc;
    acc.zero();
    for (int k0 = 0; k0 < mj; k0 += kTK) {
        for (int e = 0; e < 4; ++e) {
            int f = k0 + kq * 4 + e;
            double v = 0.0;
            if (rv && f < mj) {
                int64_t gf = m_off[j] + f;
                const double* Rk = Rf + gf * 4;
                // the tanh values the PCA kept, when it ran
                const double th = T ? T[t_off[j] + row * mj + f] : tanh(feature_z(Rk, bf[gf], xt, g.d));
                double s = 1.0 - th * th;
                double g1 = 0.0, g2 = 0.0;
                for (int q = 0; q < g.d; ++q) {
                    double rho = Rk[q] * g.inv_sigma[q];
                    g1 = fma(P1[q], rho, g1);
                    g2 = fma(P2[q], rho * rho, g2);
                }
                v = th * (P0 - 2.0 * g2 * s) + g1 * s;
            }
            As[kq * 4 + e][mm] = v;
        }
        for (int e = 0; e < 4; ++e) {
            int f = k0 + bk, c = t.tn * kTN + bc4 + e;
            Bs[bk][bc4 + e] = (f < mj && c < pj) ? Vj[(int64_t)f * pj + c] : 0.0;
        }
        __syncthreads();
        acc.step(As, Bs);
        __syncthreads();
    }
    double* Hj = H + h_off[j];
    float* Hj32 = H32 ? H32 + h_off[j] : nullptr;
    acc.each([&](int r, int c, double v) {
        int64_t gr = (int64_t)t.tm * kTM + r;
        int gc = t.tn * kTN + c;
        if (gr < n && gc < pj) {
            Hj[gr * pj + gc] = v;
            if (Hj32) Hj32[gr * pj + gc] = (float)v;
        }
    });
}

struct PairBlock {
    int j, k;          // subdomains (j <= k)
    int64_t isect;     // offset into the intersection lists (-1 when j == k)
    int64_t len;       // shared rows
    int64_t g_off;     // offset of the p_j x p_k block in the block store
};

struct LocalTile { int blk, tm, tn, pad; };

template <class T>
__global__ void __launch_bounds__(256) k_local_gram(const LocalTile* __restrict__ tiles,
                                                    const PairBlock* __restrict__ blocks,
                                                    const int32_t* __restrict__ loc_j,
                                                    const int32_t* __restrict__ loc_k,
                                                    const int32_t* __restrict__ p,
                                                    const int64_t* __restrict__ h_off,
                                                    const T* __restrict__ H, T* __restrict__ Gout) {
    __shared__ T As[kTK][kTM + kPad];
    __shared__ T Bs[kTK][kTN + kPad];
    const LocalTile t = tiles[blockIdx.x];
    const PairBlock B = blocks[t.blk];
    const int pj = p[B.j], pk = p[B.k];
    const T* Hj = H + h_off[B.j];
    const T* Hk = H + h_off[B.k];
    const int kk = threadIdx.x >> 4, c4 = (threadIdx.x & 15) * 4;
    TileAcc<T> acc;
    acc.zero();
    for (int64_t i0 = 0; i0 < B.len; i0 += kTK) {
        const int64_t i = i0 + kk;
        int64_t rj = -1, rk = -1;
        if (i < B.len) {
            if (B.isect < 0) {
                rj = i;
                rk = i;
            } else {
                rj = loc_j[B.isect + i];
                rk = loc_k[B.isect + i];
            }
        }
        for (int e = 0; e < 4; ++e) {
            int ca = t.tm * kTM + c4 + e, cb = t.tn * kTN + c4 + e;
            As[kk][c4 + e] = (rj >= 0 && ca < pj) ? Hj[rj * pj + ca] : T(0);
            Bs[kk][c4 + e] = (rk >= 0 && cb < pk) ? Hk[rk * pk + cb] : T(0);
        }
        __syncthreads();
        acc.step(As, Bs);
        __syncthreads();
    }
    T* G = Gout + B.g_off;
    acc.each([&](int r, int c, T v) {
        int gr = t.tm * kTM + r, gc = t.tn * kTN + c;
        if (gr < pj && gc < pk) G[(int64_t)gr * pk + gc] = v;
    });
}

// rows shared by the supports of j and k: positions in S_j and in S_k
template <bool kFill>
__global__ void __launch_bounds__(256) k_intersect(const PairBlock* __restrict__ blocks,
                                                   const int64_t* __restrict__ row_off,
                                                   const int32_t* __restrict__ rows,
                                                   int64_t* __restrict__ count,
                                                   int32_t* __restrict__ loc_j,
                                                   int32_t* __restrict__ loc_k) {
    const PairBlock B = blocks[blockIdx.x];
    if (B.isect < 0 && kFill) return;
    const int32_t* Sj = rows + row_off[B.j];
    const int32_t* Sk = rows + row_off[B.k];
    const int64_t nj = row_off[B.j + 1] - row_off[B.j], nk = row_off[B.k + 1] - row_off[B.k];
    __shared__ int wave_cnt[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t base = 0;
    for (int64_t a0 = 0; a0 < nj; a0 += 256) {
        int64_t a = a0 + threadIdx.x;
        int64_t pos = -1;
        if (a < nj) {
            int32_t v = Sj[a];
            int64_t lo = 0, hi = nk;
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (Sk[mid] < v) lo = mid + 1; else hi = mid;
            }
            if (lo < nk && Sk[lo] == v) pos = lo;
        }
        bool in = pos >= 0;
        uint64_t mask = __ballot(in);
        if (lane == 0) wave_cnt[wave] = __popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
        for (int w = 0; w < 4; ++w) {
            before += (w < wave) ? wave_cnt[w] : 0;
            total += wave_cnt[w];
        }
        if (kFill && in) {
            uint64_t lower = (lane == 0) ? 0ull : (mask & ((~0ull) >> (64 - lane)));
            int64_t o = B.isect + base + before + __popcll(lower);
            loc_j[o] = (int32_t)a;
            loc_k[o] = (int32_t)pos;
        }
        base += total;
        __syncthreads();
    }
    if (!kFill && threadIdx.x == 0) count[blockIdx.x] = base;
}

// assemble A_i from the Gram block store (exactly symmetric by construction)
template <class T>
__global__ void __launch_bounds__(256) k_assemble_A(int J, const int32_t* __restrict__ sten_off,
                                                    const int32_t* __restrict__ sten,
                                                    const int32_t* __restrict__ pair_of,
                                                    const PairBlock* __restrict__ blocks,
                                                    const int32_t* __restrict__ p,
                                                    const int64_t* __restrict__ f_off,
                                                    const T* __restrict__ Gs, T* __restrict__ A) {
    // blockIdx.x = block i, blockIdx.y = stencil pair (a, b) packed as a * 32 + b
    const int i = blockIdx.x;
    const int ns = sten_off[i + 1] - sten_off[i];
    const int a = blockIdx.y / 32, b = blockIdx.y % 32;
    if (a >= ns || b >= ns) return;
    int64_t q = 0, oa = 0, ob = 0;
    for (int s = 0; s < ns; ++s) {
        int js = sten[sten_off[i] + s];
        if (s == a) oa = q;
        if (s == b) ob = q;
        q += p[js];
    }
    const int ja = sten[sten_off[i] + a], jb = sten[sten_off[i] + b];
    const int pa = p[ja], pb = p[jb];
    const int pid = pair_of[sten_off[i] * 32 + a * 32 + b];  // index into blocks or -1
    T* Ai = A + f_off[i];
    for (int64_t e = threadIdx.x; e < (int64_t)pa * pb; e += blockDim.x) {
        int r = (int)(e / pb), c = (int)(e % pb);
        T v = T(0);
        if (pid >= 0) {
            const PairBlock B = blocks[pid];
            const T* G = Gs + B.g_off;
            if (ja == jb) {
                int hi = r > c ? r : c, lo = r > c ? c : r;
                v = G[(int64_t)hi * pb + lo];
            } else if (ja < jb) {
                v = G[(int64_t)r * pb + c];
            } else {
                v = G[(int64_t)c * pa + r];
            }
        }
        Ai[(oa + r) * q + ob + c] = v;
    }
}

// block row j of the normal matrix N = H^T H as a dense p_j x Q_j slab whose
// columns are those of the subdomains meeting j (ascending): block (j, k) is
// H_j^T H_k over the shared rows, read from the Gram block store
__global__ void __launch_bounds__(256) k_assemble_slab(const int32_t* __restrict__ nbr_off,
                                                       const int32_t* __restrict__ nbr,
                                                       const int32_t* __restrict__ nbr_pid,
                                                       const int64_t* __restrict__ nbr_col,
                                                       const PairBlock* __restrict__ blocks,
                                                       const int32_t* __restrict__ p,
                                                       const int64_t* __restrict__ N_off,
                                                       const int64_t* __restrict__ N_coff,
                                                       const double* __restrict__ Gs,
                                                       double* __restrict__ N) {
    const int j = blockIdx.x;
    const int a = nbr_off[j] + blockIdx.y;
    if (a >= nbr_off[j + 1]) return;
    const int k = nbr[a];
    const int pj = p[j], pk = p[k];
    const int64_t Q = N_coff[j + 1] - N_coff[j];
    const int64_t c0 = nbr_col[a];
    const PairBlock B = blocks[nbr_pid[a]];
    const double* G = Gs + B.g_off;
    double* Nj = N + N_off[j];
    for (int64_t e = threadIdx.x; e < (int64_t)pj * pk; e += blockDim.x) {
        const int r = (int)(e / pk), c = (int)(e % pk);
        double v;
        if (j == k) {
            const int hi = r > c ? r : c, lo = r > c ? c : r;
            v = G[(int64_t)hi * pk + lo];
        } else if (j < k) {
            v = G[(int64_t)r * pk + c];
        } else {
            v = G[(int64_t)c * pj + r];
        }
        Nj[r * Q + c0 + c] = v;
    }
}

// the 16 rows of slab task (j, r0) in matrix-core operand order: quad c of
// columns 4c .. 4c + 3 as 64 doubles, entry 16 g + r = N_j[r0 + r][4c + g]
// (zero past the slab)
__global__ void __launch_bounds__(256) k_tile_slab(const int2* __restrict__ tasks, const int32_t* __restrict__ p,
                                                   const int64_t* __restrict__ N_off,
                                                   const int64_t* __restrict__ N_coff,
                                                   const double* __restrict__ N, const int64_t* __restrict__ Nt_off,
                                                   double* __restrict__ Nt) {
    const int2 tk = tasks[blockIdx.x];
    const int j = tk.x, r0 = tk.y;
    const int pj = p[j];
    const int64_t Q = N_coff[j + 1] - N_coff[j];
    const int64_t nq4 = (Q + 3) / 4;
    double* out = Nt + Nt_off[j] + (int64_t)(r0 / 16) * nq4 * 64;
    const double* Nj = N + N_off[j];
    for (int64_t e = threadIdx.x; e < nq4 * 64; e += 256) {
        const int64_t c = 4 * (e / 64) + (e % 64) / 16;
        const int r = r0 + (int)(e % 16);
        out[e] = (r < pj && c < Q) ? Nj[(int64_t)r * Q + c] : 0.0;
    }
}

}  // namespace

int values_matrix(Handle& h, const PointSet& ps, int slot, const int64_t* d_out_off, double* out, double* T) {
    if (h.deep.n > 0) return deep_values(h, ps, slot, d_out_off, out);
    int64_t max_n = 0;
    for (int j = 0; j < h.geo.J; ++j) max_n = std::max(max_n, ps.row_off[j + 1] - ps.row_off[j]);
    if (max_n > 0)
        hipLaunchKernelGGL(k_psi, dim3(h.geo.J, (unsigned)((max_n + 15) / 16)), dim3(256), 0, h.stream, h.geo,
                           ps.d_row_off, ps.d_rec, slot, h.d_m, h.d_m_off, h.d_Rf, h.d_bf, d_out_off, out, T);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

int pca_gram(Handle& h, double* G, const int64_t* g_off_host, const int64_t* d_g_off) {
    (void)g_off_host;
    std::vector<GramTile> tiles;
    for (int j = 0; j < h.geo.J; ++j) {
        int nt = (h.m[j] + kTM - 1) / kTM;
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b <= a; ++b) tiles.push_back({j, a, b, 0});
    }
    GramTile* d_t = nullptr;
    RDD_TRY(dev_alloc(h, &d_t, tiles.size()));
    RDD_TRY(upload(h, d_t, tiles.data(), sizeof(GramTile) * tiles.size()));
    // the value matrices Psi_j, computed once and kept for the Gram tiles
    const int J = h.geo.J;
    std::vector<int64_t> psi_off(J + 1, 0);
    int64_t max_n = 0;
    for (int j = 0; j < J; ++j) {
        const int64_t n = h.pts.row_off[j + 1] - h.pts.row_off[j];
        psi_off[j + 1] = psi_off[j] + n * h.m[j];
        max_n = std::max(max_n, n);
    }
    int64_t* d_psi_off = nullptr;
    double* d_psi = nullptr;
    RDD_TRY(dev_alloc(h, &d_psi_off, (size_t)J + 1));
    RDD_TRY(dev_alloc(h, &d_psi, (size_t)std::max<int64_t>(1, psi_off[J])));
    RDD_TRY(upload(h, d_psi_off, psi_off.data(), sizeof(int64_t) * (J + 1)));
    (void)max_n;
    // one hidden layer: the tanh values are kept for the operator rows
    if (h.deep.n == 0 && !h.d_T) {
        RDD_TRY(dev_alloc(h, &h.d_T_off, (size_t)J + 1));
        RDD_TRY(dev_alloc(h, &h.d_T, (size_t)std::max<int64_t>(1, psi_off[J])));
        RDD_TRY(upload(h, h.d_T_off, psi_off.data(), sizeof(int64_t) * (J + 1)));
    }
    KTimer kt_(h.stream, "k_pca_gram");
    RDD_TRY(values_matrix(h, h.pts, kRecW, d_psi_off, d_psi, h.d_T));
    hipLaunchKernelGGL(k_pca_gram, dim3((unsigned)tiles.size()), dim3(256), 0, h.stream, d_t, h.pts.d_row_off,
                       h.d_m, d_psi_off, d_psi, d_g_off, G);
    kt_.stop();
    dev_free(h, d_psi);
    dev_free(h, d_psi_off);
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, d_t);
    return RANN_OK;
}

int feature_rows(Handle& h) {
    if (h.deep.n > 0) return deep_feature_rows(h);
    std::vector<GramTile> tiles;
    for (int j = 0; j < h.geo.J; ++j) {
        int64_t n = h.pts.row_off[j + 1] - h.pts.row_off[j];
        int ntm = (int)((n + kTM - 1) / kTM), ntn = (h.p[j] + kTN - 1) / kTN;
        for (int a = 0; a < ntm; ++a)
            for (int b = 0; b < ntn; ++b) tiles.push_back({j, a, b, 0});
    }
    if (tiles.empty()) return RANN_OK;
    GramTile* d_t = nullptr;
    RDD_TRY(dev_alloc(h, &d_t, tiles.size()));
    RDD_TRY(upload(h, d_t, tiles.data(), sizeof(GramTile) * tiles.size()));
    KTimer kt_(h.stream, "k_feat_rows");
    hipLaunchKernelGGL(k_feat_rows, dim3((unsigned)tiles.size()), dim3(256), 0, h.stream, h.geo, d_t,
                       h.pts.d_row_off, h.pts.d_rec, h.d_m, h.d_m_off, h.d_Rf, h.d_bf, h.d_p,
                       h.d_v_off, h.d_V, h.d_h_off, h.d_H, h.d_H32, h.d_T, h.d_T_off);
    kt_.stop();
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, d_t);
    if (h.d_T) {  // the tanh values of the PCA serve these rows only
        dev_free(h, h.d_T);
        dev_free(h, h.d_T_off);
        h.d_T = nullptr;
        h.d_T_off = nullptr;
    }
    return RANN_OK;
}

// Gram blocks H_j^T H_k of every pair of subdomains whose supports meet
// (kept in the handle until release_gram) and the block rows of the normal
// matrix N = H^T H as dense slabs (kept for the Krylov iterations).
int normal_blocks(Handle& h) {
    const int J = h.geo.J;
    auto centre = [&](int j, int i) {
        int c = j;
        for (int q = 0; q < i; ++q) c /= h.geo.l[q];
        c %= h.geo.l[i];
        return c;
    };
    std::vector<std::vector<double>> cen(J, std::vector<double>(h.geo.d));
    {
        std::vector<double> mu_all(h.geo.mu_off[h.geo.d - 1] + h.geo.l[h.geo.d - 1]);
        RDD_TRY(download(h, mu_all.data(), h.d_mu, sizeof(double) * mu_all.size()));
        for (int j = 0; j < J; ++j)
            for (int i = 0; i < h.geo.d; ++i) cen[j][i] = mu_all[h.geo.mu_off[i] + centre(j, i)];
    }
    auto meet = [&](int j, int k) {
        for (int i = 0; i < h.geo.d; ++i)
            if (!(std::fabs(cen[j][i] - cen[k][i]) < 2.0 * h.geo.sigma[i])) return false;
        return true;
    };
    // every meeting pair (j <= k), and the sorted neighbour list of each j
    std::vector<PairBlock> blocks;
    h.pair_tab.assign(J, {});
    std::vector<std::vector<int>> nbrs(J);
    for (int j = 0; j < J; ++j)
        for (int k = j; k < J; ++k) {
            if (!meet(j, k)) continue;
            h.pair_tab[j].push_back({k, (int)blocks.size()});
            blocks.push_back(PairBlock{j, k, j == k ? -1 : 0, 0, 0});
            nbrs[j].push_back(k);
            if (k != j) nbrs[k].push_back(j);
        }
    for (auto& v : nbrs) std::sort(v.begin(), v.end());
    const int nb = (int)blocks.size();
    PairBlock* d_blocks = nullptr;
    RDD_TRY(dev_alloc(h, &d_blocks, nb));
    for (auto& B : blocks) B.len = (B.isect < 0) ? (h.pts.row_off[B.j + 1] - h.pts.row_off[B.j]) : 0;
    RDD_TRY(upload(h, d_blocks, blocks.data(), sizeof(PairBlock) * nb));
    int64_t* d_cnt = nullptr;
    RDD_TRY(dev_alloc(h, &d_cnt, nb));
    hipLaunchKernelGGL((k_intersect<false>), dim3(nb), dim3(256), 0, h.stream, d_blocks,
                       h.pts.d_row_off, h.pts.d_rows, d_cnt, nullptr, nullptr);
    RDD_HIP(hipGetLastError());
    std::vector<int64_t> cnt(nb);
    RDD_TRY(download(h, cnt.data(), d_cnt, sizeof(int64_t) * nb));
    int64_t tot_isect = 0, tot_g = 0;
    for (int b = 0; b < nb; ++b) {
        auto& B = blocks[b];
        if (B.isect >= 0) {
            B.isect = tot_isect;
            B.len = cnt[b];
            tot_isect += cnt[b];
        }
        B.g_off = tot_g;
        tot_g += (int64_t)h.p[B.j] * h.p[B.k];
    }
    RDD_TRY(upload(h, d_blocks, blocks.data(), sizeof(PairBlock) * nb));
    int32_t *d_lj = nullptr, *d_lk = nullptr;
    RDD_TRY(dev_alloc(h, &d_lj, (size_t)tot_isect));
    RDD_TRY(dev_alloc(h, &d_lk, (size_t)tot_isect));
    hipLaunchKernelGGL((k_intersect<true>), dim3(nb), dim3(256), 0, h.stream, d_blocks,
                       h.pts.d_row_off, h.pts.d_rows, nullptr, d_lj, d_lk);
    RDD_HIP(hipGetLastError());
    double* d_G = nullptr;
    RDD_TRY(dev_alloc(h, &d_G, (size_t)tot_g));
    std::vector<LocalTile> tiles;
    for (int b = 0; b < nb; ++b) {
        int ta = (h.p[blocks[b].j] + kTM - 1) / kTM, tb = (h.p[blocks[b].k] + kTN - 1) / kTN;
        for (int x = 0; x < ta; ++x)
            for (int y = 0; y < tb; ++y) tiles.push_back({b, x, y, 0});
    }
    LocalTile* d_tiles = nullptr;
    RDD_TRY(dev_alloc(h, &d_tiles, tiles.size()));
    RDD_TRY(upload(h, d_tiles, tiles.data(), sizeof(LocalTile) * tiles.size()));
    if (!tiles.empty()) {
        KTimer kt_(h.stream, "k_local_gram");
        hipLaunchKernelGGL((k_local_gram<double>), dim3((unsigned)tiles.size()), dim3(256), 0, h.stream,
                           d_tiles, d_blocks, d_lj, d_lk, h.d_p, h.d_h_off, h.d_H, d_G);
        kt_.stop();
        RDD_HIP(hipGetLastError());
        if (h.d_H32) {  // the same Gram blocks from the FP32 rows on the FP32 matrix cores
            RDD_TRY(dev_alloc(h, &h.d_G32, (size_t)tot_g));
            KTimer kt32_(h.stream, "k_local_gram32");
            hipLaunchKernelGGL((k_local_gram<float>), dim3((unsigned)tiles.size()), dim3(256), 0, h.stream,
                               d_tiles, d_blocks, d_lj, d_lk, h.d_p, h.d_h_off, h.d_H32, h.d_G32);
            kt32_.stop();
            RDD_HIP(hipGetLastError());
        }
    }
    // slabs of N: block row j, columns of nbrs[j] in ascending order
    std::vector<int32_t> nbr_off(J + 1, 0), nbr_flat, nbr_pid;
    std::vector<int64_t> nbr_col;
    h.N_off.assign(J + 1, 0);
    h.N_coff.assign(J + 1, 0);
    std::vector<int32_t> N_cols;
    int max_nbr = 0;
    auto find_pair = [&](int j, int k) -> int {
        for (auto& e : h.pair_tab[j])
            if (e.first == k) return e.second;
        return -1;
    };
    for (int j = 0; j < J; ++j) {
        int64_t q = 0;
        for (int k : nbrs[j]) {
            nbr_flat.push_back(k);
            nbr_pid.push_back(find_pair(std::min(j, k), std::max(j, k)));
            nbr_col.push_back(q);
            for (int c = 0; c < h.p[k]; ++c) N_cols.push_back((int32_t)(h.col_off[k] + c));
            q += h.p[k];
        }
        nbr_off[j + 1] = (int32_t)nbr_flat.size();
        max_nbr = std::max(max_nbr, (int)nbrs[j].size());
        h.N_coff[j + 1] = h.N_coff[j] + q;
        h.N_off[j + 1] = h.N_off[j] + (int64_t)h.p[j] * q;
    }
    h.N_elems = h.N_off[J];
    int32_t *d_no = nullptr, *d_nf = nullptr, *d_np = nullptr;
    int64_t* d_nc = nullptr;
    RDD_TRY(dev_alloc(h, &d_no, nbr_off.size()));
    RDD_TRY(dev_alloc(h, &d_nf, nbr_flat.size()));
    RDD_TRY(dev_alloc(h, &d_np, nbr_pid.size()));
    RDD_TRY(dev_alloc(h, &d_nc, nbr_col.size()));
    RDD_TRY(dev_alloc(h, &h.d_N, (size_t)h.N_elems));
    RDD_TRY(dev_alloc(h, &h.d_N_off, (size_t)J + 1));
    RDD_TRY(dev_alloc(h, &h.d_N_coff, (size_t)J + 1));
    RDD_TRY(dev_alloc(h, &h.d_N_cols, N_cols.size()));
    RDD_TRY(upload(h, d_no, nbr_off.data(), sizeof(int32_t) * nbr_off.size()));
    RDD_TRY(upload(h, d_nf, nbr_flat.data(), sizeof(int32_t) * nbr_flat.size()));
    RDD_TRY(upload(h, d_np, nbr_pid.data(), sizeof(int32_t) * nbr_pid.size()));
    RDD_TRY(upload(h, d_nc, nbr_col.data(), sizeof(int64_t) * nbr_col.size()));
    RDD_TRY(upload(h, h.d_N_off, h.N_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(upload(h, h.d_N_coff, h.N_coff.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(upload(h, h.d_N_cols, N_cols.data(), sizeof(int32_t) * N_cols.size()));
    if (max_nbr > 0)
        hipLaunchKernelGGL(k_assemble_slab, dim3(J, max_nbr), dim3(256), 0, h.stream, d_no, d_nf, d_np,
                           d_nc, d_blocks, h.d_p, h.d_N_off, h.d_N_coff, d_G, h.d_N);
    RDD_HIP(hipGetLastError());
    // slab row tasks of the product kernel
    std::vector<int2> tasks;
    for (int j = 0; j < J; ++j)
        for (int r = 0; r < h.p[j]; r += kSlabRows) tasks.push_back(make_int2(j, r));
    h.n_slab_tasks = (int64_t)tasks.size();
    RDD_TRY(dev_alloc(h, &h.d_slab_tasks, tasks.size()));
    RDD_TRY(upload(h, h.d_slab_tasks, tasks.data(), sizeof(int2) * tasks.size()));
    // the slabs in matrix-core operand order (the batched product reads them)
    {
        std::vector<int64_t> nt_off(J + 1, 0);
        for (int j = 0; j < J; ++j) {
            const int64_t nq4 = (h.N_coff[j + 1] - h.N_coff[j] + 3) / 4;
            nt_off[j + 1] = nt_off[j] + (int64_t)((h.p[j] + kSlabRows - 1) / kSlabRows) * nq4 * 64;
        }
        h.Nt_elems = nt_off[J];
        RDD_TRY(dev_alloc(h, &h.d_Nt_off, (size_t)J + 1));
        RDD_TRY(dev_alloc(h, &h.d_Nt, (size_t)std::max<int64_t>(1, h.Nt_elems)));
        RDD_TRY(upload(h, h.d_Nt_off, nt_off.data(), sizeof(int64_t) * (J + 1)));
        if (h.n_slab_tasks)
            hipLaunchKernelGGL(k_tile_slab, dim3((unsigned)h.n_slab_tasks), dim3(256), 0, h.stream, h.d_slab_tasks,
                               h.d_p, h.d_N_off, h.d_N_coff, h.d_N, h.d_Nt_off, h.d_Nt);
        RDD_HIP(hipGetLastError());
    }
    RDD_HIP(hipStreamSynchronize(h.stream));
    for (void* ptr : {(void*)d_cnt, (void*)d_lj, (void*)d_lk, (void*)d_tiles, (void*)d_no, (void*)d_nf,
                      (void*)d_np, (void*)d_nc})
        dev_free(h, ptr);
    h.d_G = d_G;
    h.d_pair_blocks = d_blocks;
    return RANN_OK;
}

void release_gram(Handle& h) {
    dev_free(h, h.d_G);
    dev_free(h, h.d_pair_blocks);
    if (h.d_G32) dev_free(h, h.d_G32);
    if (h.d_H32) dev_free(h, h.d_H32);
    h.d_G = nullptr;
    h.d_G32 = nullptr;
    h.d_H32 = nullptr;
    h.d_pair_blocks = nullptr;
    h.pair_tab.clear();
}

// The Schwarz blocks A_i (device, q_i x q_i each) from the Gram block store
template <class T>
int local_blocks(Handle& h, const T* H, T* A_out) {
    (void)H;
    const int J = h.geo.J;
    auto find_pair = [&](int j, int k) -> int {
        for (auto& e : h.pair_tab[j])
            if (e.first == k) return e.second;
        return -1;
    };
    std::vector<int32_t> sten_off(J + 1, 0), sten_flat, pair_of;
    int max_ns = 0;
    for (int i = 0; i < J; ++i) {
        sten_off[i + 1] = sten_off[i] + (int32_t)h.sten[i].size();
        max_ns = std::max(max_ns, (int)h.sten[i].size());
        for (int s : h.sten[i]) sten_flat.push_back(s);
    }
    if (max_ns > 32) {
        set_error("stencil larger than 32 subdomains");
        return RANN_EINVAL;
    }
    pair_of.assign((size_t)sten_off[J] * 32, -1);
    for (int i = 0; i < J; ++i) {
        const auto& s = h.sten[i];
        for (size_t a = 0; a < s.size(); ++a)
            for (size_t b = 0; b < s.size(); ++b) {
                int j = std::min(s[a], s[b]), k = std::max(s[a], s[b]);
                pair_of[(size_t)sten_off[i] * 32 + a * 32 + b] = find_pair(j, k);
            }
    }
    int32_t *d_so = nullptr, *d_sf = nullptr, *d_po = nullptr;
    RDD_TRY(dev_alloc(h, &d_so, sten_off.size()));
    RDD_TRY(dev_alloc(h, &d_sf, sten_flat.size()));
    RDD_TRY(dev_alloc(h, &d_po, pair_of.size()));
    RDD_TRY(upload(h, d_so, sten_off.data(), sizeof(int32_t) * sten_off.size()));
    RDD_TRY(upload(h, d_sf, sten_flat.data(), sizeof(int32_t) * sten_flat.size()));
    RDD_TRY(upload(h, d_po, pair_of.data(), sizeof(int32_t) * pair_of.size()));
    const T* Gs = nullptr;
    if constexpr (sizeof(T) == sizeof(float)) Gs = reinterpret_cast<const T*>(h.d_G32);
    else Gs = reinterpret_cast<const T*>(h.d_G);
    hipLaunchKernelGGL((k_assemble_A<T>), dim3(J, max_ns * 32), dim3(256), 0, h.stream, J, d_so, d_sf,
                       d_po, static_cast<const PairBlock*>(h.d_pair_blocks), h.d_p, h.d_f_off, Gs, A_out);
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    for (void* ptr : {(void*)d_so, (void*)d_sf, (void*)d_po}) dev_free(h, ptr);
    return RANN_OK;
}

template int local_blocks<double>(Handle&, const double*, double*);
template int local_blocks<float>(Handle&, const float*, float*);

}  // namespace rdd
