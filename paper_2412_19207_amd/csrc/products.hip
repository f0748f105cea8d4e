// Products with the block-sparse collocation matrix H = [H_1 .. H_J] (paper
// Sec. 3 remark: domain decomposition makes H block sparse).
//
// Work is cut into chunks of up to kChunk consecutive rows of one block H_j
// (stored row-major, n_j x p_j, blocks concatenated), so one workgroup reads
// one contiguous piece of H:
//   * y = H x : per chunk, t_pair = H_j[row] . x_j (x_j staged in LDS, one
//               wave per row, lanes stride the row), then y[r] = sum of the
//               pair values of row r (the rows two supports share get two);
//   * x = H^T y: per chunk, column partial sums with the threads laid out as
//               (row group, column) so consecutive threads read consecutive
//               addresses, then a fixed-order sum over the chunks of a block.
// No floating-point atomics: every sum has a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "cg_step.h"
#include "mfma.h"

namespace rdd {

namespace {

constexpr int kChunk = 128;
constexpr int kHxKB = 8;    // right-hand sides per pass of H x (x_j staged in LDS)
constexpr int kHTKB = 8;    // right-hand sides per pass of H^T y

template <int KB>
__global__ void __launch_bounds__(256) k_Hx_chunk(const int32_t* __restrict__ chunk_sub,
                                                  const int64_t* __restrict__ chunk_off,
                                                  const int64_t* __restrict__ row_off,
                                                  const int32_t* __restrict__ p,
                                                  const int64_t* __restrict__ h_off,
                                                  const int64_t* __restrict__ col_off,
                                                  const double* __restrict__ H,
                                                  const double* __restrict__ x, int k, int k0,
                                                  double* __restrict__ tpair) {
    __shared__ double xs[KB][kMaxWidth];
    const int ch = blockIdx.x;
    const int j = chunk_sub[ch];
    const int pj = p[j];
    const int64_t n = row_off[j + 1] - row_off[j];
    const int64_t r0 = (ch - chunk_off[j]) * (int64_t)kChunk;
    const int64_t r1 = (r0 + kChunk < n) ? r0 + kChunk : n;
    const double* xj = x + col_off[j] * k + k0;
    for (int e = threadIdx.x; e < pj * KB; e += 256) {
        const int c = e / KB, t = e % KB;
        xs[t][c] = xj[(int64_t)c * k + t];
    }
    __syncthreads();
    // L lanes per row (L = 8 .. 64 from the block width), 64 / L rows per wave
    const int L = pj > 256 ? 64 : pj > 128 ? 32 : pj > 64 ? 16 : 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / L, l = lane % L, rpw = 64 / L;
    const double* Hj = H + h_off[j];
    for (int64_t rb = r0 + (int64_t)wave * rpw; rb < r1; rb += 4 * rpw) {
        const int64_t r = rb + sub;
        double acc[KB];
        for (int t = 0; t < KB; ++t) acc[t] = 0.0;
        if (r < r1) {
            const double* Hr = Hj + r * pj;
            for (int c = l; c < pj; c += L) {
                const double hv = Hr[c];
                for (int t = 0; t < KB; ++t) acc[t] = fma(hv, xs[t][c], acc[t]);
            }
        }
        for (int t = 0; t < KB; ++t)
            for (int off = L >> 1; off > 0; off >>= 1) acc[t] += __shfl_xor(acc[t], off);
        if (l == 0 && r < r1) {
            double* o = tpair + (row_off[j] + r) * k + k0;
            for (int t = 0; t < KB; ++t) o[t] = acc[t];
        }
    }
}

// y[r][t] = sum over the pairs of point r (ascending subdomain order)
__global__ void k_pair_to_rows(int64_t n, int k, const int64_t* __restrict__ cover_off,
                               const int64_t* __restrict__ cover, const double* __restrict__ tpair,
                               double* __restrict__ y) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * k) return;
    const int64_t r = idx / k;
    const int t = (int)(idx % k);
    double s = 0.0;
    for (int64_t c = cover_off[r]; c < cover_off[r + 1]; ++c) s += tpair[cover[c] * k + t];
    y[idx] = s;
}

template <int KB>
__global__ void __launch_bounds__(256) k_HTy_chunk(const int32_t* __restrict__ chunk_sub,
                                                   const int64_t* __restrict__ chunk_off,
                                                   const int64_t* __restrict__ part_off,
                                                   const int64_t* __restrict__ row_off,
                                                   const int32_t* __restrict__ rows,
                                                   const int32_t* __restrict__ p,
                                                   const int64_t* __restrict__ h_off,
                                                   const double* __restrict__ H,
                                                   const double* __restrict__ y, int k, int k0,
                                                   double* __restrict__ part) {
    __shared__ double ys[kChunk][KB];
    __shared__ double red[256 * KB];
    const int ch = blockIdx.x;
    const int j = chunk_sub[ch];
    const int pj = p[j];
    const int64_t n = row_off[j + 1] - row_off[j];
    const int64_t r0 = (ch - chunk_off[j]) * (int64_t)kChunk;
    const int nr = (int)((r0 + kChunk < n) ? kChunk : n - r0);
    const int32_t* Sj = rows + row_off[j];
    for (int e = threadIdx.x; e < nr * KB; e += 256) {
        const int rr = e / KB, t = e % KB;
        ys[rr][t] = y[(int64_t)Sj[r0 + rr] * k + k0 + t];
    }
    __syncthreads();
    const double* Hj = H + h_off[j] + r0 * pj;
    for (int c0 = 0; c0 < pj; c0 += 256) {
        const int pc = (pj - c0 < 256) ? pj - c0 : 256;   // columns in this pass
        const int G = 256 / pc;                            // row groups
        const int g = threadIdx.x / pc, c = threadIdx.x % pc;
        double acc[KB];
        for (int t = 0; t < KB; ++t) acc[t] = 0.0;
        if (g < G) {
            for (int rr = g; rr < nr; rr += G) {
                const double hv = Hj[(int64_t)rr * pj + c0 + c];
                for (int t = 0; t < KB; ++t) acc[t] = fma(hv, ys[rr][t], acc[t]);
            }
        }
        for (int t = 0; t < KB; ++t) red[t * 256 + threadIdx.x] = acc[t];
        __syncthreads();
        if (threadIdx.x < pc) {
            double* o = part + (part_off[ch] + c0 + threadIdx.x) * k + k0;
            for (int t = 0; t < KB; ++t) {
                double s = 0.0;
                for (int gg = 0; gg < G; ++gg) s += red[t * 256 + gg * pc + threadIdx.x];
                o[t] = s;
            }
        }
        __syncthreads();
    }
}


// s = N x from the slabs of N = H^T H: workgroup = kSlabRows rows of block row
// j, each wave kSlabRows / 4 rows (loaded together), x gathered through the
// slab's column list and staged in LDS; optional per-workgroup <x, s>.  UPD:
// x is the direction p_new = z + beta p_prev of the previous iteration.
template <int KB, bool UPD>
__global__ void __launch_bounds__(256) k_nrm_slab(const int2* __restrict__ tasks,
                                                  const int32_t* __restrict__ p,
                                                  const int64_t* __restrict__ col_off,
                                                  const int64_t* __restrict__ N_off,
                                                  const int64_t* __restrict__ N_coff,
                                                  const int32_t* __restrict__ N_cols,
                                                  const double* __restrict__ N,
                                                  const double* __restrict__ x, int k, int k0,
                                                  double* __restrict__ s, double* __restrict__ part,
                                                  PUpd pu) {
    constexpr int kXS = 4096 / KB;      // staged columns per pass
    constexpr int kRW = kSlabRows / 4;  // rows per wave
    __shared__ double xs[kXS][KB];
    __shared__ double red[4][KB];
    __shared__ double beta_s[KB], rz_s[KB], rr_s[KB], psh[256];
    __shared__ int act_s[KB];
    if (UPD) pupd_begin(pu, k, k0, KB, beta_s, act_s, rz_s, rr_s, psh);
    const int2 tk = tasks[xcd_task(blockIdx.x, gridDim.x)];
    const int j = tk.x, r0 = tk.y;
    const int pj = p[j];
    const int64_t Q = N_coff[j + 1] - N_coff[j];
    const int32_t* cols = N_cols + N_coff[j];
    const double* Nj = N + N_off[j];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc[kRW][KB];
#pragma unroll
    for (int u = 0; u < kRW; ++u)
#pragma unroll
        for (int t = 0; t < KB; ++t) acc[u][t] = 0.0;
    int nrow = 0;  // rows of this wave that exist
#pragma unroll
    for (int u = 0; u < kRW; ++u)
        if (r0 + wave + 4 * u < pj) nrow = u + 1;
    for (int64_t c0 = 0; c0 < Q; c0 += kXS) {
        const int nc = (Q - c0 < kXS) ? (int)(Q - c0) : kXS;
        __syncthreads();
        // 4 entries per thread and round, so that their loads are in flight
        // together (entries past the pass re-read its last one and are dropped)
        const double* xa_src = UPD ? pu.pprev : x;
        for (int e0 = threadIdx.x; e0 < nc * KB; e0 += 4 * 256) {
            int64_t gi[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = min(e0 + v * 256, nc * KB - 1);
                gi[v] = (int64_t)cols[c0 + e / KB] * k + k0 + e % KB;
            }
            double xa[4], xb[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                xa[v] = xa_src[gi[v]];
                xb[v] = UPD ? pu.z[gi[v]] : 0.0;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = e0 + v * 256;
                if (e < nc * KB) {
                    const int t = e % KB;
                    xs[e / KB][t] = (UPD && act_s[t]) ? fma(beta_s[t], xa[v], xb[v]) : xa[v];
                }
            }
        }
        __syncthreads();
        const double* Nr = Nj + (int64_t)(r0 + wave) * Q + c0;
        for (int cb = lane; cb < nc; cb += 4 * 64) {
            double nv[4][kRW];
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int u = 0; u < kRW; ++u) {
                    const int c = cb + v * 64;
                    nv[v][u] = (u < nrow && c < nc) ? Nr[(int64_t)4 * u * Q + c] : 0.0;
                }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = cb + v * 64;
                if (c < nc)
#pragma unroll
                    for (int u = 0; u < kRW; ++u)
#pragma unroll
                        for (int t = 0; t < KB; ++t) acc[u][t] = fma(nv[v][u], xs[c][t], acc[u][t]);
            }
        }
    }
    // the wave's kRW x KB results: lane l < kRW KB owns row u = l / KB,
    // right-hand side t = l % KB; its entry of x (or of p_prev and z) is
    // loaded before the sums are formed
    static_assert(kRW * KB <= 64 && (KB & (KB - 1)) == 0, "one result per lane");
    const int lu = lane / KB, lt = lane % KB;
    const bool own = lane < kRW * KB && lu < nrow;
    const int64_t go = (col_off[j] + (own ? r0 + wave + 4 * lu : pj - 1)) * k + k0 + lt;
    const double oa = UPD ? pu.pprev[go] : x[go];
    const double ob = UPD ? pu.z[go] : 0.0;
    double mine = 0.0;
#pragma unroll
    for (int u = 0; u < kRW; ++u) {
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            for (int off = 32; off > 0; off >>= 1) acc[u][t] += __shfl_xor(acc[u][t], off);
            if (lane == u * KB + t) mine = acc[u][t];
        }
    }
    double d = 0.0;
    if (own) {
        s[go] = mine;
        double xv = oa;
        if (UPD) {
            xv = act_s[lt] ? fma(beta_s[lt], oa, ob) : oa;
            pu.pcur[go] = xv;
        }
        d = mine * xv;
    }
    // lanes t, t + KB, t + 2 KB, t + 3 KB hold the kRW rows of right-hand side t
    for (int off = KB; off < kRW * KB; off <<= 1) d += __shfl_xor(d, off);
    if (part) {
        if (lane < KB) red[wave][lane] = d;
        __syncthreads();
        if (threadIdx.x < KB) {
            const int t = threadIdx.x;
            part[(int64_t)blockIdx.x * k + k0 + t] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
        }
    }
}

// Batched right-hand sides (KC = 16 or 32): the 16 slab rows of a task times
// x (Q x KC) on the FP64 matrix cores, from the slab in MFMA operand order
// (Nt: per task, quad c of columns 4c .. 4c + 3 as 64 consecutive doubles,
// entry l = 16 g + lr holding row r0 + lr, column 4c + g, zero past the slab),
// so that each A operand is one coalesced 512-byte load.  Wave w takes the
// 64-column sweeps w, w + 4, ...; at step u of a sweep lane (lr, g) supplies
// quad c0 / 4 + u of the A operand and the x row of column c0 + 4u + g (B
// operand, read straight from global memory: within the task each x row feeds
// one wave only).  The 4 waves' sums meet in LDS.  The loads that do not need
// the direction update (column indices, A operands, the own rows' entries)
// are issued before its partial sums are added, so that the chain of
// dependent memory rounds is: those loads, then the x rows (all of a sweep's
// in flight together: absent columns load row 0 and are discarded).  UPD: x
// is the direction p_new = z + beta p_prev of the previous iteration.  P2
// (KC = 32, k even): lane lr of the B operand takes the right-hand sides 2 lr
// and 2 lr + 1 (one 16-byte load for both column blocks) instead of lr and
// lr + 16.
template <int KC, bool UPD, bool P2>
__global__ void __launch_bounds__(256, 2) k_nrm_mfma(const int2* __restrict__ tasks,
                                                  const int32_t* __restrict__ p,
                                                  const int64_t* __restrict__ col_off,
                                                  const int64_t* __restrict__ Nt_off,
                                                  const int64_t* __restrict__ N_coff,
                                                  const int32_t* __restrict__ N_cols,
                                                  const double* __restrict__ Nt,
                                                  const double* __restrict__ x, int k, int k0,
                                                  double* __restrict__ s, double* __restrict__ part,
                                                  PUpd pu) {
    constexpr int NB = KC / 16;
    constexpr int kOwn = 16 * KC / 256;  // own-row entries per thread
    static_assert(kSlabRows == 16, "one 16-row MFMA block per task");
    static_assert(!P2 || NB == 2, "paired columns need two column blocks");
    // right-hand side (within the chunk) of column block nb, lane lr
    auto colof = [](int nb, int lr) { return P2 ? NB * lr + nb : 16 * nb + lr; };
    __shared__ double red[4][16][KC + 1];
    __shared__ double dsh[256];
    __shared__ double beta_s[KC], rz_s[KC], rr_s[KC];
    __shared__ int act_s[KC];
    const int2 tk = tasks[xcd_task(blockIdx.x, gridDim.x)];
    const int j = tk.x, r0 = tk.y;
    const int pj = p[j];
    const int64_t Q = N_coff[j + 1] - N_coff[j];
    const int64_t nq4 = (Q + 3) / 4;
    const int32_t* cols = N_cols + N_coff[j];
    const double* At = Nt + Nt_off[j] + (int64_t)(r0 / 16) * nq4 * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    // first round: column indices (this sweep and the next), A operands and
    // the own rows' entries of x (or of p_prev and z)
    int32_t ci[16], cn[16];
    double av[16];
    const int64_t c00 = 64 * w;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int64_t c = c00 + 4 * u + g;
        ci[u] = c < Q ? cols[c] : -1;
        const int64_t c2 = c + 256;
        cn[u] = c2 < Q ? cols[c2] : -1;
        av[u] = (c00 / 4 + u < nq4) ? At[(c00 / 4 + u) * 64 + lane] : 0.0;
    }
    const int t = threadIdx.x % KC;
    double bet[NB];
    bool act[NB];
    if (UPD) {
        pupd_begin(pu, k, k0, KC, beta_s, act_s, rz_s, rr_s, dsh);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            bet[nb] = beta_s[colof(nb, lr)];
            act[nb] = act_s[colof(nb, lr)] != 0;
        }
    }
    const double* xa_src = UPD ? pu.pprev : x;
    typedef Mfma<double>::acc_t acc_t;
    acc_t acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[nb][e] = 0.0;
    for (int64_t c0 = c00; c0 < Q; c0 += 256) {
        // the x rows of this sweep (absent columns: bit u of live clear)
        uint32_t live = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) live |= (ci[u] >= 0 ? 1u : 0u) << u;
        double bv[16][NB], zb[UPD ? 16 : 1][NB];
        if constexpr (P2) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int64_t gi = (int64_t)(ci[u] >= 0 ? ci[u] : 0) * k + k0 + 2 * lr;
                const double2 va = *reinterpret_cast<const double2*>(xa_src + gi);
                bv[u][0] = va.x;
                bv[u][1] = va.y;
                if (UPD) {
                    const double2 vz = *reinterpret_cast<const double2*>(pu.z + gi);
                    zb[u][0] = vz.x;
                    zb[u][1] = vz.y;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < 16; ++u)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const int64_t gi = (int64_t)(ci[u] >= 0 ? ci[u] : 0) * k + k0 + 16 * nb + lr;
                    bv[u][nb] = xa_src[gi];
                    if (UPD) zb[u][nb] = pu.z[gi];
                }
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                double b = bv[u][nb];
                if (UPD && act[nb]) b = fma(bet[nb], b, zb[u][nb]);
                bv[u][nb] = ((live >> u) & 1u) ? b : 0.0;
            }
#pragma unroll
        for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[nb] = Mfma<double>::mma(av[u], bv[u][nb], acc[nb]);
        if (c0 + 256 < Q) {  // the next sweep's A operands and the column indices after it
            const int64_t q0 = (c0 + 256) / 4;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                av[u] = (q0 + u < nq4) ? At[(q0 + u) * 64 + lane] : 0.0;
                ci[u] = cn[u];
                const int64_t c = c0 + 512 + 4 * u + g;
                cn[u] = c < Q ? cols[c] : -1;
            }
        }
    }
    // the own rows' entries of x (or of p_prev and z), loaded while the
    // matrix-core chain runs
    double own_a[kOwn], own_b[kOwn];
#pragma unroll
    for (int v = 0; v < kOwn; ++v) {
        const int rr = threadIdx.x / KC + (256 / KC) * v;
        const int64_t gi = (col_off[j] + (r0 + rr < pj ? r0 + rr : pj - 1)) * k + k0 + t;
        own_a[v] = UPD ? pu.pprev[gi] : x[gi];
        own_b[v] = UPD ? pu.z[gi] : 0.0;
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[w][Mfma<double>::out_row(lane, e)][colof(nb, lr)] = acc[nb][e];
    __syncthreads();
    double dotv = 0.0;
#pragma unroll
    for (int v = 0; v < kOwn; ++v) {
        const int rr = threadIdx.x / KC + (256 / KC) * v;
        const double val = (red[0][rr][t] + red[1][rr][t]) + (red[2][rr][t] + red[3][rr][t]);
        if (r0 + rr < pj) {
            const int64_t gi = (col_off[j] + r0 + rr) * k + k0 + t;
            s[gi] = val;
            double xv = own_a[v];
            if (UPD) {
                xv = act_s[t] ? fma(beta_s[t], own_a[v], own_b[v]) : own_a[v];
                pu.pcur[gi] = xv;
            }
            dotv = fma(val, xv, dotv);
        }
    }
    if (part) {
        dsh[threadIdx.x] = dotv;
        __syncthreads();
        if (threadIdx.x < KC) {
            double acc2 = 0.0;
            for (int u = 0; u < 256 / KC; ++u) acc2 += dsh[threadIdx.x + KC * u];
            part[(int64_t)blockIdx.x * k + k0 + threadIdx.x] = acc2;
        }
    }
}

}  // namespace

// chunk tables
int plan_products(Handle& h) {
    const int J = h.geo.J;
    h.chunk_off.assign(J + 1, 0);
    std::vector<int64_t> part_off;
    std::vector<int32_t> chunk_sub;
    int64_t poff = 0;
    for (int j = 0; j < J; ++j) {
        const int64_t n = h.pts.row_off[j + 1] - h.pts.row_off[j];
        const int64_t nc = (n + kChunk - 1) / kChunk;
        h.chunk_off[j + 1] = h.chunk_off[j] + nc;
        for (int64_t c = 0; c < nc; ++c) {
            part_off.push_back(poff);
            poff += h.p[j];
            chunk_sub.push_back(j);
        }
    }
    h.n_chunks = h.chunk_off[J];
    h.part_total = poff;
    RDD_TRY(dev_alloc(h, &h.d_chunk_sub, chunk_sub.size()));
    RDD_TRY(dev_alloc(h, &h.d_chunk_off, h.chunk_off.size()));
    RDD_TRY(dev_alloc(h, &h.d_part_off, part_off.size()));
    if (!chunk_sub.empty()) {
        RDD_TRY(upload(h, h.d_chunk_sub, chunk_sub.data(), sizeof(int32_t) * chunk_sub.size()));
        RDD_TRY(upload(h, h.d_part_off, part_off.data(), sizeof(int64_t) * part_off.size()));
    }
    RDD_TRY(upload(h, h.d_chunk_off, h.chunk_off.data(), sizeof(int64_t) * h.chunk_off.size()));
    std::vector<int32_t> col_sub(h.P), feat_sub(h.sum_m);
    for (int j = 0; j < J; ++j) {
        for (int64_t c = h.col_off[j]; c < h.col_off[j + 1]; ++c) col_sub[c] = j;
        for (int64_t f = h.m_off[j]; f < h.m_off[j + 1]; ++f) feat_sub[f] = j;
    }
    RDD_TRY(dev_alloc(h, &h.d_col_sub, col_sub.size()));
    RDD_TRY(dev_alloc(h, &h.d_feat_sub, feat_sub.size()));
    if (!col_sub.empty())
        RDD_TRY(upload(h, h.d_col_sub, col_sub.data(), sizeof(int32_t) * col_sub.size()));
    RDD_TRY(upload(h, h.d_feat_sub, feat_sub.data(), sizeof(int32_t) * feat_sub.size()));
    // per-column partial metadata for the fused reductions
    std::vector<int64_t> pbase(h.P);
    std::vector<int32_t> pstride(h.P), nch(h.P);
    for (int j = 0; j < J; ++j) {
        const int64_t ch0 = h.chunk_off[j];
        const int64_t nc = h.chunk_off[j + 1] - ch0;
        for (int64_t c = 0; c < h.p[j]; ++c) {
            const int64_t g = h.col_off[j] + c;
            pbase[g] = (nc > 0 ? part_off[ch0] : 0) + c;
            pstride[g] = h.p[j];
            nch[g] = (int32_t)nc;
        }
    }
    RDD_TRY(dev_alloc(h, &h.d_col_pbase, pbase.size()));
    RDD_TRY(dev_alloc(h, &h.d_col_pstride, pstride.size()));
    RDD_TRY(dev_alloc(h, &h.d_col_nch, nch.size()));
    if (h.P > 0) {
        RDD_TRY(upload(h, h.d_col_pbase, pbase.data(), sizeof(int64_t) * h.P));
        RDD_TRY(upload(h, h.d_col_pstride, pstride.data(), sizeof(int32_t) * h.P));
        RDD_TRY(upload(h, h.d_col_nch, nch.data(), sizeof(int32_t) * h.P));
    }
    return RANN_OK;
}

// y = H x; `tpair` holds pairs x k doubles
int launch_Hx_pairs(Handle& h, const double* x, int k, double* y, double* tpair) {
    if (h.n_chunks == 0) {
        RDD_HIP(hipMemsetAsync(y, 0, sizeof(double) * h.N * k, h.stream));
        return RANN_OK;
    }
    KTimer kt_(h.stream, "k_Hx");
    for (int k0 = 0; k0 < k;) {
        const int rem = k - k0;
        const int kb = rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
#define RDD_HXC(KBV)                                                                              \
    hipLaunchKernelGGL((k_Hx_chunk<KBV>), dim3((unsigned)h.n_chunks), dim3(256), 0, h.stream,     \
                       h.d_chunk_sub, h.d_chunk_off, h.pts.d_row_off, h.d_p, h.d_h_off, h.d_col_off, \
                       h.d_H, x, k, k0, tpair)
        switch (kb) {
            case 8: RDD_HXC(8); break;
            case 4: RDD_HXC(4); break;
            case 2: RDD_HXC(2); break;
            default: RDD_HXC(1); break;
        }
#undef RDD_HXC
        k0 += kb;
    }
    hipLaunchKernelGGL(k_pair_to_rows, dim3((unsigned)((h.N * k + 255) / 256)), dim3(256), 0, h.stream,
                       h.N, k, h.pts.d_cover_off, h.pts.d_cover, tpair, y);
    kt_.stop();
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

// part = chunk partial sums of H^T y (part_total x k)
int launch_HTy_part(Handle& h, const double* y, int k, double* part) {
    if (h.n_chunks == 0) return RANN_OK;
    KTimer kt_(h.stream, "k_HTy_part");
    for (int k0 = 0; k0 < k;) {
        const int rem = k - k0;
        const int kb = rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
#define RDD_HTC(KBV)                                                                               \
    hipLaunchKernelGGL((k_HTy_chunk<KBV>), dim3((unsigned)h.n_chunks), dim3(256), 0, h.stream,     \
                       h.d_chunk_sub, h.d_chunk_off, h.d_part_off, h.pts.d_row_off, h.pts.d_rows,  \
                       h.d_p, h.d_h_off, h.d_H, y, k, k0, part)
        switch (kb) {
            case 8: RDD_HTC(8); break;
            case 4: RDD_HTC(4); break;
            case 2: RDD_HTC(2); break;
            default: RDD_HTC(1); break;
        }
#undef RDD_HTC
        k0 += kb;
    }
    kt_.stop();
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace rdd

namespace rdd {

int normal_parts(const Handle& h, int k) {
    (void)k;
    return (int)h.n_slab_tasks;
}

int launch_normal(Handle& h, const double* x, int k, double* s, double* part, const PUpd* pup) {
    PUpd pu{};
    if (pup) pu = *pup;
    KTimer kt_(h.stream, "k_normal");
    for (int k0 = 0; k0 < k;) {
        const int rem = k - k0;
        if (rem >= 16) {  // matrix cores, 32 or 16 right-hand sides per launch
            const int kc = rem >= 32 ? 32 : 16;
            if (h.n_slab_tasks) {
#define RDD_NM(KCV, UPDV, P2V)                                                                         \
    hipLaunchKernelGGL((k_nrm_mfma<KCV, UPDV, P2V>), dim3((unsigned)h.n_slab_tasks), dim3(256), 0, h.stream, \
                       h.d_slab_tasks, h.d_p, h.d_col_off, h.d_Nt_off, h.d_N_coff, h.d_N_cols, h.d_Nt, x, k,  \
                       k0, s, part, pu)
                const bool upd = pu.pprev != nullptr;
                if (kc == 32 && k % 2 == 0) {  // 16-byte loads of right-hand-side pairs
                    if (upd) RDD_NM(32, true, true); else RDD_NM(32, false, true);
                } else if (kc == 32) {
                    if (upd) RDD_NM(32, true, false); else RDD_NM(32, false, false);
                } else {
                    if (upd) RDD_NM(16, true, false); else RDD_NM(16, false, false);
                }
#undef RDD_NM
            }
            k0 += kc;
            continue;
        }
        const int kb = rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
#define RDD_NS(KBV)                                                                                       \
    do {                                                                                                  \
        if (pu.pprev)                                                                                     \
            hipLaunchKernelGGL((k_nrm_slab<KBV, true>), dim3((unsigned)h.n_slab_tasks), dim3(256), 0,     \
                               h.stream, h.d_slab_tasks, h.d_p, h.d_col_off, h.d_N_off, h.d_N_coff,       \
                               h.d_N_cols, h.d_N, x, k, k0, s, part, pu);                                 \
        else                                                                                              \
            hipLaunchKernelGGL((k_nrm_slab<KBV, false>), dim3((unsigned)h.n_slab_tasks), dim3(256), 0,    \
                               h.stream, h.d_slab_tasks, h.d_p, h.d_col_off, h.d_N_off, h.d_N_coff,       \
                               h.d_N_cols, h.d_N, x, k, k0, s, part, pu);                                 \
    } while (0)
        if (h.n_slab_tasks) {
            switch (kb) {
                case 8: RDD_NS(8); break;
                case 4: RDD_NS(4); break;
                case 2: RDD_NS(2); break;
                default: RDD_NS(1); break;
            }
        }
#undef RDD_NS
        k0 += kb;
    }
    kt_.stop();
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace rdd
