// Overlapping Schwarz preconditioners for H^T H (paper Sec. 3).
//
//   AS : z = sum_i R_i^T A_i^{-1} R_i r
//   RAS: z = sum_i R_i^T D_i A_i^{-1} R_i r,  D_i = the columns block i owns (the
//        columns of each subdomain belong to the first block holding it)
//   SAS: D_i = 1 / (number of blocks containing the column)
//
// Block i selects the columns of every subdomain in its stencil.  The local
// inverse A_i^{-1} is kept as packed lower 64x64 tiles (factor.hip): the
// symmetric W_i itself in FP64, or the triangular factor Y_i (A_i^{-1} =
// Y_i^T Y_i) in FP32 for the mixed path.  One workgroup per tile (a, b), b <=
// a, writes the row sums R_ab = M_ab x_b and/or the column sums C_ab =
// M_ab^T x_a into slots of its own, and a reduction adds them in a fixed order
// (no atomics):
//   FP64: z_c = sum_{b <= c} R_cb + sum_{a > c} C_ac      (one pass over W)
//   FP32: u_c = sum_{b <= c} R_cb, then z_c = sum_{a >= c} C_ac with x = u
//         (two passes over Y, the second usually from cache).
#include <hip/hip_runtime.h>

#include <hip/hip_ext.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "common.h"
#include "mfma.h"

namespace rdd {

template <class T>
int local_blocks(Handle& h, const T* H, T* A_out);
int plan_tiles(Handle& h);
int factor_tiles(Handle& h, double* A, double* W);

namespace {

constexpr int kT = 64;              // tile edge
constexpr int kTE = kT * kT;        // tile elements

// 16 consecutive elements (16-byte aligned) into registers
__device__ __forceinline__ void load16(const double* p, double* v) {
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const double2 w = q[e];
        v[2 * e] = w.x;
        v[2 * e + 1] = w.y;
    }
}
__device__ __forceinline__ void load16(const float* p, float* v) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const float4 w = q[e];
        v[4 * e] = w.x;
        v[4 * e + 1] = w.y;
        v[4 * e + 2] = w.z;
        v[4 * e + 3] = w.w;
    }
}

// Column sums of one tile held in the row mapping (thread = (row, 16-column
// segment)): out[c] = sum_r tile[r][c] xv[r], through a transposed copy in
// LDS; thread (c, quarter) sums 16 rows, the 4 quarters meet by shuffles.
// With one tile per workgroup, or two buffers used alternately, one barrier
// per tile suffices.
template <class T, int KB>
__device__ __forceinline__ void tile_colsum(const T* v, const double (*xv)[KB], T (*ts)[kT + 1],
                                            double* out, int k, int cmax) {
    const int tid = threadIdx.x, row = tid >> 2, seg = tid & 3;
    const int col = tid >> 2, rq = tid & 3;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) ts[row][seg * 16 + cc] = v[cc];
    __syncthreads();
    double c[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) c[t] = 0.0;
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int r = rq * 16 + rr;
        const double tv = (double)ts[r][col];
#pragma unroll
        for (int t = 0; t < KB; ++t) c[t] = fma(tv, xv[r][t], c[t]);
    }
#pragma unroll
    for (int t = 0; t < KB; ++t) {
        c[t] += __shfl_xor(c[t], 1);
        c[t] += __shfl_xor(c[t], 2);
    }
    if (rq == 0 && col < cmax)
#pragma unroll
        for (int t = 0; t < KB; ++t) out[(int64_t)col * k + t] = c[t];
}

// One tile (a, b) of the local solves: R = M_ab x_b into the R slot (a, b)
// when WR, C = M_ab^T xa into the C slot (a, b) when WC (skipped for the
// diagonal tile of the symmetric W).  xb comes from r through the block's
// column list; xa from r (symmetric W) or from the block vector u (second
// pass of the triangular factor).
template <class T, int KB, bool WR, bool WC, bool XA_FROM_U, bool SYM>
__global__ void __launch_bounds__(256) k_tile_apply(const int4* __restrict__ tasks,
                                                    const int64_t* __restrict__ t_off,
                                                    const int64_t* __restrict__ qv,
                                                    const int64_t* __restrict__ ub_off,
                                                    const int64_t* __restrict__ s_off,
                                                    const int32_t* __restrict__ blk_cols,
                                                    const T* __restrict__ M,
                                                    const double* __restrict__ r,
                                                    const double* __restrict__ u, int k, int k0,
                                                    double* __restrict__ Rs, double* __restrict__ Cs) {
    __shared__ double xb[kT][KB];
    __shared__ double xa[kT][KB];
    __shared__ T ts[kT][kT + 1];
    const int4 tk = tasks[blockIdx.x];
    const int i = tk.x, a = tk.y, b = tk.z;
    const int64_t q = qv[i];
    const int tid = threadIdx.x, row = tid >> 2, seg = tid & 3;
    const int64_t tile = (int64_t)a * (a + 1) / 2 + b;
    T v[16];
    load16(M + t_off[i] + tile * kTE + row * kT + seg * 16, v);
    const int32_t* cols = blk_cols + ub_off[i];
    const bool do_c = WC && !(SYM && a == b);
    for (int e = tid; e < kT * KB; e += 256) {
        const int c = e / KB, t = e % KB;
        if (WR) {
            const int64_t gc = (int64_t)b * kT + c;
            xb[c][t] = (gc < q) ? r[(int64_t)cols[gc] * k + k0 + t] : 0.0;
        }
        if (do_c) {
            const int64_t gc = (int64_t)a * kT + c;
            double xv = 0.0;
            if (gc < q) xv = XA_FROM_U ? u[(ub_off[i] + gc) * k + k0 + t] : r[(int64_t)cols[gc] * k + k0 + t];
            xa[c][t] = xv;
        }
    }
    __syncthreads();
    const int64_t so = (s_off[i] + tile * kT) * k + k0;  // slot (a, b), entry 0
    if (WR) {
        double acc[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) acc[t] = 0.0;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc)
#pragma unroll
            for (int t = 0; t < KB; ++t) acc[t] = fma((double)v[cc], xb[seg * 16 + cc][t], acc[t]);
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            acc[t] += __shfl_xor(acc[t], 1);
            acc[t] += __shfl_xor(acc[t], 2);
        }
        if (seg == 0)
#pragma unroll
            for (int t = 0; t < KB; ++t) Rs[so + (int64_t)row * k + t] = acc[t];
    }
    if (do_c) {
        const int cmax = (int)((q - (int64_t)b * kT) < kT ? q - (int64_t)b * kT : kT);
        tile_colsum<T, KB>(v, xa, ts, Cs + so, k, cmax);
    }
}

// The same tile products for the symmetric FP64 W with 1 or 2 right-hand
// sides, persistent: workgroup w takes the tiles w, w + G, ... (G = grid
// size) and loads the next tile, its task record and its x values while the
// current tile is multiplied.  A tile is read with whole-line loads: thread t
// takes the 16-byte pieces t, t + 256, ..., i.e. columns 2 (t % 32), + 1 of
// the rows 8 e + t / 32 (e = 0..7), and multiplies them in registers.  Row
// sums reduce over the 32 lanes that share the rows (a reduce-scatter over
// shuffles, one row per lane group at the end); column sums reduce over the
// eight row groups (the two of a wave by a shuffle, the four waves in LDS).
template <int KB>
__global__ void __launch_bounds__(256) k_tile_apply_ps(const int4* __restrict__ tasks, int ntasks,
                                                       const int64_t* __restrict__ t_off,
                                                       const int64_t* __restrict__ qv,
                                                       const int64_t* __restrict__ ub_off,
                                                       const int64_t* __restrict__ s_off,
                                                       const int32_t* __restrict__ blk_cols,
                                                       const double* __restrict__ M,
                                                       const double* __restrict__ r, int k, int k0,
                                                       double* __restrict__ Rs, double* __restrict__ Cs) {
    static_assert(KB <= 2, "one staged x value per thread");
    __shared__ double xb[kT][KB];
    __shared__ double xa[kT][KB];
    __shared__ double red[4][kT][KB];  // column partials of the four waves
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lrow = tid >> 5, cp = tid & 31;  // rows 8 e + lrow, columns 2 cp, 2 cp + 1
    // thread tid < 64 KB stages x_b entry tid, 64 KB <= tid < 128 KB stages x_a
    const bool sb = tid < kT * KB, sa = !sb && tid < 2 * kT * KB;
    const int se = sb ? tid : tid - kT * KB;
    const int sc = se / KB, st = se % KB;
    int task = blockIdx.x;
    if (task >= ntasks) return;
#define RDD_PS_FETCH(TK_I, TK, V, XR, SO)                                                      \
    {                                                                                         \
        TK = tasks[TK_I];                                                                     \
        const int i_ = TK.x, a_ = TK.y, b_ = TK.z;                                            \
        const int64_t q_ = qv[i_];                                                            \
        const int64_t tile_ = (int64_t)a_ * (a_ + 1) / 2 + b_;                                \
        const double2* src_ = reinterpret_cast<const double2*>(M + t_off[i_] + tile_ * kTE);  \
        /* rows and columns of the tile inside the block: the zero padding of */            \
        /* the last tile row and column is not read */                                      \
        const int64_t rv_ = q_ - (int64_t)a_ * kT, cv_ = q_ - (int64_t)b_ * kT;               \
        _Pragma("unroll") for (int e = 0; e < 8; ++e) {                                      \
            const int ch_ = e * 256 + tid;                                                    \
            const bool in_ = (ch_ >> 5) < rv_ && 2 * (ch_ & 31) < cv_;                        \
            const double2 w_ = in_ ? src_[ch_] : make_double2(0.0, 0.0);                      \
            V[2 * e] = w_.x;                                                                  \
            V[2 * e + 1] = w_.y;                                                              \
        }                                                                                     \
        SO = (s_off[i_] + tile_ * kT) * k + k0;                                               \
        XR = 0.0;                                                                             \
        if (sb || (sa && a_ != b_)) {                                                         \
            const int64_t gc_ = (int64_t)(sb ? b_ : a_) * kT + sc;                            \
            if (gc_ < q_) XR = r[(int64_t)blk_cols[ub_off[i_] + gc_] * k + k0 + st];          \
        }                                                                                     \
    }
    int4 tk;
    double v[16];
    double xr;
    int64_t so;
    RDD_PS_FETCH(task, tk, v, xr, so)
    while (true) {
        const bool do_c = tk.y != tk.z;
        const int64_t q = qv[tk.x];
        const int cmax = (int)((q - (int64_t)tk.z * kT) < kT ? q - (int64_t)tk.z * kT : kT);
        if (sb) xb[sc][st] = xr;
        if (sa) xa[sc][st] = xr;
        __syncthreads();  // x staged; the previous tile's column partials are read
        const int next = task + gridDim.x;
        int4 tkn;
        double vn[16];
        double xrn;
        int64_t son;
        RDD_PS_FETCH(next < ntasks ? next : task, tkn, vn, xrn, son)  // the last round reloads its own tile
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            const double x0 = xb[2 * cp][t], x1 = xb[2 * cp + 1][t];
            // row partials of rows 8 e + lrow, e = 0..7
            double p[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) p[e] = fma(v[2 * e], x0, v[2 * e + 1] * x1);
            // reduce-scatter over lanes xor 16, 8, 4: lane keeps one row
            // (e = 4 b4 + 2 b3 + b2 from its lane bits 4, 3, 2)
            const int b4 = (cp >> 4) & 1, b3 = (cp >> 3) & 1, b2 = (cp >> 2) & 1;
            double p4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double mine = b4 ? p[4 + u] : p[u], other = b4 ? p[u] : p[4 + u];
                p4[u] = mine + __shfl_xor(other, 16);
            }
            double p2[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const double mine = b3 ? p4[2 + u] : p4[u], other = b3 ? p4[u] : p4[2 + u];
                p2[u] = mine + __shfl_xor(other, 8);
            }
            double p1;
            {
                const double mine = b2 ? p2[1] : p2[0], other = b2 ? p2[0] : p2[1];
                p1 = mine + __shfl_xor(other, 4);
            }
            p1 += __shfl_xor(p1, 2);
            p1 += __shfl_xor(p1, 1);
            if ((cp & 3) == 0) {
                const int e = 4 * b4 + 2 * b3 + b2;
                Rs[so + (int64_t)(8 * e + lrow) * k + t] = p1;
            }
            // column partials of columns 2 cp, 2 cp + 1 over this thread's rows
            if (do_c) {
                double c0 = 0.0, c1 = 0.0;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const double xv = xa[8 * e + lrow][t];
                    c0 = fma(v[2 * e], xv, c0);
                    c1 = fma(v[2 * e + 1], xv, c1);
                }
                c0 += __shfl_xor(c0, 32);  // the wave's other row group
                c1 += __shfl_xor(c1, 32);
                if (lane < 32) {
                    red[wave][2 * cp][t] = c0;
                    red[wave][2 * cp + 1][t] = c1;
                }
            }
        }
        __syncthreads();  // column partials written; x may be restaged
        if (do_c && tid < kT * KB) {
            const int col = tid / KB, t = tid % KB;
            const double c = (red[0][col][t] + red[1][col][t]) + (red[2][col][t] + red[3][col][t]);
            if (col < cmax) Cs[so + (int64_t)col * k + t] = c;
        }
        if (next >= ntasks) break;
        task = next;
        tk = tkn;
        so = son;
        xr = xrn;
        for (int e = 0; e < 16; ++e) v[e] = vn[e];
    }
#undef RDD_PS_FETCH
}

// One (block, tile row a) of the triangular factor (mixed path): u_a = sum_b
// Y_ab x_b over the contiguous tiles (a, 0..a), then C(a, b) = Y_ab^T u_a for
// every b <= a, the tile row read a second time (from cache).  Tiles are read
// with whole-line loads (thread t takes the 16-byte pieces t, t + 256, ...)
// into one of two LDS buffers, the next tile in flight meanwhile; row sums
// read LDS rows, column sums LDS columns.
template <int KB>
__global__ void __launch_bounds__(256) k_trirow_apply(const int2* __restrict__ tasks,
                                                      const int64_t* __restrict__ t_off,
                                                      const int64_t* __restrict__ qv,
                                                      const int64_t* __restrict__ ub_off,
                                                      const int64_t* __restrict__ s_off,
                                                      const int32_t* __restrict__ blk_cols,
                                                      const float* __restrict__ Y,
                                                      const double* __restrict__ r, int k, int k0,
                                                      double* __restrict__ Cs) {
    constexpr int kXC = 8;       // tiles of x staged per chunk
    constexpr int kTS = kT + 4;  // LDS row stride in floats (16-byte aligned rows)
    __shared__ double xs[kXC * kT][KB];
    __shared__ double ua[kT][KB];
    __shared__ __attribute__((aligned(16))) float ts[2][kT * kTS];
    const int2 tk = tasks[blockIdx.x];
    const int i = tk.x, a = tk.y;
    const int64_t q = qv[i];
    const int tid = threadIdx.x, row = tid >> 2, seg = tid & 3;
    const int col = tid >> 2, rq = tid & 3;
    const float4* Ya = reinterpret_cast<const float4*>(Y + t_off[i] + (int64_t)a * (a + 1) / 2 * kTE);
    const int32_t* cols = blk_cols + ub_off[i];
    double* cla = Cs + s_off[i] * k + k0 + (int64_t)a * (a + 1) / 2 * kT * k;  // slot (a, b) at cla + b kT k
    // 16-byte piece ch = e 256 + tid of a tile: row ch / 16, columns 4 (ch % 16) ..
#define RDD_TR_PUT(DST, V)                                                                              \
    _Pragma("unroll") for (int e = 0; e < 4; ++e) {                                                      \
        const int ch = e * 256 + tid;                                                                    \
        *reinterpret_cast<float4*>(DST + (ch >> 4) * kTS + 4 * (ch & 15)) =                             \
            make_float4(V[4 * e], V[4 * e + 1], V[4 * e + 2], V[4 * e + 3]);                             \
    }
#define RDD_TR_GET(V, TILE)                                                                              \
    _Pragma("unroll") for (int e = 0; e < 4; ++e) {                                                      \
        const float4 w_ = Ya[(int64_t)(TILE) * (kTE / 4) + e * 256 + tid];                              \
        V[4 * e] = w_.x;                                                                                 \
        V[4 * e + 1] = w_.y;                                                                             \
        V[4 * e + 2] = w_.z;                                                                             \
        V[4 * e + 3] = w_.w;                                                                             \
    }
    double acc[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) acc[t] = 0.0;
    float v[16], vn[16];
    RDD_TR_GET(v, 0)
    for (int b = 0; b <= a; ++b) {
        const int bb = b % kXC;
        if (bb == 0) {
            const int nb = (a + 1 - b < kXC) ? a + 1 - b : kXC;
            __syncthreads();
            for (int e = tid; e < nb * kT * KB; e += 256) {
                const int c = e / KB, t = e % KB;
                const int64_t gc = (int64_t)b * kT + c;
                xs[c][t] = (gc < q) ? r[(int64_t)cols[gc] * k + k0 + t] : 0.0;
            }
        }
        float* tb = ts[b & 1];
        RDD_TR_PUT(tb, v)
        __syncthreads();
        RDD_TR_GET(vn, (b < a) ? b + 1 : b)
        const float* trow = tb + row * kTS + seg * 16;
        const double (*xr)[KB] = xs + bb * kT + seg * 16;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc)
#pragma unroll
            for (int t = 0; t < KB; ++t) acc[t] = fma((double)trow[cc], xr[cc][t], acc[t]);
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = vn[e];
    }
#pragma unroll
    for (int t = 0; t < KB; ++t) {
        acc[t] += __shfl_xor(acc[t], 1);
        acc[t] += __shfl_xor(acc[t], 2);
    }
    if (seg == 0)
#pragma unroll
        for (int t = 0; t < KB; ++t) ua[row][t] = acc[t];
    RDD_TR_GET(v, 0)
    __syncthreads();  // u_a complete; both LDS buffers free
    for (int b = 0; b <= a; ++b) {
        float* tb = ts[b & 1];
        RDD_TR_PUT(tb, v)
        __syncthreads();
        RDD_TR_GET(vn, (b < a) ? b + 1 : b)
        const int cmax = (int)((q - (int64_t)b * kT) < kT ? q - (int64_t)b * kT : kT);
        double c[KB];
#pragma unroll
        for (int t = 0; t < KB; ++t) c[t] = 0.0;
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            const int rw = rq + 4 * rr;
            const double tv = (double)tb[rw * kTS + col];
#pragma unroll
            for (int t = 0; t < KB; ++t) c[t] = fma(tv, ua[rw][t], c[t]);
        }
#pragma unroll
        for (int t = 0; t < KB; ++t) {
            c[t] += __shfl_xor(c[t], 1);
            c[t] += __shfl_xor(c[t], 2);
        }
        if (rq == 0 && col < cmax)
#pragma unroll
            for (int t = 0; t < KB; ++t) cla[(int64_t)b * kT * k + (int64_t)col * k + t] = c[t];
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = vn[e];
    }
#undef RDD_TR_GET
#undef RDD_TR_PUT
}

// Batched right-hand sides (KC = 16 or 32 of them per launch) on the matrix
// cores.  MFMA 16x16x4 lane layout: lane l = 16 g + lr supplies A[lr][g] and
// B[g][lr]; wave w owns the 16 output rows 16 w .. 16 w + 15 of a tile.  A
// lane loads its row of a tile as one 16-element run (columns 16 g .. 16 g +
// 15), which is the A operand of the row product directly (K index 16 g + s
// at step s); products with a transposed tile read it from LDS.
// Every workgroup owns a 64-entry piece of a block result and accumulates it
// in its MFMA registers, so the results go straight to the block vector (no
// slots, no reduction pass).

// FP64 symmetric W, one (block, tile a) per workgroup: z_a = sum_b W_ab x_b
// over the stored tiles (a, b), b <= a, and the transposes of the tiles
// (b, a), b > a.  Every tile off the diagonal is read by two workgroups.  Both
// kinds of tile go straight from global memory into the A operand: lane
// (lr, g) of wave w takes row 16 w + lr of a stored tile at the columns
// 8 (s / 2) + 2 g + s % 2 (K index at step s; the four lanes of a row read 64
// consecutive bytes per load), or column 16 w + lr of a transposed one at the
// rows 16 g + s (16 rows 64 apart, each load reading 16 consecutive entries
// across the lanes).  The x segment of
// tile b is staged in one of two LDS buffers while tile b - 1 is multiplied
// (one barrier per tile); the next tile is loaded meanwhile.
template <int KC>
__global__ void __launch_bounds__(256) k_rowcol_mfma64(const int2* __restrict__ tasks,
                                                       const int64_t* __restrict__ t_off,
                                                       const int64_t* __restrict__ qv,
                                                       const int64_t* __restrict__ ub_off,
                                                       const int32_t* __restrict__ blk_cols,
                                                       const double* __restrict__ W,
                                                       const double* __restrict__ r, int k, int k0,
                                                       double* __restrict__ z) {
    constexpr int NB = KC / 16;
    constexpr int XPT = kT * KC / 256;  // x values staged per thread
    __shared__ double xs[2][kT][KC + 1];
    const int2 tk = tasks[blockIdx.x];
    const int i = tk.x, a = tk.y;
    const int64_t q = qv[i];
    const int nt = (int)((q + kT - 1) / kT);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const double* Wi = W + t_off[i];
    const int32_t* cols = blk_cols + ub_off[i];
    // a stored tile's row 16 w + lr is read as 8 pairs: at step s lane
    // (lr, g) supplies K index 8 (s / 2) + 2 g + s % 2, so that the lanes of
    // a row read 64 consecutive bytes per load; a transposed tile's K index is
    // 16 g + s (16 consecutive entries across the lanes of each g)
    auto load_w = [&](int b, double* v) {
        if (b <= a) {
            const double2* src = reinterpret_cast<const double2*>(
                Wi + ((int64_t)a * (a + 1) / 2 + b) * kTE + (16 * w + lr) * kT + 2 * g);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const double2 t2 = src[4 * e];
                v[2 * e] = t2.x;
                v[2 * e + 1] = t2.y;
            }
        } else {
            const double* T = Wi + ((int64_t)b * (b + 1) / 2 + a) * kTE + (16 * g) * kT + 16 * w + lr;
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = T[s * kT];
        }
    };
    // the column indices of an x segment are loaded one step before its
    // values, so that each step waits for one round of loads
    auto load_cols = [&](int b, int32_t* ci) {
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int e = threadIdx.x + 256 * m;
            const int64_t gc = (int64_t)b * kT + e / KC;
            ci[m] = (gc < q) ? cols[gc] : -1;
        }
    };
    auto load_x = [&](const int32_t* ci, double* xr) {
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int e = threadIdx.x + 256 * m;
            xr[m] = (ci[m] >= 0) ? r[(int64_t)ci[m] * k + k0 + e % KC] : 0.0;
        }
    };
    auto put_x = [&](int buf, const double* xr) {
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int e = threadIdx.x + 256 * m;
            xs[buf][e / KC][e % KC] = xr[m];
        }
    };
    typedef Mfma<double>::acc_t acc_t;
    acc_t Z[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) Z[nb][e] = 0.0;
    double v[16], xr[XPT];
    int32_t ci[XPT], cn[XPT];
    load_cols(0, ci);
    load_w(0, v);
    load_x(ci, xr);
    put_x(0, xr);
    if (nt > 1) load_cols(1, ci);
    __syncthreads();
    for (int b = 0; b < nt; ++b) {
        double vn[16];
        const bool more = b + 1 < nt;
        if (more) {
            load_w(b + 1, vn);
            load_x(ci, xr);
            if (b + 2 < nt) load_cols(b + 2, cn);
        }
        const int buf = b & 1;
        // the B operands from LDS first (K order of the stored tile or of its
        // transpose), then the matrix-core chain
        double xb[16][NB];
        if (b <= a) {
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) xb[s][nb] = xs[buf][8 * (s >> 1) + 2 * g + (s & 1)][16 * nb + lr];
        } else {
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) xb[s][nb] = xs[buf][16 * g + s][16 * nb + lr];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) Z[nb] = Mfma<double>::mma(v[s], xb[s][nb], Z[nb]);
        if (more) {
            put_x(buf ^ 1, xr);
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = vn[s];
            if (b + 2 < nt)
#pragma unroll
                for (int m = 0; m < XPT; ++m) ci[m] = cn[m];
        }
        __syncthreads();
    }
    double* zi = z + ub_off[i] * k + k0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t ga = (int64_t)a * kT + 16 * w + Mfma<double>::out_row(lane, e);
            if (ga < q) zi[ga * k + 16 * nb + lr] = Z[nb][e];
        }
}

constexpr int kBlkNT = 6;

// Stages x = r[cols[row]][k0 .. k0 + KC) of one block (rows < q; zero rows up
// to kBlkNT tiles) into LDS with the workgroup's 512 threads: every column
// index of a thread's rows first, then all of its loads in flight, then the
// LDS stores.  Rows past q re-read row q - 1 and store zero, so that no load
// sits behind a branch.
template <int KC, typename T>
__device__ __forceinline__ void stage_block_x(T (*xs)[KC + 1], const int32_t* __restrict__ cols,
                                              const double* __restrict__ r, int64_t q, int k, int k0) {
    constexpr int kSE = kBlkNT * kT * KC / 512;
    static_assert(kSE * 512 == kBlkNT * kT * KC, "whole rows per sweep");
    const int tid = threadIdx.x, t = tid % KC;
    int32_t c[kSE];
#pragma unroll
    for (int m = 0; m < kSE; ++m) {
        const int64_t row = (tid + 512 * m) / KC;
        c[m] = cols[row < q ? row : q - 1];
    }
    double x[kSE];
#pragma unroll
    for (int m = 0; m < kSE; ++m) x[m] = r[(int64_t)c[m] * k + k0 + t];
#pragma unroll
    for (int m = 0; m < kSE; ++m) {
        const int row = (tid + 512 * m) / KC;
        xs[row][t] = (row < q) ? (T)x[m] : (T)0;
    }
}

// Symmetric W (FP64, or its FP32 copy on the mixed path), one block per
// workgroup of eight waves (blocks of at most kBlkNT tiles per edge): z = W x
// over the whole block, every stored tile read from memory once per use
// inside the workgroup.  x (q x KC) is gathered into LDS once.  Output tile a
// of the block takes the products with all nt input tiles b: the stored tile
// (a, b) for b <= a, the transpose of (b, a) for b > a (column runs straight
// into the A operand, as in k_rowcol_mfma64).  Wave w computes rows
// 16 (w % 4) .. + 15 of the output tiles a = w / 4, w / 4 + 2, ...,
// accumulating each in registers over b and storing it; the next product's
// tile rows are loaded while the current one is multiplied.  T is the type of
// W, x in LDS and the matrix-core arithmetic; z is written in FP64.
template <class T, int KC>
__device__ __forceinline__ void blk_apply(T (*xs)[KC + 1], const int32_t* __restrict__ blocks,
                                          const int64_t* __restrict__ t_off, const int64_t* __restrict__ qv,
                                          const int64_t* __restrict__ ub_off, const int32_t* __restrict__ blk_cols,
                                          const T* __restrict__ W, const double* __restrict__ r, int k, int k0,
                                          double* __restrict__ z) {
    constexpr int NB = KC / 16;
    const int i = blocks[blockIdx.x];
    const int64_t q = qv[i];
    const int nt = (int)((q + kT - 1) / kT);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int rg = w & 3, half = w >> 2;
    const T* Wi = W + t_off[i];
    const int32_t* cols = blk_cols + ub_off[i];
    // this wave's products: (a, b) for a = half, half + 2, ..., b = 0 .. nt - 1
    const int na = (nt - half + 1) / 2;
    const int njobs = na * nt;
    auto load_job = [&](int jb, T* v) {
        const int a = half + 2 * (jb / nt), b = jb % nt;
        if (b <= a) {
            load16(Wi + ((int64_t)a * (a + 1) / 2 + b) * kTE + (16 * rg + lr) * kT + 16 * g, v);
        } else {
            const T* Tt = Wi + ((int64_t)b * (b + 1) / 2 + a) * kTE + (16 * g) * kT + 16 * rg + lr;
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = Tt[s * kT];
        }
    };
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t Z[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) Z[nb][e] = T(0);
    T v[16], vn[16];
    if (njobs > 0) load_job(0, v);
    stage_block_x<KC>(xs, cols, r, q, k, k0);
    __syncthreads();  // x staged
    double* zi = z + ub_off[i] * k + k0;
    for (int jb = 0; jb < njobs; ++jb) {
        const int a = half + 2 * (jb / nt), b = jb % nt;
        if (jb + 1 < njobs) load_job(jb + 1, vn);
        // all of the product's B operands from LDS first, so that the
        // matrix-core chain does not wait on each read
        T xb[16][NB];
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) xb[s][nb] = xs[b * kT + 16 * g + s][16 * nb + lr];
        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the chain
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) Z[nb] = Mfma<T>::mma(v[s], xb[s][nb], Z[nb]);
        if (b == nt - 1) {  // output tile a complete
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int64_t ga = (int64_t)a * kT + 16 * rg + Mfma<T>::out_row(lane, e);
                    if (ga < q) zi[ga * k + 16 * nb + lr] = (double)Z[nb][e];
                    Z[nb][e] = T(0);
                }
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) v[s] = vn[s];
    }
}

template <int KC>
__global__ void __launch_bounds__(512) k_blk_mfma64(const int32_t* __restrict__ blocks,
                                                    const int64_t* __restrict__ t_off,
                                                    const int64_t* __restrict__ qv,
                                                    const int64_t* __restrict__ ub_off,
                                                    const int32_t* __restrict__ blk_cols,
                                                    const double* __restrict__ W,
                                                    const double* __restrict__ r, int k, int k0,
                                                    double* __restrict__ z) {
    __shared__ double xs[kBlkNT * kT][KC + 1];
    blk_apply<double, KC>(xs, blocks, t_off, qv, ub_off, blk_cols, W, r, k, k0, z);
}

// The mixed path's single-pass local solves: the same product with the FP32
// copy of W, FP32 operands and accumulation on the matrix cores.
template <int KC>
__global__ void __launch_bounds__(512) k_blk_w32(const int32_t* __restrict__ blocks,
                                                 const int64_t* __restrict__ t_off,
                                                 const int64_t* __restrict__ qv,
                                                 const int64_t* __restrict__ ub_off,
                                                 const int32_t* __restrict__ blk_cols,
                                                 const float* __restrict__ W,
                                                 const double* __restrict__ r, int k, int k0,
                                                 double* __restrict__ z) {
    __shared__ float xs[kBlkNT * kT][KC + 1];
    blk_apply<float, KC>(xs, blocks, t_off, qv, ub_off, blk_cols, W, r, k, k0, z);
}

// FP32 triangular factor Y (mixed path), one block per workgroup of eight
// waves (blocks of at most kBlkNT tiles per edge): u = Y x, then z = Y^T u,
// FP32 operands and accumulation on the matrix cores, z widened to FP64.  x
// (rounded to FP32) and u stay in LDS; wave w computes rows 16 (w % 4) .. + 15
// of the output tiles w / 4, w / 4 + 2, ... of each pass.  Pass 1 reads the
// stored tiles (a, b), b <= a, as row runs; pass 2 their transposes as column
// runs, both straight into the A operand; the next tile's rows are loaded
// while the current one is multiplied.
template <int KC>
__global__ void __launch_bounds__(512) k_blk_mfma32(const int32_t* __restrict__ blocks,
                                                    const int64_t* __restrict__ t_off,
                                                    const int64_t* __restrict__ qv,
                                                    const int64_t* __restrict__ ub_off,
                                                    const int32_t* __restrict__ blk_cols,
                                                    const float* __restrict__ Y,
                                                    const double* __restrict__ r, int k, int k0,
                                                    double* __restrict__ z) {
    constexpr int NB = KC / 16;
    __shared__ float xs[kBlkNT * kT][KC + 1];
    __shared__ float us[kBlkNT * kT][KC + 1];
    const int i = blocks[blockIdx.x];
    const int64_t q = qv[i];
    const int nt = (int)((q + kT - 1) / kT);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const int rg = w & 3, half = w >> 2;
    const float* Yi = Y + t_off[i];
    const int32_t* cols = blk_cols + ub_off[i];
    stage_block_x<KC>(xs, cols, r, q, k, k0);
    typedef Mfma<float>::acc_t acc_t;
    // pass 1 jobs (a, b), b <= a, for a = half, half + 2, ...; pass 2 jobs
    // (c, a), a >= c, for c = half, half + 2, ...  Job lists are walked by
    // (output tile, input tile) in order.
    auto next_job = [&](int pass, int& o, int& in) -> bool {  // advance; false at the end
        if (pass == 1) {
            if (++in > o) {
                o += 2;
                in = 0;
            }
        } else {
            if (++in >= nt) {
                o += 2;
                in = o;
            }
        }
        return o < nt;
    };
    auto load = [&](int pass, int o, int in, float* v) {
        if (pass == 1) {  // Y_oin, row run
            load16(Yi + ((int64_t)o * (o + 1) / 2 + in) * kTE + (16 * rg + lr) * kT + 16 * g, v);
        } else {          // Y_{in, o}^T, column run
            const float* T = Yi + ((int64_t)in * (in + 1) / 2 + o) * kTE + (16 * g) * kT + 16 * rg + lr;
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = T[s * kT];
        }
    };
    double* zi = z + ub_off[i] * k + k0;
    for (int pass = 1; pass <= 2; ++pass) {
        float (*src)[KC + 1] = (pass == 1) ? xs : us;
        int o = half, in = (pass == 1) ? 0 : half;
        float v[16], vn[16];
        bool any = o < nt;
        if (any) load(pass, o, in, v);
        __syncthreads();  // pass 1: x staged; pass 2: u complete
        acc_t Acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e) Acc[nb][e] = 0.0f;
        while (any) {
            int o2 = o, in2 = in;
            const bool more = next_job(pass, o2, in2);
            if (more) load(pass, o2, in2, vn);
            float xb[16][NB];  // B operands from LDS first
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) xb[s][nb] = src[in * kT + 16 * g + s][16 * nb + lr];
            __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the chain
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) Acc[nb] = Mfma<float>::mma(v[s], xb[s][nb], Acc[nb]);
            const bool last = (pass == 1) ? (in == o) : (in == nt - 1);
            if (last) {  // output tile o complete
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int rr = 16 * rg + Mfma<float>::out_row(lane, e);
                        const int64_t ga = (int64_t)o * kT + rr;
                        if (pass == 1) {
                            us[o * kT + rr][16 * nb + lr] = Acc[nb][e];
                        } else if (ga < q) {
                            zi[ga * k + 16 * nb + lr] = (double)Acc[nb][e];
                        }
                        Acc[nb][e] = 0.0f;
                    }
            }
            o = o2;
            in = in2;
            any = more;
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = vn[s];
        }
    }
}

// FP32 triangular factor Y (mixed path), first pass, one (block, tile row a)
// per workgroup: u_a = sum_{b <= a} Y_ab x_b in FP32, stored as FP32.
template <int KC>
__global__ void __launch_bounds__(256) k_urow_mfma32(const int2* __restrict__ tasks,
                                                     const int64_t* __restrict__ t_off,
                                                     const int64_t* __restrict__ qv,
                                                     const int64_t* __restrict__ ub_off,
                                                     const int32_t* __restrict__ blk_cols,
                                                     const float* __restrict__ Y,
                                                     const double* __restrict__ r, int k, int k0,
                                                     float* __restrict__ u) {
    constexpr int NB = KC / 16;
    constexpr int XPT = kT * KC / 256;
    __shared__ float xs[2][kT][KC + 1];
    const int2 tk = tasks[blockIdx.x];
    const int i = tk.x, a = tk.y;
    const int64_t q = qv[i];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const float* Ya = Y + t_off[i] + (int64_t)a * (a + 1) / 2 * kTE + (16 * w + lr) * kT + 16 * g;
    const int32_t* cols = blk_cols + ub_off[i];
    auto load_x = [&](int b, float* xr) {  // rows past q re-read row q - 1 and are discarded
        double xd[XPT];
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int e = threadIdx.x + 256 * m;
            const int64_t gc = (int64_t)b * kT + e / KC;
            xd[m] = r[(int64_t)cols[gc < q ? gc : q - 1] * k + k0 + e % KC];
        }
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int64_t gc = (int64_t)b * kT + (threadIdx.x + 256 * m) / KC;
            xr[m] = (gc < q) ? (float)xd[m] : 0.0f;
        }
    };
    typedef Mfma<float>::acc_t acc_t;
    acc_t U[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) U[nb][e] = 0.0f;
    float v[16], xr[XPT];
    load16(Ya, v);
    load_x(0, xr);
    for (int b = 0; b <= a; ++b) {
        float (*xb)[KC + 1] = xs[b & 1];
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int e = threadIdx.x + 256 * m;
            xb[e / KC][e % KC] = xr[m];
        }
        __syncthreads();  // xs[b & 1] written; its previous reads (step b - 2) ended before step b - 1's barrier
        float vn[16];
        if (b < a) {
            load16(Ya + (int64_t)(b + 1) * kTE, vn);
            load_x(b + 1, xr);
        }
        float bo[16][NB];  // B operands from LDS first
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bo[s][nb] = xb[16 * g + s][16 * nb + lr];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) U[nb] = Mfma<float>::mma(v[s], bo[s][nb], U[nb]);
        if (b < a)
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = vn[s];
    }
    float* ui = u + ub_off[i] * k + k0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t ga = (int64_t)a * kT + 16 * w + Mfma<float>::out_row(lane, e);
            if (ga < q) ui[ga * k + 16 * nb + lr] = U[nb][e];
        }
}

// Second pass, one (block, tile column c) per workgroup: z_c = sum_{a >= c}
// Y_ac^T u_a (FP32 operands and accumulation), written as FP64.
template <int KC>
__global__ void __launch_bounds__(256) k_zcol_mfma32(const int2* __restrict__ tasks,
                                                     const int64_t* __restrict__ t_off,
                                                     const int64_t* __restrict__ qv,
                                                     const int64_t* __restrict__ ub_off,
                                                     const float* __restrict__ Y,
                                                     const float* __restrict__ u, int k, int k0,
                                                     double* __restrict__ z) {
    constexpr int NB = KC / 16;
    constexpr int XPT = kT * KC / 256;
    __shared__ float us[kT][KC + 1];
    __shared__ float ts[kT][kT + 1];
    const int2 tk = tasks[blockIdx.x];
    const int i = tk.x, c = tk.y;
    const int64_t q = qv[i];
    const int nt = (int)((q + kT - 1) / kT);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lr = lane & 15, g = lane >> 4;
    const float* Yi = Y + t_off[i] + (16 * w + lr) * kT + 16 * g;
    const float* ui = u + ub_off[i] * k + k0;
    auto load_u = [&](int a, float* ur) {
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int e = threadIdx.x + 256 * m;
            const int64_t ga = (int64_t)a * kT + e / KC;
            ur[m] = (ga < q) ? ui[ga * k + e % KC] : 0.0f;
        }
    };
    typedef Mfma<float>::acc_t acc_t;
    acc_t Z[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) Z[nb][e] = 0.0f;
    float v[16], ur[XPT];
    load16(Yi + ((int64_t)c * (c + 1) / 2 + c) * kTE, v);
    load_u(c, ur);
    for (int a = c; a < nt; ++a) {
        __syncthreads();  // the previous step's reads of us and ts are done
#pragma unroll
        for (int m = 0; m < XPT; ++m) {
            const int e = threadIdx.x + 256 * m;
            us[e / KC][e % KC] = ur[m];
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) ts[16 * w + lr][16 * g + s] = v[s];
        __syncthreads();
        float vn[16];
        if (a + 1 < nt) {
            load16(Yi + ((int64_t)(a + 1) * (a + 2) / 2 + c) * kTE, vn);
            load_u(a + 1, ur);
        }
        float ao[16], bo[16][NB];  // operands from LDS first
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            ao[s] = ts[16 * g + s][16 * w + lr];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bo[s][nb] = us[16 * g + s][16 * nb + lr];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) Z[nb] = Mfma<float>::mma(ao[s], bo[s][nb], Z[nb]);
        if (a + 1 < nt)
#pragma unroll
            for (int s = 0; s < 16; ++s) v[s] = vn[s];
    }
    double* zi = z + ub_off[i] * k + k0;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t gcol = (int64_t)c * kT + 16 * w + Mfma<float>::out_row(lane, e);
            if (gcol < q) zi[gcol * k + 16 * nb + lr] = (double)Z[nb][e];
        }
}

// z[e] for block entry e in tile column c (offset o):
//   (with R) sum_{b <= c} R(c, b)[o]  +  (with C) sum_{a >= c + c_skip} C(a, c)[o]
// (right-hand sides t0 .. t0 + kt - 1 of the k)
__global__ void k_slot_reduce(int64_t nent, int k, int t0, int kt, int use_r, int use_c, int c_skip,
                              const int32_t* __restrict__ ent_blk, const int64_t* __restrict__ ub_off,
                              const int64_t* __restrict__ s_off, const int64_t* __restrict__ qv,
                              const double* __restrict__ Rs, const double* __restrict__ Cs,
                              double* __restrict__ z) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= nent * kt) return;
    const int64_t e = idx / kt;
    const int t = t0 + (int)(idx % kt);
    const int i = ent_blk[e];
    const int64_t c = e - ub_off[i];
    const int tc = (int)(c / kT), o = (int)(c % kT);
    const int nt = (int)((qv[i] + kT - 1) / kT);
    const int64_t base = s_off[i] * k + t + (int64_t)o * k;
    // 8 slots per round (their loads in flight together), fixed order
    double s = 0.0;
    if (use_r) {
        const int64_t row0 = (int64_t)tc * (tc + 1) / 2;
        for (int b0 = 0; b0 <= tc; b0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = (b0 + u <= tc) ? Rs[base + (row0 + b0 + u) * kT * k] : 0.0;
            s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
        }
    }
    if (use_c)
        for (int a0 = tc + c_skip; a0 < nt; a0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int a = a0 + u;
                v[u] = (a < nt) ? Cs[base + ((int64_t)a * (a + 1) / 2 + tc) * kT * k] : 0.0;
            }
            s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
        }
    z[e * k + t] = s;
}


// z[g] = sum over (block entry e containing column g) of w_e u[e]; unit
// weights when gat_w is null
__global__ void k_gather_sum(int64_t P, int k, const int64_t* __restrict__ gat_off,
                             const int64_t* __restrict__ gat, const double* __restrict__ gat_w,
                             const double* __restrict__ u, double* __restrict__ z) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= P * k) return;
    int64_t g = idx / k;
    int t = (int)(idx % k);
    double s = 0.0;
    if (gat_w) {
        for (int64_t e = gat_off[g]; e < gat_off[g + 1]; ++e) s += gat_w[e] * u[gat[e] * k + t];
    } else {
        for (int64_t e = gat_off[g]; e < gat_off[g + 1]; ++e) s += u[gat[e] * k + t];
    }
    z[idx] = s;
}

// out[g] = r[g] / (number of blocks containing column g), the count being the
// length of g's gather list (every entry is listed: AS and SAS plans)
__global__ void k_div_count(int64_t P, int k, const int64_t* __restrict__ gat_off,
                            const double* __restrict__ r, double* __restrict__ out) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= P * k) return;
    const int64_t g = idx / k;
    out[idx] = r[idx] / (double)(gat_off[g + 1] - gat_off[g]);
}

// out = (double) in
__global__ void k_widen_f32(int64_t n, const float* __restrict__ in, double* __restrict__ out) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < n) out[idx] = (double)in[idx];
}

// out = [r; 0]: the n entries of r followed by pad zeros
__global__ void k_copy_pad(int64_t n, int64_t pad, const double* __restrict__ r, double* __restrict__ out) {
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < n) out[idx] = r[idx];
    else if (idx < n + pad) out[idx] = 0.0;
}

}  // namespace

// stencil of block i, ascending subdomain order
static std::vector<int> make_stencil(const Handle& h, int i, const std::vector<std::vector<double>>& cen) {
    const Geo& g = h.geo;
    std::vector<int> out;
    std::vector<int> ci(g.d);
    int t = i;
    for (int q = 0; q < g.d; ++q) {
        ci[q] = t % g.l[q];
        t /= g.l[q];
    }
    for (int j = 0; j < g.J; ++j) {
        int tj = j, diff = 0;
        bool full_ok = true;
        for (int q = 0; q < g.d; ++q) {
            int cq = tj % g.l[q];
            tj /= g.l[q];
            diff += std::abs(cq - ci[q]);
            if (!(std::fabs(cen[i][q] - cen[j][q]) < 2.0 * g.sigma[q])) full_ok = false;
        }
        if (h.stencil == RANN_STENCIL_SELF) {
            if (j == i) out.push_back(j);
        } else if (h.stencil == RANN_STENCIL_FACE) {
            if (diff <= 1) out.push_back(j);
        } else {
            if (full_ok) out.push_back(j);
        }
    }
    return out;
}

// The columns of subdomain j belong to the first block (increasing index)
// whose stencil holds j: the Boolean algebraic partition of unity D_i of RAS,
// sum_i R_i^T D_i R_i = I.
static std::vector<int> ras_owner(const std::vector<std::vector<int>>& sten) {
    std::vector<int> owner(sten.size(), -1);
    for (size_t i = 0; i < sten.size(); ++i)
        for (int j : sten[i])
            if (owner[j] < 0) owner[j] = (int)i;
    return owner;
}

// One application plan (see ApplyPlan).  Forward: block i gathers the entries
// of the subdomains use(i, j) selects, with weight w(column); the tile rows
// computed start at the tile of the first used entry.  Masked (the transposed
// RAS apply): the entries of subdomains block i does not own read the zero
// row P of the input, every entry of a block that owns anything is gathered
// with unit weight, and blocks that own nothing are skipped.
static int build_plan(Handle& h, const std::vector<int64_t>& ub_off, const std::vector<int>& mult,
                      const std::vector<int>& owner, bool masked, ApplyPlan& pl) {
    const int J = h.geo.J;
    const bool ras = (h.precond == RANN_PRECOND_RAS);
    std::vector<int32_t> blk_cols((size_t)ub_off[J]);
    std::vector<int64_t> row_lo(J, 0), row_hi(J, 0);  // block entries [lo, hi) of the result needed
    std::vector<char> used((size_t)ub_off[J], 0);
    std::vector<int64_t> ent_col((size_t)ub_off[J]);  // global column of each block entry
    for (int i = 0; i < J; ++i) {
        bool owns = false;
        for (int j : h.sten[i]) owns |= (owner[j] == i);
        int64_t e = ub_off[i], pos = 0, lo = -1, hi = 0;
        for (int j : h.sten[i]) {
            const bool mine = (owner[j] == i);
            const bool use = masked ? owns : (!ras || mine);
            for (int c = 0; c < h.p[j]; ++c, ++e, ++pos) {
                const int64_t gcol = h.col_off[j] + c;
                blk_cols[e] = (int32_t)((masked && !mine) ? h.P : gcol);
                ent_col[e] = gcol;
                used[e] = use ? 1 : 0;
                if (use) {
                    if (lo < 0) lo = pos;
                    hi = pos + 1;
                }
            }
        }
        row_lo[i] = lo < 0 ? 0 : lo;
        row_hi[i] = lo < 0 ? 0 : hi;
    }
    // gather lists: CSR over global columns, entries in block order
    std::vector<int64_t> gat_off(h.P + 1, 0);
    for (int i = 0; i < J; ++i)
        for (int64_t e = ub_off[i]; e < ub_off[i + 1]; ++e)
            if (used[e]) gat_off[ent_col[e] + 1]++;
    for (int64_t g = 0; g < h.P; ++g) gat_off[g + 1] += gat_off[g];
    std::vector<int64_t> gat((size_t)gat_off[h.P]), fill(gat_off.begin(), gat_off.end() - 1);
    std::vector<double> gat_w((size_t)gat_off[h.P]);
    for (int64_t e = 0; e < ub_off[J]; ++e) {
        if (!used[e]) continue;
        const int64_t gcol = ent_col[e];
        const int64_t slot = fill[gcol]++;
        gat[slot] = e;
        gat_w[slot] = (!masked && h.precond == RANN_PRECOND_SAS) ? 1.0 / (double)mult[gcol] : 1.0;
    }
    // segments: block i's entries of subdomain j, when used, in block order per j
    {
        std::vector<std::vector<std::pair<int64_t, double>>> segs(J);
        for (int i = 0; i < J; ++i) {
            int64_t e = ub_off[i];
            for (int j : h.sten[i]) {
                if (h.p[j] > 0 && used[e])
                    segs[j].push_back({e, (!masked && h.precond == RANN_PRECOND_SAS)
                                              ? 1.0 / (double)mult[h.col_off[j]] : 1.0});
                e += h.p[j];
            }
        }
        std::vector<int64_t> seg_off(J + 1, 0), seg_src;
        std::vector<double> seg_w;
        for (int j = 0; j < J; ++j) {
            std::sort(segs[j].begin(), segs[j].end(),
                      [](const std::pair<int64_t, double>& x, const std::pair<int64_t, double>& y) {
                          return x.first < y.first;
                      });
            for (auto& sg : segs[j]) {
                seg_src.push_back(sg.first);
                seg_w.push_back(sg.second);
            }
            seg_off[j + 1] = (int64_t)seg_src.size();
        }
        RDD_TRY(dev_alloc(h, &pl.d_seg_off, seg_off.size()));
        RDD_TRY(dev_alloc(h, &pl.d_seg_src, std::max<size_t>(seg_src.size(), 1)));
        RDD_TRY(dev_alloc(h, &pl.d_seg_w, std::max<size_t>(seg_w.size(), 1)));
        RDD_TRY(upload(h, pl.d_seg_off, seg_off.data(), sizeof(int64_t) * seg_off.size()));
        if (!seg_src.empty()) {
            RDD_TRY(upload(h, pl.d_seg_src, seg_src.data(), sizeof(int64_t) * seg_src.size()));
            RDD_TRY(upload(h, pl.d_seg_w, seg_w.data(), sizeof(double) * seg_w.size()));
        }
    }
    RDD_TRY(dev_alloc(h, &pl.d_blk_cols, blk_cols.size()));
    RDD_TRY(dev_alloc(h, &pl.d_gat_off, gat_off.size()));
    RDD_TRY(dev_alloc(h, &pl.d_gat, gat.size()));
    RDD_TRY(dev_alloc(h, &pl.d_gat_w, gat_w.size()));
    RDD_TRY(upload(h, pl.d_blk_cols, blk_cols.data(), sizeof(int32_t) * blk_cols.size()));
    RDD_TRY(upload(h, pl.d_gat_off, gat_off.data(), sizeof(int64_t) * gat_off.size()));
    if (!gat.empty()) {
        RDD_TRY(upload(h, pl.d_gat, gat.data(), sizeof(int64_t) * gat.size()));
        RDD_TRY(upload(h, pl.d_gat_w, gat_w.data(), sizeof(double) * gat_w.size()));
    }
    // packed tiles, one task per stored tile of the tile rows from the first
    // needed one on (the symmetric apply's rows c need the row sums of tile
    // row c and the column sums of the tile rows below it)
    std::vector<int4> tv;
    for (int i = 0; i < J; ++i) {
        const int nt = h.nt[i];
        if (nt == 0 || row_hi[i] == 0) continue;
        const int b_lo = (int)(row_lo[i] / 64);
        for (int a = b_lo; a < nt; ++a)
            for (int b = 0; b <= a; ++b) tv.push_back(make_int4(i, a, b, 0));
    }
    pl.n_tile_tasks = (int64_t)tv.size();
    RDD_TRY(dev_alloc(h, &pl.d_tile_tasks, tv.size()));
    if (!tv.empty()) RDD_TRY(upload(h, pl.d_tile_tasks, tv.data(), sizeof(int4) * tv.size()));
    // tile rows, longest first (triangular factor of the mixed path)
    std::vector<std::pair<int, int2>> rt;
    for (const int4& t4 : tv)
        if (t4.z == 0) rt.push_back({t4.y + 1, make_int2(t4.x, t4.y)});
    std::stable_sort(rt.begin(), rt.end(), [](const std::pair<int, int2>& x, const std::pair<int, int2>& y) {
        return x.first > y.first;
    });
    std::vector<int2> rtv;
    for (auto& e : rt) rtv.push_back(e.second);
    pl.n_row_tasks = (int64_t)rtv.size();
    RDD_TRY(dev_alloc(h, &pl.d_row_tasks, rtv.size()));
    if (!rtv.empty()) RDD_TRY(upload(h, pl.d_row_tasks, rtv.data(), sizeof(int2) * rtv.size()));
    // tiles of the block results that are used, ordered by the tiles a column
    // pass reads, longest first
    std::vector<std::pair<int, int2>> ct;
    for (int i = 0; i < J; ++i) {
        const int nt = h.nt[i];
        if (nt == 0 || row_hi[i] == 0) continue;
        const int c_lo = (int)(row_lo[i] / 64);
        const int c_hi = (int)((row_hi[i] - 1) / 64);
        for (int c = c_lo; c <= c_hi; ++c) ct.push_back({nt - c, make_int2(i, c)});
    }
    std::stable_sort(ct.begin(), ct.end(), [](const std::pair<int, int2>& x, const std::pair<int, int2>& y) {
        return x.first > y.first;
    });
    std::vector<int2> ctv;
    for (auto& e : ct) ctv.push_back(e.second);
    pl.n_col_tasks = (int64_t)ctv.size();
    RDD_TRY(dev_alloc(h, &pl.d_col_tasks, ctv.size()));
    if (!ctv.empty()) RDD_TRY(upload(h, pl.d_col_tasks, ctv.data(), sizeof(int2) * ctv.size()));
    // whole blocks, widest first (the batched FP64 local solves of narrow blocks)
    std::vector<std::pair<int, int>> bl;
    pl.max_nt = 0;
    for (int i = 0; i < J; ++i)
        if (h.nt[i] > 0 && row_hi[i] > 0) {
            bl.push_back({h.nt[i], i});
            pl.max_nt = std::max(pl.max_nt, (int)h.nt[i]);
        }
    std::stable_sort(bl.begin(), bl.end(), [](const std::pair<int, int>& x, const std::pair<int, int>& y) {
        return x.first > y.first;
    });
    std::vector<int32_t> blv;
    for (auto& e : bl) blv.push_back(e.second);
    pl.n_blk_list = (int64_t)blv.size();
    RDD_TRY(dev_alloc(h, &pl.d_blk_list, std::max<size_t>(blv.size(), 1)));
    if (!blv.empty()) RDD_TRY(upload(h, pl.d_blk_list, blv.data(), sizeof(int32_t) * blv.size()));
    return RANN_OK;
}

int build_schwarz(Handle& h) {
    const int J = h.geo.J;
    if (h.precond == RANN_PRECOND_NONE) return RANN_OK;
    std::vector<std::vector<double>> cen(J, std::vector<double>(h.geo.d));
    {
        std::vector<double> mu_all(h.geo.mu_off[h.geo.d - 1] + h.geo.l[h.geo.d - 1]);
        RDD_TRY(download(h, mu_all.data(), h.d_mu, sizeof(double) * mu_all.size()));
        for (int j = 0; j < J; ++j) {
            int t = j;
            for (int i = 0; i < h.geo.d; ++i) {
                cen[j][i] = mu_all[h.geo.mu_off[i] + t % h.geo.l[i]];
                t /= h.geo.l[i];
            }
        }
    }
    h.sten.assign(J, {});
    h.q.assign(J, 0);
    h.f_off.assign(J + 1, 0);
    std::vector<int64_t> ub_off(J + 1, 0);
    h.max_q = 0;
    for (int i = 0; i < J; ++i) {
        h.sten[i] = make_stencil(h, i, cen);
        int64_t q = 0;
        for (int j : h.sten[i]) q += h.p[j];
        h.q[i] = q;
        h.f_off[i + 1] = h.f_off[i] + q * q;
        ub_off[i + 1] = ub_off[i] + q;
        h.max_q = std::max<int>(h.max_q, (int)q);
    }
    h.factor_elems = h.f_off[J];
    std::vector<int> mult(h.P, 0);
    for (int i = 0; i < J; ++i)
        for (int j : h.sten[i])
            for (int c = 0; c < h.p[j]; ++c) mult[h.col_off[j] + c]++;
    const std::vector<int> owner = ras_owner(h.sten);
    RDD_TRY(dev_alloc(h, &h.d_f_off, J + 1));
    RDD_TRY(dev_alloc(h, &h.d_q, J));
    RDD_TRY(dev_alloc(h, &h.d_ub_off, J + 1));
    RDD_TRY(upload(h, h.d_f_off, h.f_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(upload(h, h.d_q, h.q.data(), sizeof(int64_t) * J));
    RDD_TRY(upload(h, h.d_ub_off, ub_off.data(), sizeof(int64_t) * (J + 1)));
    h.ub_total = ub_off[J];

    // the tiles of the local inverses, the application plans and the slot
    // layout of the row and column sums
    RDD_TRY(plan_tiles(h));
    RDD_TRY(build_plan(h, ub_off, mult, owner, false, h.ap));
    if (h.precond == RANN_PRECOND_RAS) RDD_TRY(build_plan(h, ub_off, mult, owner, true, h.apT));
    std::vector<int64_t> s_off(J + 1, 0);
    std::vector<int32_t> ent_blk((size_t)h.ub_total);
    for (int i = 0; i < J; ++i) {
        const int nt = h.nt[i];
        s_off[i + 1] = s_off[i] + (int64_t)nt * (nt + 1) / 2 * 64;
        for (int64_t e = ub_off[i]; e < ub_off[i + 1]; ++e) ent_blk[e] = i;
    }
    h.slot_total = s_off[J];
    RDD_TRY(dev_alloc(h, &h.d_s_off, s_off.size()));
    RDD_TRY(dev_alloc(h, &h.d_ent_blk, ent_blk.size()));
    RDD_TRY(upload(h, h.d_s_off, s_off.data(), sizeof(int64_t) * s_off.size()));
    if (!ent_blk.empty()) RDD_TRY(upload(h, h.d_ent_blk, ent_blk.data(), sizeof(int32_t) * ent_blk.size()));

    // local Gram blocks (FP64) and their factorisation
    double *d_A = nullptr, *d_W = nullptr;
    RDD_TRY(dev_alloc(h, &d_A, (size_t)h.factor_elems));
    RDD_TRY(dev_alloc(h, &d_W, (size_t)h.factor_elems));
    if (h.precision == RANN_MIXED) {
        RDD_TRY(dev_alloc(h, &h.d_M32, (size_t)h.tile_elems));
        int ntmax = 0;
        for (int i = 0; i < J; ++i) ntmax = std::max(ntmax, (int)h.nt[i]);
        // the single-pass FP32 local solves of narrow blocks apply W itself
        if (ntmax <= kBlkNT) RDD_TRY(dev_alloc(h, &h.d_W32, (size_t)h.tile_elems));
    } else
        RDD_TRY(dev_alloc(h, &h.d_M64, (size_t)h.tile_elems));
    if (h.d_G32) {
        // A_i from the FP32 Gram blocks, widened for the FP64 factorisation
        float* d_A32 = reinterpret_cast<float*>(d_W);  // d_W is free until the factorisation
        RDD_TRY(local_blocks<float>(h, h.d_H32, d_A32));
        hipLaunchKernelGGL(k_widen_f32, dim3((unsigned)((h.factor_elems + 255) / 256)), dim3(256), 0, h.stream,
                           h.factor_elems, d_A32, d_A);
        RDD_HIP(hipGetLastError());
    } else {
        RDD_TRY(local_blocks<double>(h, h.d_H, d_A));
    }
    const int rc = factor_tiles(h, d_A, d_W);
    dev_free(h, d_A);
    dev_free(h, d_W);
    return rc;
}

// u_i = A_i^{-1} r_{N(i)} for every block (the local solves only).  ub holds
// (2 ub_total + 2 slot_total) k doubles: the result, the intermediate block
// vector of the triangular factor, and the row and column sum slots.
int launch_precond_local(Handle& h, const ApplyPlan& pl, const double* r, int k, double* ub) {
    double* u1 = ub + h.ub_total * k;
    double* Rs = u1 + h.ub_total * k;
    double* Cs = Rs + h.slot_total * k;
    const int64_t tot = h.ub_total * k;
    const unsigned tgrid = (unsigned)pl.n_tile_tasks;
    if (tgrid == 0 || tot == 0) return RANN_OK;
    // FP64 with one or two right-hand sides is a single persistent launch,
    // timed by the events it records itself
    const bool one_launch = h.precision != RANN_MIXED && (k <= 2 || k == 16 || k == 32);
    KTimer kt_(h.stream, "k_tile_apply", one_launch);
    int kv0 = 0;  // right-hand sides from kv0 on take the slot path
    for (int k0 = 0; k0 < k;) {
        const int rem = k - k0;
        if (rem >= 16) {  // matrix cores, 32 or 16 right-hand sides per launch, no slots
            const int kc = rem >= 32 ? 32 : 16;
            float* u32 = reinterpret_cast<float*>(u1);
            if (h.precision == RANN_MIXED && h.d_W32 && pl.max_nt <= kBlkNT && pl.n_blk_list > 0) {
                if (kc == 32)
                    hipLaunchKernelGGL((k_blk_w32<32>), dim3((unsigned)pl.n_blk_list), dim3(512), 0, h.stream,
                                       pl.d_blk_list, h.d_t_off, h.d_q, h.d_ub_off, pl.d_blk_cols, h.d_W32, r, k,
                                       k0, ub);
                else
                    hipLaunchKernelGGL((k_blk_w32<16>), dim3((unsigned)pl.n_blk_list), dim3(512), 0, h.stream,
                                       pl.d_blk_list, h.d_t_off, h.d_q, h.d_ub_off, pl.d_blk_cols, h.d_W32, r, k,
                                       k0, ub);
            } else if (h.precision == RANN_MIXED && pl.max_nt <= kBlkNT && pl.n_blk_list > 0) {
                if (kc == 32)
                    hipLaunchKernelGGL((k_blk_mfma32<32>), dim3((unsigned)pl.n_blk_list), dim3(512), 0, h.stream,
                                       pl.d_blk_list, h.d_t_off, h.d_q, h.d_ub_off, pl.d_blk_cols, h.d_M32, r, k,
                                       k0, ub);
                else
                    hipLaunchKernelGGL((k_blk_mfma32<16>), dim3((unsigned)pl.n_blk_list), dim3(512), 0, h.stream,
                                       pl.d_blk_list, h.d_t_off, h.d_q, h.d_ub_off, pl.d_blk_cols, h.d_M32, r, k,
                                       k0, ub);
            } else if (h.precision == RANN_MIXED) {
#define RDD_MX(KCV)                                                                                        \
    hipLaunchKernelGGL((k_urow_mfma32<KCV>), dim3((unsigned)pl.n_row_tasks), dim3(256), 0, h.stream,          \
                       pl.d_row_tasks, h.d_t_off, h.d_q, h.d_ub_off, pl.d_blk_cols, h.d_M32, r, k, k0, u32);  \
    hipLaunchKernelGGL((k_zcol_mfma32<KCV>), dim3((unsigned)pl.n_col_tasks), dim3(256), 0, h.stream,          \
                       pl.d_col_tasks, h.d_t_off, h.d_q, h.d_ub_off, h.d_M32, u32, k, k0, ub)
                if (kc == 32) {
                    RDD_MX(32);
                } else {
                    RDD_MX(16);
                }
#undef RDD_MX
            } else {
                hipEvent_t ea = one_launch ? kt_.a : nullptr, eb = one_launch ? kt_.b : nullptr;
                if (pl.max_nt <= kBlkNT && pl.n_blk_list > 0) {
                    if (kc == 32)
                        hipExtLaunchKernelGGL((k_blk_mfma64<32>), dim3((unsigned)pl.n_blk_list), dim3(512), 0,
                                              h.stream, ea, eb, 0, (const int32_t*)pl.d_blk_list,
                                              (const int64_t*)h.d_t_off, (const int64_t*)h.d_q,
                                              (const int64_t*)h.d_ub_off, (const int32_t*)pl.d_blk_cols,
                                              (const double*)h.d_M64, r, k, k0, ub);
                    else
                        hipExtLaunchKernelGGL((k_blk_mfma64<16>), dim3((unsigned)pl.n_blk_list), dim3(512), 0,
                                              h.stream, ea, eb, 0, (const int32_t*)pl.d_blk_list,
                                              (const int64_t*)h.d_t_off, (const int64_t*)h.d_q,
                                              (const int64_t*)h.d_ub_off, (const int32_t*)pl.d_blk_cols,
                                              (const double*)h.d_M64, r, k, k0, ub);
                } else if (kc == 32)
                    hipExtLaunchKernelGGL((k_rowcol_mfma64<32>), dim3((unsigned)pl.n_col_tasks), dim3(256), 0,
                                          h.stream, ea, eb, 0, (const int2*)pl.d_col_tasks, (const int64_t*)h.d_t_off,
                                          (const int64_t*)h.d_q, (const int64_t*)h.d_ub_off,
                                          (const int32_t*)pl.d_blk_cols, (const double*)h.d_M64, r, k, k0, ub);
                else
                    hipExtLaunchKernelGGL((k_rowcol_mfma64<16>), dim3((unsigned)pl.n_col_tasks), dim3(256), 0,
                                          h.stream, ea, eb, 0, (const int2*)pl.d_col_tasks, (const int64_t*)h.d_t_off,
                                          (const int64_t*)h.d_q, (const int64_t*)h.d_ub_off,
                                          (const int32_t*)pl.d_blk_cols, (const double*)h.d_M64, r, k, k0, ub);
            }
            k0 += kc;
            kv0 = k0;
            continue;
        }
        const int kb = rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
#define RDD_TA(T, M, KBV, WR, WC, XU, SY)                                                          \
    hipLaunchKernelGGL((k_tile_apply<T, KBV, WR, WC, XU, SY>), dim3(tgrid), dim3(256), 0, h.stream, \
                       pl.d_tile_tasks, h.d_t_off, h.d_q, h.d_ub_off, h.d_s_off, pl.d_blk_cols, M, r, \
                       u1, k, k0, Rs, Cs)
#define RDD_TR(KBV)                                                                                 \
    hipLaunchKernelGGL((k_trirow_apply<KBV>), dim3((unsigned)pl.n_row_tasks), dim3(256), 0, h.stream, \
                       pl.d_row_tasks, h.d_t_off, h.d_q, h.d_ub_off, h.d_s_off, pl.d_blk_cols, h.d_M32, r, \
                       k, k0, Cs)
#define RDD_TA_KB(T, M, WR, WC, XU, SY)                  \
    switch (kb) {                                        \
        case 8: RDD_TA(T, M, 8, WR, WC, XU, SY); break;  \
        case 4: RDD_TA(T, M, 4, WR, WC, XU, SY); break;  \
        case 2: RDD_TA(T, M, 2, WR, WC, XU, SY); break;  \
        default: RDD_TA(T, M, 1, WR, WC, XU, SY); break; \
    }
        if (h.precision == RANN_MIXED) {
            switch (kb) {
                case 8: RDD_TR(8); break;
                case 4: RDD_TR(4); break;
                case 2: RDD_TR(2); break;
                default: RDD_TR(1); break;
            }
        } else if (kb <= 2) {
            // persistent over tune.tile_grid workgroups (default 768: three per
            // compute unit, which its register budget admits)
            const unsigned pg = std::min<unsigned>(tgrid, (unsigned)h.tune.tile_grid);
            hipEvent_t ea = one_launch ? kt_.a : nullptr, eb = one_launch ? kt_.b : nullptr;
            if (kb == 2)
                hipExtLaunchKernelGGL((k_tile_apply_ps<2>), dim3(pg), dim3(256), 0, h.stream, ea, eb, 0,
                                      (const int4*)pl.d_tile_tasks, (int)pl.n_tile_tasks, (const int64_t*)h.d_t_off,
                                      (const int64_t*)h.d_q, (const int64_t*)h.d_ub_off, (const int64_t*)h.d_s_off,
                                      (const int32_t*)pl.d_blk_cols, (const double*)h.d_M64, r, k, k0, Rs, Cs);
            else
                hipExtLaunchKernelGGL((k_tile_apply_ps<1>), dim3(pg), dim3(256), 0, h.stream, ea, eb, 0,
                                      (const int4*)pl.d_tile_tasks, (int)pl.n_tile_tasks, (const int64_t*)h.d_t_off,
                                      (const int64_t*)h.d_q, (const int64_t*)h.d_ub_off, (const int64_t*)h.d_s_off,
                                      (const int32_t*)pl.d_blk_cols, (const double*)h.d_M64, r, k, k0, Rs, Cs);
        } else {
            RDD_TA_KB(double, h.d_M64, true, true, false, true);
        }
        k0 += kb;
    }
    kt_.stop();
    // the slot reduction runs (and is timed) only for right-hand sides past
    // the matrix-core chunks
    const int kt = k - kv0;
    if (kt > 0) {
        KTimer kr_(h.stream, "k_slot_reduce");
        const unsigned rgrid = (unsigned)((h.ub_total * kt + 255) / 256);
        if (h.precision == RANN_MIXED)
            hipLaunchKernelGGL(k_slot_reduce, dim3(rgrid), dim3(256), 0, h.stream, h.ub_total, k, kv0, kt, 0, 1, 0,
                               h.d_ent_blk, h.d_ub_off, h.d_s_off, h.d_q, Rs, Cs, ub);
        else
            hipLaunchKernelGGL(k_slot_reduce, dim3(rgrid), dim3(256), 0, h.stream, h.ub_total, k, kv0, kt, 1, 1, 1,
                               h.d_ent_blk, h.d_ub_off, h.d_s_off, h.d_q, Rs, Cs, ub);
        kr_.stop();
    }
#undef RDD_TA_KB
#undef RDD_TR
#undef RDD_TA
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

int launch_precond(Handle& h, const double* r, int k, double* z, double* ub) {
    if (h.precond == RANN_PRECOND_NONE) {
        RDD_HIP(hipMemcpyAsync(z, r, sizeof(double) * h.P * k, hipMemcpyDeviceToDevice, h.stream));
        return RANN_OK;
    }
    RDD_TRY(launch_precond_local(h, h.ap, r, k, ub));
    return launch_gather(h, h.ap, ub, nullptr, k, z, nullptr);
}

// z = M^{-T} r.  The local inverses are symmetric, so the transpose moves the
// weights D_i from the local results onto the restricted input:
// M^{-T} = sum_i R_i^T A_i^{-1} D_i R_i.  AS: M^{-T} = M^{-1}.  SAS: D_i R_i =
// R_i D with D = 1/multiplicity, so M^{-T} r is the AS apply of D r.  RAS: the
// masked plan feeds each block its owned entries of r (the others read the
// zero row P of tmp = [r; 0]) and gathers the full local results.
int launch_precond_T(Handle& h, const double* r, int k, double* z, double* ub, double* tmp) {
    if (h.precond == RANN_PRECOND_NONE || h.precond == RANN_PRECOND_AS) return launch_precond(h, r, k, z, ub);
    const int64_t tot = h.P * k;
    const unsigned g = (unsigned)((tot + 255) / 256);
    if (h.precond == RANN_PRECOND_RAS) {
        const unsigned g1 = (unsigned)((tot + k + 255) / 256);
        hipLaunchKernelGGL(k_copy_pad, dim3(g1), dim3(256), 0, h.stream, tot, (int64_t)k, r, tmp);
        RDD_TRY(launch_precond_local(h, h.apT, tmp, k, ub));
        return launch_gather(h, h.apT, ub, nullptr, k, z, nullptr);
    }
    hipLaunchKernelGGL(k_div_count, dim3(g), dim3(256), 0, h.stream, h.P, k, h.ap.d_gat_off, r, tmp);
    RDD_TRY(launch_precond_local(h, h.ap, tmp, k, ub));
    hipLaunchKernelGGL(k_gather_sum, dim3(g), dim3(256), 0, h.stream, h.P, k, h.ap.d_gat_off, h.ap.d_gat,
                       (const double*)nullptr, ub, z);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace rdd
