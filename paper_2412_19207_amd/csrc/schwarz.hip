// Overlapping Schwarz preconditioners for H^T H (paper Sec. 3).
//
//   AS : z = sum_i R_i^T A_i^{-1} R_i r
//   RAS: z = sum_i R_i^T D_i A_i^{-1} R_i r,  D_i = the columns subdomain i owns
//   SAS: D_i = 1 / (number of blocks containing the column)
//
// Block i selects the columns of every subdomain in its stencil.  The local
// inverse is kept as the packed lower-triangular tiles of Y_i = L_i^{-1} D_i
// (factor.hip), A_i^{-1} = Y_i^T Y_i, and applied as two streaming passes
// instead of two dependent triangular solves:
//   row pass   : u_a = sum_{b <= a} Y_ab x_b   (one workgroup per tile row)
//   column pass: z_b = sum_{a >= b} Y_ab^T u_a (one workgroup per tile column)
// Tile rows of Y are contiguous in memory; every tile is read once per pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "common.h"

namespace rdd {

template <class T>
int local_blocks(Handle& h, const T* H, T* A_out);
int plan_tiles(Handle& h);
int factor_tiles(Handle& h, double* A, double* W);

namespace {

constexpr int kT = 64;              // tile edge
constexpr int kTE = kT * kT;        // tile elements
constexpr int kXChunk = 8;          // tiles of the input vector staged in LDS at once

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

// row pass: u_a = sum_{b <= a} Y_ab x_b with x = r gathered through the block's
// column list.  Thread (row, seg) owns 16 consecutive columns of one tile row;
// FP64 accumulation.
template <class T, int KB>
__global__ void __launch_bounds__(256) k_tri_row(const int2* __restrict__ tasks,
                                                 const int64_t* __restrict__ t_off,
                                                 const int64_t* __restrict__ qv,
                                                 const int64_t* __restrict__ ub_off,
                                                 const int32_t* __restrict__ blk_cols,
                                                 const T* __restrict__ Y,
                                                 const double* __restrict__ r, int k, int k0,
                                                 double* __restrict__ u) {
    __shared__ double xs[kXChunk * kT][KB];
    const int2 tk = tasks[blockIdx.x];
    const int i = tk.x, a = tk.y;
    const int64_t q = qv[i];
    const int tid = threadIdx.x, row = tid >> 2, seg = tid & 3;
    const T* Ya = Y + t_off[i] + (int64_t)a * (a + 1) / 2 * kTE + row * kT + seg * 16;
    const int32_t* cols = blk_cols + ub_off[i];
    double acc[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) acc[t] = 0.0;
    for (int b0 = 0; b0 <= a; b0 += kXChunk) {
        const int nb = (a + 1 - b0 < kXChunk) ? a + 1 - b0 : kXChunk;
        __syncthreads();
        for (int e = tid; e < nb * kT * KB; e += 256) {
            const int c = e / KB, t = e % KB;
            const int64_t gc = (int64_t)b0 * kT + c;
            xs[c][t] = (gc < q) ? r[(int64_t)cols[gc] * k + k0 + t] : 0.0;
        }
        __syncthreads();
        for (int bb = 0; bb < nb; ++bb) {
            T v[16];
            load16(Ya + (int64_t)(b0 + bb) * kTE, v);
            const double (*xr)[KB] = xs + bb * kT + seg * 16;
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
#pragma unroll
                for (int t = 0; t < KB; ++t) acc[t] = fma((double)v[cc], xr[cc][t], acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < KB; ++t) {
        acc[t] += __shfl_xor(acc[t], 1);
        acc[t] += __shfl_xor(acc[t], 2);
    }
    const int64_t gr = (int64_t)a * kT + row;
    if (seg == 0 && gr < q) {
        double* o = u + (ub_off[i] + gr) * k + k0;
#pragma unroll
        for (int t = 0; t < KB; ++t) o[t] = acc[t];
    }
}

// column pass: z_b = sum_{a >= b} Y_ab^T x_a with x the row-pass output.
// Thread (col, wave) owns 16 rows of one tile column; the four waves are
// summed in LDS at the end.
template <class T, int KB>
__global__ void __launch_bounds__(256) k_tri_col(const int2* __restrict__ tasks,
                                                 const int64_t* __restrict__ t_off,
                                                 const int64_t* __restrict__ qv,
                                                 const int64_t* __restrict__ ub_off,
                                                 const T* __restrict__ Y,
                                                 const double* __restrict__ x, int k, int k0,
                                                 double* __restrict__ z) {
    __shared__ double xs[kXChunk * kT][KB];
    __shared__ double red[4][kT][KB];
    const int2 tk = tasks[blockIdx.x];
    const int i = tk.x, b = tk.y;
    const int64_t q = qv[i];
    const int nt = (int)((q + kT - 1) / kT);
    const int tid = threadIdx.x, col = tid & 63, rs = tid >> 6;
    const T* Yi = Y + t_off[i] + (int64_t)(rs * 16) * kT + col;
    const double* xi = x + ub_off[i] * k + k0;
    double acc[KB];
#pragma unroll
    for (int t = 0; t < KB; ++t) acc[t] = 0.0;
    for (int a0 = b; a0 < nt; a0 += kXChunk) {
        const int na = (nt - a0 < kXChunk) ? nt - a0 : kXChunk;
        __syncthreads();
        for (int e = tid; e < na * kT * KB; e += 256) {
            const int c = e / KB, t = e % KB;
            const int64_t gr = (int64_t)a0 * kT + c;
            xs[c][t] = (gr < q) ? xi[gr * k + t] : 0.0;
        }
        __syncthreads();
        for (int aa = 0; aa < na; ++aa) {
            const int a = a0 + aa;
            const T* src = Yi + ((int64_t)a * (a + 1) / 2 + b) * kTE;
            T v[16];
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) v[rr] = src[rr * kT];
            const double (*xr)[KB] = xs + aa * kT + rs * 16;
#pragma unroll
            for (int rr = 0; rr < 16; ++rr)
#pragma unroll
                for (int t = 0; t < KB; ++t) acc[t] = fma((double)v[rr], xr[rr][t], acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < KB; ++t) red[rs][col][t] = acc[t];
    __syncthreads();
    const int64_t gc = (int64_t)b * kT + col;
    if (rs == 0 && gc < q) {
        double* o = z + (ub_off[i] + gc) * k + k0;
#pragma unroll
        for (int t = 0; t < KB; ++t) o[t] = red[0][col][t] + red[1][col][t] + red[2][col][t] + red[3][col][t];
    }
}

// z[g] = sum over (block entry e containing column g) of w_e u[e]
__global__ void k_gather_sum(int64_t P, int k, const int64_t* __restrict__ gat_off,
                             const int64_t* __restrict__ gat, const double* __restrict__ gat_w,
                             const double* __restrict__ u, double* __restrict__ z) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= P * k) return;
    int64_t g = idx / k;
    int t = (int)(idx % k);
    double s = 0.0;
    for (int64_t e = gat_off[g]; e < gat_off[g + 1]; ++e) s += gat_w[e] * u[gat[e] * k + t];
    z[idx] = s;
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

struct PrecondPlan {
    std::vector<int64_t> row_start, row_cnt;  // rows of each block that are applied
};

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
    // block entry -> global column, and the gather lists
    std::vector<int32_t> blk_cols(ub_off[J]);
    std::vector<std::vector<std::pair<int64_t, double>>> per_col(h.P);
    std::vector<int> mult(h.P, 0);
    for (int i = 0; i < J; ++i) {
        int64_t e = ub_off[i];
        for (int j : h.sten[i])
            for (int c = 0; c < h.p[j]; ++c) {
                int64_t gcol = h.col_off[j] + c;
                blk_cols[e++] = (int32_t)gcol;
                mult[gcol]++;
            }
    }
    PrecondPlan plan;
    plan.row_start.assign(J, 0);
    plan.row_cnt.assign(J, 0);
    for (int i = 0; i < J; ++i) {
        int64_t e = ub_off[i], pos = 0;
        for (int j : h.sten[i]) {
            for (int c = 0; c < h.p[j]; ++c) {
                int64_t gcol = h.col_off[j] + c;
                double w = 1.0;
                bool use = true;
                if (h.precond == RANN_PRECOND_SAS) w = 1.0 / (double)mult[gcol];
                if (h.precond == RANN_PRECOND_RAS) use = (j == i);
                if (use) per_col[gcol].push_back({e, w});
                ++e;
            }
            if (j == i) {
                plan.row_start[i] = pos;
                plan.row_cnt[i] = h.p[j];
            }
            pos += h.p[j];
        }
        if (h.precond != RANN_PRECOND_RAS) {
            plan.row_start[i] = 0;
            plan.row_cnt[i] = h.q[i];
        }
    }
    std::vector<int64_t> gat_off(h.P + 1, 0), gat;
    std::vector<double> gat_w;
    for (int64_t g = 0; g < h.P; ++g) {
        for (auto& pr : per_col[g]) {
            gat.push_back(pr.first);
            gat_w.push_back(pr.second);
        }
        gat_off[g + 1] = (int64_t)gat.size();
    }
    // device copies
    RDD_TRY(dev_alloc(h, &h.d_f_off, J + 1));
    RDD_TRY(dev_alloc(h, &h.d_q, J));
    RDD_TRY(dev_alloc(h, &h.d_ub_off, J + 1));
    RDD_TRY(dev_alloc(h, &h.d_blk_cols, blk_cols.size()));
    RDD_TRY(dev_alloc(h, &h.d_gat_off, gat_off.size()));
    RDD_TRY(dev_alloc(h, &h.d_gat, gat.size()));
    RDD_TRY(dev_alloc(h, &h.d_gat_w, gat_w.size()));
    RDD_TRY(upload(h, h.d_f_off, h.f_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(upload(h, h.d_q, h.q.data(), sizeof(int64_t) * J));
    RDD_TRY(upload(h, h.d_ub_off, ub_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(upload(h, h.d_blk_cols, blk_cols.data(), sizeof(int32_t) * blk_cols.size()));
    RDD_TRY(upload(h, h.d_gat_off, gat_off.data(), sizeof(int64_t) * gat_off.size()));
    if (!gat.empty()) {
        RDD_TRY(upload(h, h.d_gat, gat.data(), sizeof(int64_t) * gat.size()));
        RDD_TRY(upload(h, h.d_gat_w, gat_w.data(), sizeof(double) * gat_w.size()));
    }
    h.ub_total = ub_off[J];

    // packed tiles and the task lists of the two passes (RAS: only the tile
    // columns holding owned unknowns, and the tile rows they need)
    RDD_TRY(plan_tiles(h));
    std::vector<std::pair<int, int2>> rt, ct;  // (work, task)
    for (int i = 0; i < J; ++i) {
        const int nt = h.nt[i];
        if (nt == 0 || plan.row_cnt[i] == 0) continue;
        const int b_lo = (int)(plan.row_start[i] / 64);
        const int b_hi = (int)((plan.row_start[i] + plan.row_cnt[i] - 1) / 64);
        for (int a = b_lo; a < nt; ++a) rt.push_back({a + 1, make_int2(i, a)});
        for (int b = b_lo; b <= b_hi; ++b) ct.push_back({nt - b, make_int2(i, b)});
    }
    auto by_work = [](const std::pair<int, int2>& x, const std::pair<int, int2>& y) {
        return x.first > y.first;
    };
    std::stable_sort(rt.begin(), rt.end(), by_work);
    std::stable_sort(ct.begin(), ct.end(), by_work);
    std::vector<int2> rtv, ctv;
    for (auto& e : rt) rtv.push_back(e.second);
    for (auto& e : ct) ctv.push_back(e.second);
    h.n_row_tasks = (int64_t)rtv.size();
    h.n_col_tasks = (int64_t)ctv.size();
    RDD_TRY(dev_alloc(h, &h.d_row_tasks, rtv.size()));
    RDD_TRY(dev_alloc(h, &h.d_col_tasks, ctv.size()));
    if (!rtv.empty())
        RDD_TRY(upload(h, h.d_row_tasks, rtv.data(), sizeof(int2) * rtv.size()));
    if (!ctv.empty())
        RDD_TRY(upload(h, h.d_col_tasks, ctv.data(), sizeof(int2) * ctv.size()));

    // local Gram blocks (FP64) and their factorisation
    double *d_A = nullptr, *d_W = nullptr;
    RDD_TRY(dev_alloc(h, &d_A, (size_t)h.factor_elems));
    RDD_TRY(dev_alloc(h, &d_W, (size_t)h.factor_elems));
    if (h.precision == RANN_MIXED)
        RDD_TRY(dev_alloc(h, &h.d_M32, (size_t)h.tile_elems));
    else
        RDD_TRY(dev_alloc(h, &h.d_M64, (size_t)h.tile_elems));
    RDD_TRY(local_blocks<double>(h, h.d_H, d_A));
    const int rc = factor_tiles(h, d_A, d_W);
    dev_free(h, d_A);
    dev_free(h, d_W);
    return rc;
}

// u_i = A_i^{-1} r_{N(i)} for every block (the local solves only).  ub holds
// 2 ub_total k doubles: the result, then the row-pass intermediate.
int launch_precond_local(Handle& h, const double* r, int k, double* ub) {
    double* u1 = ub + h.ub_total * k;
    KTimer kt_(h.stream, "k_local_apply");
    for (int k0 = 0; k0 < k;) {
        const int rem = k - k0;
        const int kb = rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
#define RDD_TRI(T, M, KBV)                                                                         \
    do {                                                                                           \
        if (h.n_row_tasks)                                                                         \
            hipLaunchKernelGGL((k_tri_row<T, KBV>), dim3((unsigned)h.n_row_tasks), dim3(256), 0,   \
                               h.stream, h.d_row_tasks, h.d_t_off, h.d_q, h.d_ub_off,              \
                               h.d_blk_cols, M, r, k, k0, u1);                                     \
        if (h.n_col_tasks)                                                                         \
            hipLaunchKernelGGL((k_tri_col<T, KBV>), dim3((unsigned)h.n_col_tasks), dim3(256), 0,   \
                               h.stream, h.d_col_tasks, h.d_t_off, h.d_q, h.d_ub_off, M, u1, k,    \
                               k0, ub);                                                            \
    } while (0)
#define RDD_TRI_ALL(T, M)                   \
    switch (kb) {                           \
        case 8: RDD_TRI(T, M, 8); break;    \
        case 4: RDD_TRI(T, M, 4); break;    \
        case 2: RDD_TRI(T, M, 2); break;    \
        default: RDD_TRI(T, M, 1); break;   \
    }
        if (h.precision == RANN_MIXED) {
            RDD_TRI_ALL(float, h.d_M32);
        } else {
            RDD_TRI_ALL(double, h.d_M64);
        }
#undef RDD_TRI_ALL
#undef RDD_TRI
        k0 += kb;
    }
    kt_.stop();
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

int launch_precond(Handle& h, const double* r, int k, double* z, double* ub) {
    if (h.precond == RANN_PRECOND_NONE) {
        RDD_HIP(hipMemcpyAsync(z, r, sizeof(double) * h.P * k, hipMemcpyDeviceToDevice, h.stream));
        return RANN_OK;
    }
    RDD_TRY(launch_precond_local(h, r, k, ub));
    const int64_t tot = h.P * k;
    hipLaunchKernelGGL(k_gather_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, h.stream,
                       h.P, k, h.d_gat_off, h.d_gat, h.d_gat_w, ub, z);
    RDD_HIP(hipGetLastError());
    return RANN_OK;
}

}  // namespace rdd
