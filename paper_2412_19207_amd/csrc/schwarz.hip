// Overlapping Schwarz preconditioners for H^T H (paper Sec. 3).
//
//   AS : z = sum_i R_i^T A_i^{-1} R_i r
//   RAS: z = sum_i R_i^T D_i A_i^{-1} R_i r,  D_i = the columns subdomain i owns
//   SAS: D_i = 1 / (number of blocks containing the column)
//
// Block i selects the columns of every subdomain in its stencil.  The local
// inverse (factor.hip) is stored explicitly as the symmetric matrix
// A_i^{-1} = D L^{-T} L^{-1} D, so that applying it is a streaming
// matrix-vector product instead of two dependent triangular solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "common.h"

namespace rdd {

template <class T>
int local_blocks(Handle& h, const T* H, T* A_out);
template <class T>
int factor_inverse(Handle& h, T* A, T* M, T* D, int32_t* flags);

namespace {

// u_i = A_i^{-1} r_{N(i)} for the rows [row_lo_i, row_hi_i) of each block; one
// wave per row, lanes stride the row (coalesced), FP64 accumulation.
template <class T, int KB>
__global__ void __launch_bounds__(256) k_local_apply(const int64_t* __restrict__ row_start,
                                                     int64_t nrows_total, int J,
                                                     const int64_t* __restrict__ row_blk_off,
                                                     const int32_t* __restrict__ row_blk,
                                                     const int64_t* __restrict__ f_off,
                                                     const int64_t* __restrict__ qv,
                                                     const int64_t* __restrict__ ub_off,
                                                     const int32_t* __restrict__ blk_cols,
                                                     const T* __restrict__ Minv,
                                                     const double* __restrict__ r, int k, int k0,
                                                     double* __restrict__ u) {
    const int lane = threadIdx.x & 63;
    const int64_t gr = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gr >= nrows_total) return;
    const int i = row_blk[gr];
    const int64_t row = row_start[i] + (gr - row_blk_off[i]);
    const int64_t q = qv[i];
    const T* Mr = Minv + f_off[i] + row * q;
    const int32_t* cols = blk_cols + ub_off[i];
    double acc[KB];
    for (int t = 0; t < KB; ++t) acc[t] = 0.0;
    for (int64_t c = lane; c < q; c += 64) {
        const double mv = (double)Mr[c];
        const double* rc = r + (int64_t)cols[c] * k + k0;
        for (int t = 0; t < KB; ++t) acc[t] = fma(mv, rc[t], acc[t]);
    }
    for (int t = 0; t < KB; ++t)
        for (int off = 32; off > 0; off >>= 1) acc[t] += __shfl_xor(acc[t], off);
    if (lane == 0) {
        double* uo = u + (ub_off[i] + row) * k + k0;
        for (int t = 0; t < KB; ++t) uo[t] = acc[t];
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
        RDD_HIP(hipMemcpy(mu_all.data(), h.d_mu, sizeof(double) * mu_all.size(),
                          hipMemcpyDeviceToHost));
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
    RDD_HIP(hipMemcpy(h.d_f_off, h.f_off.data(), sizeof(int64_t) * (J + 1), hipMemcpyHostToDevice));
    RDD_HIP(hipMemcpy(h.d_q, h.q.data(), sizeof(int64_t) * J, hipMemcpyHostToDevice));
    RDD_HIP(hipMemcpy(h.d_ub_off, ub_off.data(), sizeof(int64_t) * (J + 1), hipMemcpyHostToDevice));
    RDD_HIP(hipMemcpy(h.d_blk_cols, blk_cols.data(), sizeof(int32_t) * blk_cols.size(),
                      hipMemcpyHostToDevice));
    RDD_HIP(hipMemcpy(h.d_gat_off, gat_off.data(), sizeof(int64_t) * gat_off.size(),
                      hipMemcpyHostToDevice));
    if (!gat.empty()) {
        RDD_HIP(hipMemcpy(h.d_gat, gat.data(), sizeof(int64_t) * gat.size(), hipMemcpyHostToDevice));
        RDD_HIP(hipMemcpy(h.d_gat_w, gat_w.data(), sizeof(double) * gat_w.size(),
                          hipMemcpyHostToDevice));
    }
    // applied rows per block (RAS: owned rows only)
    std::vector<int64_t> row_blk_off(J + 1, 0), row_start(J);
    std::vector<int32_t> row_blk;
    for (int i = 0; i < J; ++i) {
        row_start[i] = plan.row_start[i];
        row_blk_off[i + 1] = row_blk_off[i] + plan.row_cnt[i];
        for (int64_t t = 0; t < plan.row_cnt[i]; ++t) row_blk.push_back(i);
    }
    int64_t *d_rs = nullptr, *d_rbo = nullptr;
    int32_t* d_rb = nullptr;
    RDD_TRY(dev_alloc(h, &d_rs, J));
    RDD_TRY(dev_alloc(h, &d_rbo, J + 1));
    RDD_TRY(dev_alloc(h, &d_rb, row_blk.size()));
    RDD_HIP(hipMemcpy(d_rs, row_start.data(), sizeof(int64_t) * J, hipMemcpyHostToDevice));
    RDD_HIP(hipMemcpy(d_rbo, row_blk_off.data(), sizeof(int64_t) * (J + 1), hipMemcpyHostToDevice));
    RDD_HIP(hipMemcpy(d_rb, row_blk.data(), sizeof(int32_t) * row_blk.size(), hipMemcpyHostToDevice));
    h.prec_rows = row_blk_off[J];
    h.d_prec_row_start = d_rs;
    h.d_prec_row_blk_off = d_rbo;
    h.d_prec_row_blk = d_rb;
    h.ub_total = ub_off[J];

    // local Gram blocks, factorisation and explicit inverses
    int32_t* d_flags = nullptr;
    RDD_TRY(dev_alloc(h, &d_flags, 2));
    RDD_HIP(hipMemsetAsync(d_flags, 0, sizeof(int32_t) * 2, h.stream));
    if (h.precision == RANN_MIXED) {
        float *d_A = nullptr, *d_D = nullptr;
        RDD_TRY(dev_alloc(h, &d_A, (size_t)h.factor_elems));
        RDD_TRY(dev_alloc(h, &d_D, (size_t)ub_off[J]));
        RDD_TRY(dev_alloc(h, &h.d_M32, (size_t)h.factor_elems));
        RDD_TRY(local_blocks<float>(h, h.d_H32, d_A));
        RDD_TRY(factor_inverse<float>(h, d_A, h.d_M32, d_D, d_flags));
        RDD_HIP(hipStreamSynchronize(h.stream));
        dev_free(h, d_A);
        dev_free(h, d_D);
    } else {
        double *d_A = nullptr, *d_D = nullptr;
        RDD_TRY(dev_alloc(h, &d_A, (size_t)h.factor_elems));
        RDD_TRY(dev_alloc(h, &d_D, (size_t)ub_off[J]));
        RDD_TRY(dev_alloc(h, &h.d_M64, (size_t)h.factor_elems));
        RDD_TRY(local_blocks<double>(h, h.d_H, d_A));
        RDD_TRY(factor_inverse<double>(h, d_A, h.d_M64, d_D, d_flags));
        RDD_HIP(hipStreamSynchronize(h.stream));
        dev_free(h, d_A);
        dev_free(h, d_D);
    }
    int32_t flags[2] = {0, 0};
    RDD_HIP(hipMemcpy(flags, d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    dev_free(h, d_flags);
    h.shifts = flags[0];
    if (flags[1] != 0) {
        set_error("a local Schwarz block is not positive definite even after diagonal shifts");
        return RANN_EBREAKDOWN;
    }
    return RANN_OK;
}

// u_i = A_i^{-1} r_{N(i)} for every block (the local solves only)
int launch_precond_local(Handle& h, const double* r, int k, double* ub) {
    const unsigned grid = (unsigned)((h.prec_rows + 3) / 4);
    KTimer kt_(h.stream, "k_local_apply");
    for (int k0 = 0; k0 < k;) {
        int rem = k - k0;
        int kb = rem >= 32 ? 32 : rem >= 16 ? 16 : rem >= 8 ? 8 : rem >= 4 ? 4 : rem >= 2 ? 2 : 1;
#define RDD_LA(T, M, KBV)                                                                         \
    hipLaunchKernelGGL((k_local_apply<T, KBV>), dim3(grid), dim3(256), 0, h.stream,               \
                       h.d_prec_row_start, h.prec_rows, h.geo.J, h.d_prec_row_blk_off,            \
                       h.d_prec_row_blk, h.d_f_off, h.d_q, h.d_ub_off, h.d_blk_cols, M, r, k, k0, ub)
#define RDD_LA_ALL(T, M)                     \
    switch (kb) {                            \
        case 32: RDD_LA(T, M, 32); break;    \
        case 16: RDD_LA(T, M, 16); break;    \
        case 8: RDD_LA(T, M, 8); break;      \
        case 4: RDD_LA(T, M, 4); break;      \
        case 2: RDD_LA(T, M, 2); break;      \
        default: RDD_LA(T, M, 1); break;     \
    }
        if (h.precision == RANN_MIXED) {
            RDD_LA_ALL(float, h.d_M32);
        } else {
            RDD_LA_ALL(double, h.d_M64);
        }
#undef RDD_LA_ALL
#undef RDD_LA
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
