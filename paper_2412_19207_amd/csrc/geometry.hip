// Support binning, window partition of unity and operator coefficients.
//
// Paper Sec. 2 (local spaces glued by window functions that sum to one),
// Sec. 5 Example 1 (window = product of [1 + cos(pi (x_i - mu_i)/sigma_i)]^2,
// normalised by the sum over subdomains; inputs normalised per subdomain), and
// eqs. (sum)/(system) (rows A[L w_j phi_k](x_i)).
//
// Every kernel here is integer or light FP64 work; the binning is
// deterministic (ballot compaction in point order), so the row sets S_j are
// sorted and identical from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"

namespace rdd {

namespace {

__device__ inline void sub_coords(const Geo& g, int j, int* c) {
    for (int i = 0; i < g.d; ++i) {
        c[i] = j % g.l[i];
        j /= g.l[i];
    }
}

__device__ inline bool inside(const Geo& g, const double* mu, const int* c, const double* x) {
    bool in = true;
    for (int i = 0; i < g.d; ++i) {
        double m = mu[g.mu_off[i] + c[i]];
        in = in && (fabs(x[i] - m) < g.sigma[i] * kEdge);
    }
    return in;
}

// workgroup (j, chunk) scans the points of one contiguous chunk of the point
// range for subdomain j; pass 0 counts (count[j * nchunk + chunk]), pass 1
// writes the sorted row list by ballot compaction from the chunk's offset
// off[j * nchunk + chunk] (chunks in order, so S_j stays ascending)
template <bool kFill>
__global__ void __launch_bounds__(256) k_bin(Geo g, const double* __restrict__ mu,
                                             const double* __restrict__ X, int64_t n,
                                             int64_t* __restrict__ count,
                                             const int64_t* __restrict__ off,
                                             int32_t* __restrict__ rows,
                                             int32_t* __restrict__ pair_sub) {
    const int j = blockIdx.x;
    const int nchunk = gridDim.y;
    const int64_t lo = n * blockIdx.y / nchunk, hi = n * (blockIdx.y + 1) / nchunk;
    int c[kMaxDim];
    sub_coords(g, j, c);
    __shared__ int wave_cnt[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t base = kFill ? off[(int64_t)j * nchunk + blockIdx.y] : 0;
    for (int64_t p0 = lo; p0 < hi; p0 += 256) {
        int64_t p = p0 + threadIdx.x;
        bool in = false;
        if (p < hi) {
            double x[kMaxDim];
            for (int i = 0; i < g.d; ++i) x[i] = X[p * g.d + i];
            in = inside(g, mu, c, x);
        }
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
            int64_t pos = base + before + __popcll(lower);
            rows[pos] = (int32_t)p;
            pair_sub[pos] = j;
        }
        base += total;
        __syncthreads();
    }
    if (!kFill && threadIdx.x == 0) count[(int64_t)j * nchunk + blockIdx.y] = base;
}

// number of subdomains whose support contains each point (a tensor product of
// per-dimension ranges, since the support test separates by dimension)
__global__ void k_cover_count(Geo g, const double* __restrict__ mu, const double* __restrict__ X,
                              int64_t n, int64_t* __restrict__ cnt) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t tot = 1;
    for (int i = 0; i < g.d; ++i) {
        double x = X[p * g.d + i];
        int ci = 0;
        for (int cc = 0; cc < g.l[i]; ++cc)
            ci += (fabs(x - mu[g.mu_off[i] + cc]) < g.sigma[i] * kEdge) ? 1 : 0;
        tot *= ci;
    }
    cnt[p] = tot;
}

__device__ inline int64_t lower_bound_i32(const int32_t* a, int64_t n, int32_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// pair ids of each point in ascending subdomain order
__global__ void k_cover_fill(Geo g, const double* __restrict__ mu, const double* __restrict__ X,
                             int64_t n, const int64_t* __restrict__ cover_off,
                             const int64_t* __restrict__ row_off,
                             const int32_t* __restrict__ rows, int64_t* __restrict__ cover) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int lo[kMaxDim], cnt[kMaxDim];
    for (int i = 0; i < g.d; ++i) {
        double x = X[p * g.d + i];
        lo[i] = -1;
        cnt[i] = 0;
        for (int cc = 0; cc < g.l[i]; ++cc) {
            if (fabs(x - mu[g.mu_off[i] + cc]) < g.sigma[i] * kEdge) {
                if (lo[i] < 0) lo[i] = cc;
                cnt[i]++;
            }
        }
    }
    int64_t total = cover_off[p + 1] - cover_off[p];
    int idx[kMaxDim] = {0, 0, 0, 0};
    for (int64_t t = 0; t < total; ++t) {
        // subdomain with tensor coordinates lo + idx; dimension 0 fastest -> ascending j
        int j = 0;
        for (int i = g.d - 1; i >= 0; --i) j = j * g.l[i] + lo[i] + idx[i];
        int64_t b = row_off[j], e = row_off[j + 1];
        cover[cover_off[p] + t] = b + lower_bound_i32(rows + b, e - b, (int32_t)p);
        for (int i = 0; i < g.d; ++i) {
            if (++idx[i] < cnt[i]) break;
            idx[i] = 0;
        }
    }
}

// raw window of subdomain j at x and its derivatives in x
__device__ inline void raw_window(const Geo& g, const double* mu, int j, const double* x,
                                  double& w, double* gw, double* hw) {
    int c[kMaxDim];
    sub_coords(g, j, c);
    double v[kMaxDim], d1[kMaxDim], d2[kMaxDim];
    for (int i = 0; i < g.d; ++i) {
        double tau = (x[i] - mu[g.mu_off[i] + c[i]]) * g.inv_sigma[i];
        double s, co;
        sincospi(tau, &s, &co);
        double opc = 1.0 + co;
        v[i] = opc * opc;
        d1[i] = -2.0 * M_PI * opc * s * g.inv_sigma[i];
        d2[i] = 2.0 * M_PI * M_PI * (s * s - opc * co) * g.inv_sigma[i] * g.inv_sigma[i];
    }
    w = 1.0;
    for (int i = 0; i < g.d; ++i) w *= v[i];
    for (int i = 0; i < g.d; ++i) {
        double other = 1.0;
        for (int q = 0; q < g.d; ++q)
            if (q != i) other *= v[q];
        gw[i] = d1[i] * other;
        hw[i] = d2[i] * other;
    }
}

// one thread per (point, subdomain) pair: window w_j = w^_j / S with the
// quotient rule, multiplier M = L w_j, and the operator coefficients
__global__ void k_pair_records(Geo g, const double* __restrict__ mu, const double* __restrict__ X,
                               int64_t n_int, const double* __restrict__ a,
                               const double* __restrict__ beta, const double* __restrict__ cc,
                               const double* __restrict__ Lfun, const double* __restrict__ Lq,
                               double lambda_B, int value_only, int64_t pairs,
                               const int32_t* __restrict__ rows,
                               const int32_t* __restrict__ pair_sub,
                               const int64_t* __restrict__ cover_off,
                               const int64_t* __restrict__ cover, double* __restrict__ rec) {
    int64_t pid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pid >= pairs) return;
    const int d = g.d;
    const int j = pair_sub[pid];
    const int64_t r = rows[pid];
    double x[kMaxDim];
    for (int i = 0; i < d; ++i) x[i] = X[r * d + i];
    double S = 0.0, Sg[kMaxDim] = {0, 0, 0, 0}, Sh[kMaxDim] = {0, 0, 0, 0};
    double w = 0.0, wg[kMaxDim] = {0, 0, 0, 0}, wh[kMaxDim] = {0, 0, 0, 0};
    for (int64_t t = cover_off[r]; t < cover_off[r + 1]; ++t) {
        int jj = pair_sub[cover[t]];
        double v, gv[kMaxDim], hv[kMaxDim];
        raw_window(g, mu, jj, x, v, gv, hv);
        S += v;
        for (int i = 0; i < d; ++i) {
            Sg[i] += gv[i];
            Sh[i] += hv[i];
        }
        if (jj == j) {
            w = v;
            for (int i = 0; i < d; ++i) {
                wg[i] = gv[i];
                wh[i] = hv[i];
            }
        }
    }
    const double om = w / S;
    double omg[kMaxDim], omh[kMaxDim];
    for (int i = 0; i < d; ++i) {
        omg[i] = (wg[i] - om * Sg[i]) / S;
        omh[i] = (wh[i] - 2.0 * omg[i] * Sg[i] - om * Sh[i]) / S;
    }
    double* o = rec + pid * kPairRec;
    int cj[kMaxDim];
    sub_coords(g, j, cj);
    for (int i = 0; i < kMaxDim; ++i)
        o[kRecX + i] = (i < d) ? (x[i] - mu[g.mu_off[i] + cj[i]]) * g.inv_sigma[i] : 0.0;
    o[kRecW] = om;
    for (int i = 0; i < kMaxDim; ++i) {
        o[kRecP1 + i] = 0.0;
        o[kRecP2 + i] = 0.0;
    }
    o[14] = 0.0;
    o[15] = 0.0;
    if (value_only) {
        double L = Lq ? Lq[r] : 1.0;
        o[kRecP0] = L * om;
        return;
    }
    // multiplier M = L w_j (product rule)
    double M = om, Mg[kMaxDim], Mh[kMaxDim];
    for (int i = 0; i < d; ++i) {
        Mg[i] = omg[i];
        Mh[i] = omh[i];
    }
    if (Lfun) {
        const double* Lr = Lfun + r * (1 + 2 * d);
        double L = Lr[0];
        for (int i = 0; i < d; ++i) {
            double Li = Lr[1 + i], Lii = Lr[1 + d + i];
            Mh[i] = Lii * om + 2.0 * Li * omg[i] + L * omh[i];
            Mg[i] = Li * om + L * omg[i];
        }
        M = L * om;
    }
    if (r < n_int) {
        double P0 = cc[r] * M;
        for (int i = 0; i < d; ++i) {
            double ai = a[r * d + i], bi = beta[r * d + i];
            P0 += -ai * Mh[i] + bi * Mg[i];
            o[kRecP1 + i] = -2.0 * ai * Mg[i] + bi * M;
            o[kRecP2 + i] = -ai * M;
        }
        o[kRecP0] = P0;
    } else {
        o[kRecP0] = lambda_B * M;
    }
}

// -------------------------------------------------------------- prefix sums
constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(256) k_scan_block(const int64_t* __restrict__ in, int64_t n,
                                                    int64_t* __restrict__ out,
                                                    int64_t* __restrict__ block_sums) {
    __shared__ int64_t s[256];
    int64_t base = blockIdx.x * (int64_t)kScanBlock;
    int64_t v[4];
    int64_t local = 0;
    for (int t = 0; t < 4; ++t) {
        int64_t i = base + threadIdx.x * 4 + t;
        v[t] = (i < n) ? in[i] : 0;
        local += v[t];
    }
    s[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int64_t add = (threadIdx.x >= off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t run = s[threadIdx.x] - local;  // exclusive within block
    for (int t = 0; t < 4; ++t) {
        int64_t i = base + threadIdx.x * 4 + t;
        if (i < n) out[i + 1] = run + v[t];
        run += v[t];
    }
    if (threadIdx.x == 255) block_sums[blockIdx.x] = s[255];
}

__global__ void __launch_bounds__(256) k_scan_sums(int64_t* __restrict__ sums, int64_t nb) {
    // single workgroup, sequential over chunks of 256 (nb is small)
    __shared__ int64_t s[256];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        int64_t i = b0 + threadIdx.x;
        int64_t v = (i < nb) ? sums[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            int64_t add = (threadIdx.x >= off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + s[threadIdx.x] - v;  // exclusive
        __syncthreads();
        if (threadIdx.x == 255) carry += s[255];
        __syncthreads();
    }
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ sums) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i == 0) out[0] = 0;
    if (i < n) out[i + 1] += sums[i / kScanBlock];
}

}  // namespace

int exclusive_scan_i64(Handle& h, const int64_t* in, int64_t* out, int64_t n) {
    if (n == 0) {
        RDD_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), h.stream));
        return RANN_OK;
    }
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    int64_t* sums = nullptr;
    RDD_TRY(dev_alloc(h, &sums, (size_t)nb));
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(256), 0, h.stream, in, n, out, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, h.stream, sums, nb);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h.stream, out, n,
                       sums);
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    dev_free(h, sums);
    return RANN_OK;
}

int bin_points(Handle& h, const double* X, int64_t n, PointSet& ps) {
    const Geo& g = h.geo;
    ps.n = n;
    // chunks of the point range per subdomain, about 4096 points each
    const int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(64, (n + 4095) / 4096));
    const size_t ncell = (size_t)g.J * nchunk;
    int64_t* d_cnt = nullptr;
    RDD_TRY(dev_alloc(h, &d_cnt, ncell));
    hipLaunchKernelGGL((k_bin<false>), dim3(g.J, nchunk), dim3(256), 0, h.stream, g, h.d_mu, X, n, d_cnt,
                       nullptr, nullptr, nullptr);
    RDD_HIP(hipGetLastError());
    std::vector<int64_t> cnt(ncell), coff(ncell);
    RDD_TRY(download(h, cnt.data(), d_cnt, sizeof(int64_t) * ncell));
    RDD_HIP(hipStreamSynchronize(h.stream));
    ps.row_off.assign(g.J + 1, 0);
    for (int j = 0; j < g.J; ++j) {
        int64_t o = ps.row_off[j];
        for (int c = 0; c < nchunk; ++c) {
            coff[(size_t)j * nchunk + c] = o;
            o += cnt[(size_t)j * nchunk + c];
        }
        ps.row_off[j + 1] = o;
    }
    ps.pairs = ps.row_off[g.J];
    if (ps.pairs >= (int64_t)INT32_MAX) {
        set_error("too many (point, subdomain) pairs");
        return RANN_EINVAL;
    }
    RDD_TRY(dev_alloc(h, &ps.d_row_off, (size_t)g.J + 1));
    RDD_TRY(dev_alloc(h, &ps.d_rows, (size_t)ps.pairs));
    RDD_TRY(dev_alloc(h, &ps.d_pair_sub, (size_t)ps.pairs));
    RDD_TRY(upload(h, ps.d_row_off, ps.row_off.data(), sizeof(int64_t) * (g.J + 1)));
    RDD_TRY(upload(h, d_cnt, coff.data(), sizeof(int64_t) * ncell));  // chunk offsets
    hipLaunchKernelGGL((k_bin<true>), dim3(g.J, nchunk), dim3(256), 0, h.stream, g, h.d_mu, X, n, nullptr,
                       d_cnt, ps.d_rows, ps.d_pair_sub);
    RDD_HIP(hipGetLastError());
    dev_free(h, d_cnt);
    // point -> pairs
    int64_t* d_cc = nullptr;
    RDD_TRY(dev_alloc(h, &d_cc, (size_t)n));
    RDD_TRY(dev_alloc(h, &ps.d_cover_off, (size_t)n + 1));
    unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_cover_count, dim3(nb), dim3(256), 0, h.stream, g, h.d_mu, X, n, d_cc);
    RDD_HIP(hipGetLastError());
    RDD_TRY(exclusive_scan_i64(h, d_cc, ps.d_cover_off, n));
    int64_t total = 0;
    RDD_TRY(download(h, &total, ps.d_cover_off + n, sizeof(int64_t)));
    // uncovered points: detected through the per-point count
    std::vector<int64_t> cc_host;
    RDD_HIP(hipStreamSynchronize(h.stream));
    if (total != ps.pairs) {
        set_error("internal: pair count mismatch in binning");
        return RANN_EDEVICE;
    }
    {
        // minimum cover must be >= 1: read the counts back (integers, cheap)
        cc_host.resize(n);
        RDD_TRY(download(h, cc_host.data(), d_cc, sizeof(int64_t) * n));
        int64_t mx = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (cc_host[i] == 0) {
                set_error("point " + std::to_string(i) + " lies outside every subdomain support");
                dev_free(h, d_cc);
                return RANN_EINVAL;
            }
            mx = cc_host[i] > mx ? cc_host[i] : mx;
        }
        ps.max_cover = (int)mx;
    }
    dev_free(h, d_cc);
    RDD_TRY(dev_alloc(h, &ps.d_cover, (size_t)ps.pairs));
    hipLaunchKernelGGL(k_cover_fill, dim3(nb), dim3(256), 0, h.stream, g, h.d_mu, X, n,
                       ps.d_cover_off, ps.d_row_off, ps.d_rows, ps.d_cover);
    RDD_HIP(hipGetLastError());
    RDD_HIP(hipStreamSynchronize(h.stream));
    return RANN_OK;
}

int pair_records(Handle& h, const double* X, int64_t n_int, const double* a, const double* beta,
                 const double* c, const double* Lfun, int64_t n_all, double lambda_B,
                 bool value_rows_only, const double* Lq, PointSet& ps) {
    (void)n_all;
    RDD_TRY(dev_alloc(h, &ps.d_rec, (size_t)ps.pairs * kPairRec));
    unsigned nb = (unsigned)((ps.pairs + 255) / 256);
    if (ps.pairs > 0) {
        hipLaunchKernelGGL(k_pair_records, dim3(nb), dim3(256), 0, h.stream, h.geo, h.d_mu, X,
                           n_int, a, beta, c, Lfun, Lq, lambda_B, value_rows_only ? 1 : 0,
                           ps.pairs, ps.d_rows, ps.d_pair_sub, ps.d_cover_off, ps.d_cover,
                           ps.d_rec);
        RDD_HIP(hipGetLastError());
    }
    return RANN_OK;
}

}  // namespace rdd
