// Linearisation of a semilinear reaction for Picard and Newton iterations
// (paper Sec. 2, the remark after eq. (sum): for a nonlinear operator each step
// of a Picard or Newton iteration solves one linear least-squares problem).
//
// Problem A[u] + g(u) = f with the linear operator A of the handle's
// description (reaction c0) and g(u) = sum_p gamma_p u^p.  About the current
// values u_k at the interior collocation points:
//   Newton: reaction c0 + g'(u_k), interior right-hand side f - g(u_k) + g'(u_k) u_k
//   Picard: reaction c0 + q(u_k),  interior right-hand side f - gamma_0,
//           with g(u) = gamma_0 + u q(u)
// The next step assembles the linear problem with these data.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "common.h"

namespace rdd {

namespace {

constexpr int kIncBlocks = 256;

struct Poly {
    double c[RANN_MAX_GAMMA];
    int n;
};

__global__ void __launch_bounds__(256) k_linearize(int64_t n, Poly g, int mode, const double* __restrict__ u,
                                                   const double* __restrict__ c0, const double* __restrict__ f,
                                                   double* __restrict__ c_out, double* __restrict__ f_out) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = u[i];
    if (mode == RANN_LIN_NEWTON) {
        double gv = 0.0, gp = 0.0;  // g and g' by Horner's rule
        for (int p = g.n - 1; p >= 0; --p) {
            gp = fma(gp, x, gv);
            gv = fma(gv, x, g.c[p]);
        }
        c_out[i] = c0[i] + gp;
        f_out[i] = f[i] - gv + gp * x;
    } else {
        double q = 0.0;  // q(u) = sum_{p>=1} gamma_p u^{p-1}
        for (int p = g.n - 1; p >= 1; --p) q = fma(q, x, g.c[p]);
        c_out[i] = c0[i] + q;
        f_out[i] = f[i] - g.c[0];
    }
}

// partial[b] = sum over this block's entries of (u - up)^2, partial[nb + b] of u^2
__global__ void __launch_bounds__(256) k_inc_part(int64_t n, const double* __restrict__ u,
                                                  const double* __restrict__ up, double* __restrict__ part) {
    __shared__ double s1[256], s2[256];
    double a1 = 0.0, a2 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double d = u[i] - up[i];
        a1 = fma(d, d, a1);
        a2 = fma(u[i], u[i], a2);
    }
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s1[threadIdx.x] += s1[threadIdx.x + w];
            s2[threadIdx.x] += s2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s1[0];
        part[gridDim.x + blockIdx.x] = s2[0];
    }
}

}  // namespace

int linearize(Handle& h, const double* u, const double* c0, const double* f, int64_t n, const double* gamma,
              int n_gamma, int mode, double* c_out, double* f_out, const double* u_prev, double* inc) {
    Poly g{};
    g.n = n_gamma;
    for (int p = 0; p < n_gamma; ++p) g.c[p] = gamma[p];
    if (n > 0) {
        hipLaunchKernelGGL(k_linearize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h.stream, n, g, mode, u,
                           c0, f, c_out, f_out);
        RDD_HIP(hipGetLastError());
    }
    if (!inc) return RANN_OK;
    *inc = 0.0;
    if (!u_prev || n == 0) return RANN_OK;
    double* part = nullptr;
    RDD_TRY(dev_alloc(h, &part, 2 * (size_t)kIncBlocks));
    hipLaunchKernelGGL(k_inc_part, dim3(kIncBlocks), dim3(256), 0, h.stream, n, u, u_prev, part);
    std::vector<double> ph(2 * kIncBlocks);
    int rc = (hipGetLastError() == hipSuccess) ? RANN_OK : RANN_EDEVICE;
    if (rc == RANN_OK) rc = download(h, ph.data(), part, sizeof(double) * 2 * kIncBlocks);
    if (rc == RANN_OK && hipStreamSynchronize(h.stream) != hipSuccess) rc = RANN_EDEVICE;
    dev_free(h, part);
    if (rc != RANN_OK) {
        set_error("linearize: device error");
        return rc;
    }
    double d2 = 0.0, u2 = 0.0;
    for (int b = 0; b < kIncBlocks; ++b) {
        d2 += ph[b];
        u2 += ph[kIncBlocks + b];
    }
    *inc = u2 > 0.0 ? std::sqrt(d2 / u2) : std::sqrt(d2);
    return RANN_OK;
}

}  // namespace rdd
