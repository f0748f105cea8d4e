// Pieces shared by the CG kernels and the normal-matrix product, which can
// finish the previous CG iteration on the fly: with the direction update
// p_new = z + beta p (beta = <r, z> / rho, per right-hand side, only where the
// right-hand side is still active) folded into the product s = N p_new, the
// separate direction-update launch disappears inside a check window.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rdd {

// res[t] = sum over the nparts partials part[b * k + k0 + t], for t < kb:
// the 256 / kb threads of each t read 32 partials per round, all in flight
// together (the last round's surplus loads re-read the last partial and are
// discarded, so that no load waits behind a branch), into 8 accumulators;
// accumulators and threads meet in a fixed-order tree
__device__ inline void sum_partials_kb(const double* part, int nparts, int k, int k0, int kb, double* res,
                                       double* sh) {
    constexpr int kR = 32;
    const int per = 256 / kb;
    const int t = threadIdx.x % kb, ro = threadIdx.x / kb;
    double acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = 0.0;
    if (ro < per) {
        for (int b = ro; b < nparts; b += kR * per) {
            double v[kR];
#pragma unroll
            for (int u = 0; u < kR; ++u) {
                const int bu = b + u * per;
                v[u] = part[(int64_t)(bu < nparts ? bu : nparts - 1) * k + k0 + t];
            }
#pragma unroll
            for (int u = 0; u < kR; ++u)
                if (b + u * per >= nparts) v[u] = 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += (v[u] + v[u + 8]) + (v[u + 16] + v[u + 24]);
        }
    }
    const double a = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    if (kb <= 64 && (kb & (kb - 1)) == 0) {
        // the lanes of a wave that share t differ in the bits from kb up: a
        // butterfly over those, then the four waves through LDS
        double w = a;
        for (int off = 32; off >= kb; off >>= 1) w += __shfl_xor(w, off);
        const int lane = threadIdx.x & 63;
        if (lane < kb) sh[(threadIdx.x >> 6) * kb + lane] = w;
        __syncthreads();
        if (threadIdx.x < kb)
            res[threadIdx.x] = (sh[threadIdx.x] + sh[kb + threadIdx.x]) +
                               (sh[2 * kb + threadIdx.x] + sh[3 * kb + threadIdx.x]);
        __syncthreads();
        return;
    }
    sh[threadIdx.x] = (ro < per) ? a : 0.0;
    __syncthreads();
    for (int st = 1; st < per; st <<= 1) {
        if (ro < per && (ro % (2 * st)) == 0 && ro + st < per) sh[threadIdx.x] += sh[threadIdx.x + st * kb];
        __syncthreads();
    }
    if (threadIdx.x < kb) res[threadIdx.x] = sh[threadIdx.x];
    __syncthreads();
}

// the previous iteration's direction update and bookkeeping, carried by a
// normal-matrix product (pprev == nullptr: plain product of x)
struct PUpd {
    const double* pprev;     // p of the previous iteration
    const double* z;         // preconditioned residual
    double* pcur;            // p of this iteration (rows of the product's own slab rows)
    const double* partB;     // partials of <r, r>  (nB workgroups)
    const double* partC;     // partials of <r, z>  (nC workgroups)
    int nB;
    int nC;
    const double* bn2;       // ||rhs||^2
    const double* tol2;      // tolerance^2
    const double* rho_in;    // rho of the previous iteration
    double* rho_out;
    const int32_t* act_in;   // activity of the previous iteration
    int32_t* act_out;
    int32_t* iters;
    double* rres;            // recurrence residual
};

// beta and activity for the right-hand sides k0 .. k0 + kb - 1 into
// beta_s / act_s (shared); workgroup 0 also writes the bookkeeping.  The
// per-right-hand-side state is loaded before the partials are added.
__device__ inline void pupd_begin(const PUpd& u, int k, int k0, int kb, double* beta_s, int* act_s, double* rz_s,
                                  double* rr_s, double* sh) {
    const bool lead = threadIdx.x < kb;
    const int t = k0 + (lead ? (int)threadIdx.x : 0);
    const int act = u.act_in[t];
    const double rho = u.rho_in[t];
    const double tl2 = u.tol2[t], b2 = u.bn2[t];
    sum_partials_kb(u.partC, u.nC, k, k0, kb, rz_s, sh);
    if (blockIdx.x == 0) sum_partials_kb(u.partB, u.nB, k, k0, kb, rr_s, sh);
    if (lead) {
        const double rz = rz_s[threadIdx.x];
        beta_s[threadIdx.x] = act ? rz / rho : 0.0;
        act_s[threadIdx.x] = act;
        if (blockIdx.x == 0) {
            const double rr = rr_s[threadIdx.x];
            u.rho_out[t] = act ? rz : rho;
            u.act_out[t] = (act && !(rr <= tl2 * b2)) ? 1 : 0;
            if (act) {
                u.iters[t] += 1;
                u.rres[t] = sqrt(rr / b2);
            }
        }
    }
    __syncthreads();
}

// p_new at flat index gi (right-hand side slot tl of the chunk)
__device__ __forceinline__ double pupd_value(const PUpd& u, int64_t gi, int tl, const double* beta_s,
                                             const int* act_s) {
    const double pp = u.pprev[gi];
    return act_s[tl] ? fma(beta_s[tl], pp, u.z[gi]) : pp;
}

}  // namespace rdd
