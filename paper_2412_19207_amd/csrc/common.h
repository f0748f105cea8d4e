// Shared definitions of the RaNN overlapping-Schwarz library (host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rann_dd.h"

namespace rdd {

constexpr int kMaxDim = 4;
constexpr int kMaxWidth = 1024;     // hidden width limit per subdomain
constexpr int kPairRec = 16;        // doubles per (point, subdomain) record
// pair record layout: [0..3] normalised coordinates, [4] window value w_j,
// [5] P0, [6..9] P1_i, [10..13] P2_i (operator row = P0 t + (sum P1_i rho_i) s
// - 2 (sum P2_i rho_i^2) t s with t = tanh z, s = 1 - t^2, rho_i = R_i / sigma_i)
constexpr int kRecX = 0, kRecW = 4, kRecP0 = 5, kRecP1 = 6, kRecP2 = 10;
constexpr double kEdge = 1.0 - 1e-12;  // strict support test factor

// inner hidden layers of every subdomain network (paper eq. (net)); n = 0: one
// hidden layer acting on the normalised input
constexpr int kMaxInner = 3, kMaxInnerWidth = 64;

// The command processor hands workgroup b of a launch to XCD b % 8 (each XCD
// with its own L2).  xcd_task(b, n) numbers the n workgroups so that each XCD
// takes one contiguous eighth of a task list: tasks of neighbouring
// subdomains, which read the same rows of the vectors, then share an L2.  A
// bijection of 0 .. n - 1.
__device__ __forceinline__ int xcd_task(int b, int n) {
    constexpr int kXcd = 8;
    const int x = b % kXcd, l = b / kXcd;
    const int per = n / kXcd, rem = n % kXcd;
    return x * per + (x < rem ? x : rem) + l;
}
struct DeepNet {             // passed by value to kernels
    int n = 0;               // inner layers
    int w[kMaxInner + 1] = {0, 0, 0, 0};  // w[0] = d, then the inner widths
    int lo[kMaxInner] = {0, 0, 0};        // offset of layer i in a subdomain's packed weights
    int stride = 0;          // packed weights per subdomain
};

struct Geo {                 // passed by value to kernels
    int d;
    int l[kMaxDim];
    int mu_off[kMaxDim];     // offset of dimension i's centres in the mu array
    double sigma[kMaxDim];
    double inv_sigma[kMaxDim];
    int J;
};

// A point set binned into the subdomain supports: the row sets S_j, the
// (row -> pairs) map, and one record per (point, subdomain) pair.
struct PointSet {
    int64_t n = 0;                 // points
    int64_t pairs = 0;             // sum_j n_j
    std::vector<int64_t> row_off;  // host J+1
    int64_t* d_row_off = nullptr;  // device J+1
    int32_t* d_rows = nullptr;     // device pairs: global row of each pair (S_j concatenated)
    int32_t* d_pair_sub = nullptr; // device pairs: subdomain of each pair
    int64_t* d_cover_off = nullptr;// device n+1: pairs of each point (CSR)
    int64_t* d_cover = nullptr;    // device: pair ids, ascending subdomain order
    double* d_rec = nullptr;       // device pairs x kPairRec
    int max_cover = 0;
};

// What one application of the local solves and their sum computes: the tile
// tasks, the input column of each block entry, and the gather lists that add
// the used block entries into each global column.
struct ApplyPlan {
    int4* d_tile_tasks = nullptr;  // (block, tile row, tile column) of the local solves
    int64_t n_tile_tasks = 0;
    int2* d_row_tasks = nullptr;   // (block, tile row), longest first (triangular factor)
    int64_t n_row_tasks = 0;
    int2* d_col_tasks = nullptr;   // (block, tile of the result that is used), longest first
    int64_t n_col_tasks = 0;
    int32_t* d_blk_cols = nullptr; // sum q_i: input column of each block entry
    // gather form of the sum: for each global column, the (block entry) list
    int64_t* d_gat_off = nullptr;  // P+1
    int64_t* d_gat = nullptr;      // entries
    double* d_gat_w = nullptr;     // weights (AS 1, SAS 1/mult, RAS 1 on owned entries only)
    // the same sum by subdomain: the columns of subdomain j are the weighted sum
    // of contiguous segments of the block results (one per block that uses j)
    int64_t* d_seg_off = nullptr;  // J+1
    int64_t* d_seg_src = nullptr;  // first block entry of each segment
    double* d_seg_w = nullptr;     // its weight
    // blocks with a used result, widest first, and the most 64-wide tiles per edge
    int32_t* d_blk_list = nullptr;
    int64_t n_blk_list = 0;
    int max_nt = 0;
};

struct Handle {
    hipStream_t stream = nullptr;
    int device = 0;
    Geo geo{};
    double lambda_B = 1.0;
    int precision = RANN_FP64, stencil = RANN_STENCIL_FULL, precond = RANN_PRECOND_AS;
    int64_t n_int = 0, n_bnd = 0, N = 0;
    std::vector<int32_t> m;        // host widths
    std::vector<int64_t> m_off;    // host J+1
    int64_t sum_m = 0;
    double* d_mu = nullptr;        // device sum(l)
    double* d_Rf = nullptr;        // device sum_m x 4 (padded)
    double* d_bf = nullptr;        // device sum_m
    DeepNet deep;                  // inner layers (deep.n == 0: none)
    double* d_inner = nullptr;     // device J x deep.stride packed inner weights
    double* d_Rl = nullptr;        // device sum_m x w_last: last-layer weights (deep.n > 0)
    int64_t* d_m_off = nullptr;    // device J+1
    int32_t* d_m = nullptr;        // device J
    PointSet pts;                  // collocation points

    // PCA
    bool pca_done = false;
    std::vector<int32_t> p;        // host J
    std::vector<int64_t> col_off;  // host J+1
    std::vector<int64_t> v_off;    // host J+1 (sum m_j p_j)
    std::vector<int64_t> h_off;    // host J+1 (sum n_j p_j)
    int64_t P = 0, nnz = 0;
    int32_t* d_p = nullptr;
    int64_t* d_col_off = nullptr;
    int64_t* d_v_off = nullptr;
    int64_t* d_h_off = nullptr;
    double* d_eig = nullptr;       // sum m_j, descending
    double* d_V = nullptr;         // sum m_j p_j
    double* d_H = nullptr;         // nnz FP64
    float* d_H32 = nullptr;        // nnz FP32 (mixed precision with FP32 local Gram blocks only)
    float* d_G32 = nullptr;        // their Gram blocks (set-up only)
    double* d_T = nullptr;         // tanh of every (pair, feature) from the PCA's value matrices,
    int64_t* d_T_off = nullptr;    // n_j x m_j per subdomain, kept for the operator rows (set-up only)

    // Schwarz blocks
    std::vector<std::vector<int>> sten;  // stencil of each block (ascending)
    std::vector<int64_t> q;        // block sizes
    std::vector<int64_t> f_off;    // J+1 offsets of the q_i^2 set-up work arrays
    int64_t factor_elems = 0;      // sum q_i^2
    int max_q = 0;
    std::vector<int32_t> nt;       // 64-wide tiles per edge of each block
    std::vector<int64_t> t_off;    // J+1 offsets of the packed lower tiles
    int64_t tile_elems = 0;        // sum nt_i (nt_i + 1) / 2 * 4096
    int64_t* d_t_off = nullptr;
    double* d_M64 = nullptr;       // W_i = A_i^{-1}, packed lower tiles, FP64
    float* d_M32 = nullptr;        // Y_i = L_i^{-1} D_i (A_i^{-1} = Y_i^T Y_i), packed tiles, FP32 (mixed)
    float* d_W32 = nullptr;        // W_i in FP32 (mixed, blocks of at most 6 tiles per edge)
    ApplyPlan ap;                  // the preconditioner M^{-1}
    ApplyPlan apT;                 // RAS only: its transpose M^{-T} (masked input, full local results)
    int64_t slot_total = 0;        // row- or column-sum slots per right-hand side (sum nt(nt+1)/2 * 64)
    int64_t* d_s_off = nullptr;    // J+1 slot offsets
    int32_t* d_ent_blk = nullptr;  // ub_total: block of each block entry
    int64_t* d_f_off = nullptr;
    int64_t* d_q = nullptr;
    int64_t* d_ub_off = nullptr;   // J+1 offsets of per-block local vectors (sum q_i)
    int32_t shifts = 0;
    int64_t ub_total = 0;          // sum q_i

    // normal matrix N = H^T H: block row j as a dense p_j x Q_j slab over the
    // columns of the subdomains meeting j (N_cols); Gram blocks of meeting
    // pairs kept during set-up only
    std::vector<int64_t> N_off, N_coff;  // J+1: slab elements / column-list offsets
    int64_t N_elems = 0;
    double* d_N = nullptr;
    int64_t* d_N_off = nullptr;
    int64_t* d_N_coff = nullptr;
    int32_t* d_N_cols = nullptr;
    int2* d_slab_tasks = nullptr;   // (subdomain, first row) per product workgroup
    int64_t n_slab_tasks = 0;
    // the slabs again in matrix-core operand order, per 16-row task: quad c
    // of columns 4c .. 4c + 3 as 64 doubles (entry 16 g + r: row r, column
    // 4c + g; zero past the slab)
    double* d_Nt = nullptr;
    int64_t* d_Nt_off = nullptr;    // device J+1
    int64_t Nt_elems = 0;
    std::vector<std::vector<std::pair<int, int>>> pair_tab;  // j -> (k >= j, pair id)
    double* d_G = nullptr;
    void* d_pair_blocks = nullptr;

    // products with H: row chunks of each block, partial sums per chunk
    std::vector<int64_t> chunk_off; // J+1 (chunks per subdomain)
    int64_t n_chunks = 0, part_total = 0;
    int64_t* d_chunk_off = nullptr; // J+1
    int32_t* d_chunk_sub = nullptr; // n_chunks: subdomain of each chunk
    int64_t* d_part_off = nullptr;  // n_chunks: column offset of each chunk's partial
    int64_t* d_col_pbase = nullptr; // P: first chunk partial of each column
    int32_t* d_col_pstride = nullptr; // P: distance between its chunk partials (p_j)
    int32_t* d_col_nch = nullptr;   // P: number of chunk partials
    double* d_tpair = nullptr;      // per-pair values of H x
    size_t tpair_elems = 0;
    int32_t* d_col_sub = nullptr;   // P: subdomain of each column
    int32_t* d_feat_sub = nullptr;  // sum_m: subdomain of each hidden feature

    // workspace (grows on demand)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* ws2 = nullptr;           // true-residual scratch
    size_t ws2_bytes = 0;
    double* pinned = nullptr;      // host pinned scalars
    std::vector<std::pair<char*, size_t>> stage;  // pinned staging chunks (last one current)
    size_t stage_used = 0;

    double setup_ms[4] = {0, 0, 0, 0};  // assemble, pca+factor host-clock times

    // launch parameters chosen by the autotuner (rann_dd_autotune) or the caller
    rann_dd_tuning tune{768, 240, 1, 1, 0, 0};
    // executable graphs of CG check windows, keyed by what their launches bake in
    struct CgGraph {
        hipGraphExec_t exec = nullptr;
        uint64_t key = 0;
    };
    CgGraph cg_graph[4];
    int cg_graph_next = 0;
    int graph_broken = 0;          // a capture failed once: eager launches from then on
    hipStream_t cap_stream = nullptr;  // private stream the windows are captured on

    std::vector<void*> allocs;     // everything to free
};

// ---------------------------------------------------------------------------
// error handling
void set_error(const std::string& msg);

#define RDD_HIP(call)                                                          \
    do {                                                                       \
        hipError_t e_ = (call);                                                \
        if (e_ != hipSuccess) {                                                \
            ::rdd::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return RANN_EDEVICE;                                               \
        }                                                                      \
    } while (0)

#define RDD_TRY(call)                                                          \
    do {                                                                       \
        int r_ = (call);                                                       \
        if (r_ < 0) return r_;                                                 \
    } while (0)

// Device memory comes from a process-wide cache: blocks released by dev_free
// are kept per device and size and handed out again, so the set-up and solve
// calls do not pay for hipMalloc/hipFree each time (rann_dd_trim_cache returns
// them to the runtime).
void* cache_alloc(int device, size_t bytes, hipStream_t stream, hipError_t* err);
void cache_free(int device, void* p, hipStream_t stream);

template <class T>
int dev_alloc(Handle& h, T** ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipSuccess;
    void* p = cache_alloc(h.device, count * sizeof(T), h.stream, &e);
    if (!p) {
        set_error("device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed: " +
                  hipGetErrorString(e));
        return RANN_ENOMEM;
    }
    h.allocs.push_back(p);
    *ptr = static_cast<T*>(p);
    return RANN_OK;
}

// Host -> device copy ordered on the handle's stream through pinned staging
// memory (the source may be released on return).
int upload(Handle& h, void* dst, const void* src, size_t bytes);
// Device -> host copy through pinned staging memory; synchronises the stream.
int download(Handle& h, void* dst, const void* src, size_t bytes);
// Release staging space; call only when the handle's stream is idle.
void stage_reset(Handle& h);

void dev_free(Handle& h, void* p);
int ensure_ws(Handle& h, size_t bytes);

// Optional per-kernel timing with HIP events on the launch stream (process-wide,
// off by default): KTimer t(stream, "k_name"); <launch>; t.stop();
bool ktime_enabled();
// The timers are off on this thread while a KTimeOff lives (graph capture, the
// allocation-free entry point: no events may be created or recorded there).
extern thread_local int g_ktime_off;
struct KTimeOff {
    bool on;
    explicit KTimeOff(bool b = true) : on(b) {
        if (on) ++g_ktime_off;
    }
    ~KTimeOff() {
        if (on) --g_ktime_off;
    }
    KTimeOff(const KTimeOff&) = delete;
    KTimeOff& operator=(const KTimeOff&) = delete;
};
void ktime_record(const char* name, hipEvent_t a, hipEvent_t b);
// Times the launches between construction and stop() with two events on the
// stream.  With on_launch, the region is one launch that records the events
// itself (hipExtLaunchKernelGGL with a and b: its start and end), so the
// figure is that kernel's own duration.
struct KTimer {
    hipStream_t s;
    const char* name;
    hipEvent_t a = nullptr, b = nullptr;
    bool on_launch = false;
    KTimer(hipStream_t stream, const char* n, bool by_launch = false) : s(stream), name(n), on_launch(by_launch) {
        if (ktime_enabled() && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
            if (!on_launch) (void)hipEventRecord(a, s);
        } else {
            a = b = nullptr;
        }
    }
    void stop() {
        if (a) {
            if (!on_launch) (void)hipEventRecord(b, s);
            ktime_record(name, a, b);
            a = b = nullptr;
        }
    }
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files)
int bin_points(Handle& h, const double* X, int64_t n, PointSet& ps);
int pair_records(Handle& h, const double* X, int64_t n_int, const double* a,
                 const double* beta, const double* c, const double* Lfun, int64_t n_all,
                 double lambda_B, bool value_rows_only, const double* Lq, PointSet& ps);
int exclusive_scan_i64(Handle& h, const int64_t* in, int64_t* out, int64_t n);

int pca_gram(Handle& h, double* G, const int64_t* g_off_host, const int64_t* d_g_off);
int eig_batched(Handle& h, double* G, const int64_t* d_g_off, double* S, const int64_t* d_s_off,
                double* Y, double tol, int mode, int32_t* d_p, double* d_eig, int32_t* d_tie);
// sizes of a batch of symmetric matrices for the eigensolver
struct EigDims {
    int J;
    const int32_t* m;      // host, J sizes
    const int32_t* d_m;    // device, J sizes
    const int64_t* d_m_off;  // device, J+1 offsets of the eigenvalues
    int64_t sum_m;
};
// eigenvalues (descending, at d_eig + m_off) of every matrix of the batch, the
// count p above the threshold (d_p, and the tie flag), and the eigenvectors of
// the d_nvec[j] largest (all of them when d_nvec is null: d_p) as the columns
// of Y (row-major m x m per matrix, at d_g_off like G, which is overwritten)
int eig_batched_dims(Handle& h, const EigDims& dm, double* G, const int64_t* d_g_off, double* S,
                     const int64_t* d_s_off, double* Y, double tol, int mode, int32_t* d_p, double* d_eig,
                     int32_t* d_flags, const int32_t* d_nvec);
int compact_V(Handle& h, const double* Z, const int64_t* d_g_off, double* V);
// the eigen-PCA by subspace iteration with Rayleigh-Ritz (subspace.hip); returns
// kSubspaceDecline when a subdomain would need a block wider than its limit
constexpr int kSubspaceDecline = 100;
int eig_subspace(Handle& h, const double* G, const std::vector<int64_t>& g_off, const int64_t* d_g_off,
                 double tol, int mode, int32_t* d_p, double* d_eig, int32_t* d_flags, double* Yfull);
int64_t eig_scratch_elems(int m);
int feature_rows(Handle& h);
// several hidden layers (deep.hip): set-up from the descriptor, the value
// matrices (slot kRecW) or probe values (slot kRecP0) of a point set into out
// (n_j x m_j at d_out_off[j]), the operator rows H (and H32)
int deep_setup(Handle& h, const rann_dd_desc* ds);
int deep_values(Handle& h, const PointSet& ps, int slot, const int64_t* d_out_off, double* out);
int deep_feature_rows(Handle& h);
// the same values for one or several hidden layers (gemm.hip)
// (with T and one hidden layer: the tanh values themselves into T as well)
int values_matrix(Handle& h, const PointSet& ps, int slot, const int64_t* d_out_off, double* out,
                  double* T = nullptr);
// probe evaluation through the explicit probe values T_j and batched
// products: y = per-pair values (x: raw coefficients, sum_m x k) or, with
// transpose, y = raw-coefficient gradient (x: per point, M x k)
int eval_explicit(Handle& h, const PointSet& ps, const double* x, int k, double* y, bool transpose);
// raw-neuron coefficients c_j = V_j W_j (or, with transpose, V_j^T c_j) as
// batched matrix-core products
int coeffs_batched(Handle& h, const double* x, int k, double* y, bool transpose);
int build_schwarz(Handle& h);
template <class T>
int local_blocks(Handle& h, const T* H, T* A_out);
int plan_products(Handle& h);
int normal_blocks(Handle& h);
void release_gram(Handle& h);
constexpr int kSlabRows = 16;       // slab rows per product workgroup
// s = N x (N = H^T H from the slabs); with part != null also per-workgroup
// partials of <x, s> at part[wg * k + t] (n_slab_tasks workgroups)
// s = N x; with part, also the per-workgroup partials of <x, s>.  With pu,
// x is the previous CG direction and the product first forms the new one
// (p = z + beta p, written to pu->pcur) and the previous iteration's
// bookkeeping (see cg_step.h); the partials are then those of <p, s>.
struct PUpd;
int launch_normal(Handle& h, const double* x, int k, double* s, double* part, const PUpd* pu = nullptr);
// workgroups whose partials of <x, s> launch_normal writes (rows of part)
int normal_parts(const Handle& h, int k);

int launch_Hx(Handle& h, const double* x, int k, double* y, bool scale_bnd);
int launch_HTy(Handle& h, const double* y, int k, double* x, double* partial);
int launch_precond(Handle& h, const double* r, int k, double* z, double* ub);
// z = sum of the weighted local results of plan pl by subdomain segments and,
// with part, the partials of <r, z> (gather_parts(h, k) workgroups)
int launch_gather(Handle& h, const ApplyPlan& pl, const double* ub, const double* r, int k, double* z,
                  double* part);
int gather_parts(const Handle& h, int k);
// z = M^{-T} r; tmp: (P + 1) k scratch
int launch_precond_T(Handle& h, const double* r, int k, double* z, double* ub, double* tmp);
// ub: (2 ub_total + 2 slot_total) k doubles of scratch
int launch_precond_local(Handle& h, const ApplyPlan& pl, const double* r, int k, double* ub);

int krylov_cg(Handle& h, const double* rhs, int k, const double* W0, const rann_dd_solve_opts& o,
              double* W, rann_dd_stats* st, int* status);
int adjoint_cg(Handle& h, const double* dW, int k, const rann_dd_solve_opts& o, double* z,
               rann_dd_stats* st, int* status);
int adjoint_gmres(Handle& h, const double* dW, int k, const rann_dd_solve_opts& o, double* z,
                  rann_dd_stats* st, int* status);
int krylov_gmres(Handle& h, const double* rhs, int k, const double* W0,
                 const rann_dd_solve_opts& o, double* W, rann_dd_stats* st, int* status);
// Picard / Newton linearisation of a polynomial reaction (nonlinear.hip)
int linearize(Handle& h, const double* u, const double* c0, const double* f, int64_t n, const double* gamma,
              int n_gamma, int mode, double* c_out, double* f_out, const double* u_prev, double* inc);
// CGS and BiCG (method RANN_METHOD_CGS / RANN_METHOD_BICG); Fs = null: adjoint
int krylov_lanczos(Handle& h, const double* rhs, const double* Fs, int k, const double* W0,
                   const rann_dd_solve_opts& o, double* W, rann_dd_stats* st, int* status);
int true_residual(Handle& h, const double* Fs, const double* W, int k, double* out_host,
                  double* rhs_norm_host);
int time_cg_iterations(Handle& h, int k, int iters, double* rhs, double* W, double* us_per_iter);
int scale_boundary(Handle& h, const double* F, int k, double* Fs, double factor);
int eval_points(Handle& h, const double* Xq, int64_t M, const double* Lq, const double* W,
                int k, double* U, bool transpose);
int coeffs_raw(Handle& h, const double* W, int k, double* c, bool transpose);

}  // namespace rdd
