// C entry points (include/rann_dd.h): validation, ownership, phase ordering.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace rdd {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

// ------------------------------------------------------------ kernel timing
namespace {
std::atomic<int> g_ktime_on{0};
std::mutex g_ktime_mu;
struct KRec {
    std::string name;
    hipEvent_t a, b;
};
std::vector<KRec> g_ktime_pending;
std::map<std::string, std::pair<double, int64_t>> g_ktime_acc;

void ktime_flush_locked() {
    for (auto& r : g_ktime_pending) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto& e = g_ktime_acc[r.name];
            e.first += ms;
            e.second += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_ktime_pending.clear();
}
}  // namespace

// entry points and captures that must not create events turn the timers off
// for their own thread (KTimeOff)
thread_local int g_ktime_off = 0;

bool ktime_enabled() { return g_ktime_off == 0 && g_ktime_on.load(std::memory_order_relaxed) != 0; }

// ------------------------------------------------------------ static scratch
// Device memory of the allocation-free apply: a file-scope array that every GPU
// the library runs on holds until the process ends.  Host code never uses the
// array's name as an address: its device address is looked up once per device
// (with that device current) and kept in g_scratch_dev.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];
namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;  // per device; null until looked up
}  // namespace

// Looks up the current device's address of the scratch array (once per
// device); called with `device` current.
static int scratch_resolve(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0) return RANN_EDEVICE;
    if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
    if (g_scratch_dev[device]) return RANN_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        return RANN_EDEVICE;
    }
    g_scratch_dev[device] = static_cast<double*>(ptr);
    return RANN_OK;
}

static double* scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (device >= 0 && device < (int)g_scratch_dev.size()) ? g_scratch_dev[device] : nullptr;
}

void ktime_record(const char* name, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_ktime_mu);
    g_ktime_pending.push_back({name, a, b});
    if (g_ktime_pending.size() > 4096) ktime_flush_locked();
}

namespace {

struct CachedBlock {
    void* p;
    hipStream_t stream;  // stream of the last use
};

constexpr int kCacheDevices = 64;

struct DeviceCache {
    std::mutex mu;
    std::multimap<size_t, CachedBlock> free_blocks[kCacheDevices];
    std::unordered_map<void*, size_t> size_of;  // every block the cache owns
    std::multimap<size_t, char*> free_pinned;
    std::unordered_map<char*, size_t> pinned_size;
};

// leaked on purpose: it outlives every handle and needs no teardown ordering
DeviceCache& device_cache() {
    static DeviceCache* c = new DeviceCache();
    return *c;
}

size_t round_block(size_t b) {
    if (b <= (size_t(1) << 20)) return (b + 511) & ~size_t(511);
    const size_t g = size_t(2) << 20;
    return (b + g - 1) / g * g;
}

size_t trim_device(DeviceCache& c, int device) {
    size_t released = 0;
    auto& fb = c.free_blocks[device];
    for (auto& e : fb) {
        (void)hipFree(e.second.p);
        c.size_of.erase(e.second.p);
        released += e.first;
    }
    fb.clear();
    return released;
}

char* pinned_get(size_t bytes) {
    DeviceCache& c = device_cache();
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto it = c.free_pinned.lower_bound(bytes);
        if (it != c.free_pinned.end()) {
            char* p = it->second;
            c.free_pinned.erase(it);
            return p;
        }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(c.mu);
    c.pinned_size[static_cast<char*>(p)] = bytes;
    return static_cast<char*>(p);
}

void pinned_put(char* p) {
    DeviceCache& c = device_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    c.free_pinned.insert({c.pinned_size[p], p});
}

}  // namespace

void* cache_alloc(int device, size_t bytes, hipStream_t stream, hipError_t* err) {
    DeviceCache& c = device_cache();
    const size_t r = round_block(bytes);
    if (device < 0 || device >= kCacheDevices) device = 0;
    {
        std::lock_guard<std::mutex> lk(c.mu);
        auto& fb = c.free_blocks[device];
        auto it = fb.lower_bound(r);
        if (it != fb.end() && it->first <= r + r / 4) {
            CachedBlock b = it->second;
            fb.erase(it);
            // a block last used on another stream may still be read there
            if (b.stream != stream) (void)hipDeviceSynchronize();
            return b.p;
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, r);
    if (e != hipSuccess) {
        {
            std::lock_guard<std::mutex> lk(c.mu);
            (void)hipDeviceSynchronize();
            trim_device(c, device);
        }
        (void)hipGetLastError();
        e = hipMalloc(&p, r);
    }
    if (e != hipSuccess) {
        if (err) *err = e;
        (void)hipGetLastError();
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(c.mu);
    c.size_of[p] = r;
    return p;
}

void release_pinned(char* p) { pinned_put(p); }

size_t cache_trim_all() {
    DeviceCache& c = device_cache();
    (void)hipDeviceSynchronize();
    std::lock_guard<std::mutex> lk(c.mu);
    size_t released = 0;
    for (int d = 0; d < kCacheDevices; ++d) released += trim_device(c, d);
    for (auto& e : c.free_pinned) {
        (void)hipHostFree(e.second);
        c.pinned_size.erase(e.second);
        released += e.first;
    }
    c.free_pinned.clear();
    return released;
}

void cache_free(int device, void* p, hipStream_t stream) {
    if (!p) return;
    DeviceCache& c = device_cache();
    if (device < 0 || device >= kCacheDevices) device = 0;
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.size_of.find(p);
    if (it == c.size_of.end()) return;
    c.free_blocks[device].insert({it->second, CachedBlock{p, stream}});
}

void dev_free(Handle& h, void* p) {
    if (!p) return;
    auto it = std::find(h.allocs.begin(), h.allocs.end(), p);
    if (it != h.allocs.end()) {
        h.allocs.erase(it);
        cache_free(h.device, p, h.stream);
    }
}

int upload(Handle& h, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return RANN_OK;
    const size_t need = (bytes + 255) & ~size_t(255);
    if (h.stage.empty() || h.stage_used + need > h.stage.back().second) {
        const size_t cap = std::max(need, size_t(4) << 20);
        char* p = pinned_get(cap);
        if (!p) {
            set_error("pinned staging allocation failed");
            return RANN_ENOMEM;
        }
        DeviceCache& c = device_cache();
        size_t got = cap;
        {
            std::lock_guard<std::mutex> lk(c.mu);
            got = c.pinned_size[p];
        }
        h.stage.push_back({p, got});
        h.stage_used = 0;
    }
    char* s = h.stage.back().first + h.stage_used;
    std::memcpy(s, src, bytes);
    h.stage_used += need;
    RDD_HIP(hipMemcpyAsync(dst, s, bytes, hipMemcpyHostToDevice, h.stream));
    return RANN_OK;
}

int download(Handle& h, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return RANN_OK;
    const size_t need = (bytes + 255) & ~size_t(255);
    if (h.stage.empty() || h.stage_used + need > h.stage.back().second) {
        const size_t cap = std::max(need, size_t(4) << 20);
        char* p = pinned_get(cap);
        if (!p) {
            set_error("pinned staging allocation failed");
            return RANN_ENOMEM;
        }
        DeviceCache& c = device_cache();
        size_t got = cap;
        {
            std::lock_guard<std::mutex> lk(c.mu);
            got = c.pinned_size[p];
        }
        h.stage.push_back({p, got});
        h.stage_used = 0;
    }
    char* s = h.stage.back().first + h.stage_used;
    RDD_HIP(hipMemcpyAsync(s, src, bytes, hipMemcpyDeviceToHost, h.stream));
    RDD_HIP(hipStreamSynchronize(h.stream));
    std::memcpy(dst, s, bytes);
    stage_reset(h);  // the stream is idle: every staged copy has completed
    return RANN_OK;
}

void stage_reset(Handle& h) {
    // keep the current chunk, give the older ones back
    if (h.stage.size() > 1) {
        for (size_t i = 0; i + 1 < h.stage.size(); ++i) pinned_put(h.stage[i].first);
        h.stage.erase(h.stage.begin(), h.stage.end() - 1);
    }
    h.stage_used = 0;
}

int ensure_ws(Handle& h, size_t bytes) {
    if (h.ws_bytes >= bytes) return RANN_OK;
    if (h.ws) dev_free(h, h.ws);
    h.ws = nullptr;
    h.ws_bytes = 0;
    unsigned char* p = nullptr;
    RDD_TRY(dev_alloc(h, &p, bytes + (bytes >> 3)));
    h.ws = p;
    h.ws_bytes = bytes + (bytes >> 3);
    return RANN_OK;
}

namespace {

__global__ void k_pad_features(int64_t sum_m, int d, const double* __restrict__ R,
                               double* __restrict__ Rf) {
    int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (f >= sum_m) return;
    for (int i = 0; i < 4; ++i) Rf[f * 4 + i] = (i < d) ? R[f * d + i] : 0.0;
}

__global__ void k_identity_V(const int32_t* __restrict__ m, const int64_t* __restrict__ v_off,
                             double* __restrict__ V) {
    const int j = blockIdx.x;
    const int mj = m[j];
    for (int64_t e = threadIdx.x; e < (int64_t)mj * mj; e += blockDim.x)
        V[v_off[j] + e] = ((e / mj) == (e % mj)) ? 1.0 : 0.0;
}

__global__ void k_concat_points(int64_t n_int, int64_t n_bnd, int d, const double* __restrict__ Xi,
                                const double* __restrict__ Xb, double* __restrict__ X) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t tot = (n_int + n_bnd) * d;
    if (idx >= tot) return;
    X[idx] = (idx < n_int * d) ? Xi[idx] : Xb[idx - n_int * d];
}

__global__ void k_scale_tail(int64_t row0, int64_t rows, int k, double f, double* __restrict__ a) {
    int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < rows * k) a[row0 * k + idx] *= f;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int validate_opts(const rann_dd_solve_opts* o) {
    if (!o) {
        set_error("opts is NULL");
        return RANN_EINVAL;
    }
    if (!(o->tol > 0.0) || o->maxiter < 1 || o->check_every < 1 ||
        o->method < RANN_METHOD_CG || o->method > RANN_METHOD_BICG ||
        ((o->method == RANN_METHOD_GMRES || o->method == RANN_METHOD_GMRES_RIGHT) &&
         (o->restart < 1 || o->restart > 128))) {
        set_error("invalid solve options");
        return RANN_EINVAL;
    }
    return RANN_OK;
}

}  // namespace

static int assemble_impl(const rann_dd_desc* ds, void* stream, Handle*& hp) {
    if (!ds) {
        set_error("desc is NULL");
        return RANN_EINVAL;
    }
    const int d = ds->d;
    if (d < 1 || d > kMaxDim) {
        set_error("d must be 1..4");
        return RANN_EINVAL;
    }
    int64_t J = 1, sum_l = 0;
    for (int i = 0; i < d; ++i) {
        if (ds->l[i] < 1 || ds->l[i] > 4096) {
            set_error("l[i] must be 1..4096");
            return RANN_EINVAL;
        }
        if (!(ds->sigma[i] > 0.0) || !std::isfinite(ds->sigma[i])) {
            set_error("sigma[i] must be positive and finite");
            return RANN_EINVAL;
        }
        J *= ds->l[i];
        sum_l += ds->l[i];
    }
    if (J > (1 << 20)) {
        set_error("too many subdomains");
        return RANN_EINVAL;
    }
    if (!ds->mu || !ds->m || !ds->R || !ds->b || !ds->X_int || !ds->a || !ds->beta || !ds->c ||
        ds->n_int < 1 || ds->n_bnd < 0 || (ds->n_bnd > 0 && !ds->X_bnd)) {
        set_error("missing array or empty point set in the descriptor");
        return RANN_EINVAL;
    }
    if (!(ds->lambda_B > 0.0) || !std::isfinite(ds->lambda_B)) {
        set_error("lambda_B must be positive and finite");
        return RANN_EINVAL;
    }
    if (ds->precision != RANN_FP64 && ds->precision != RANN_MIXED) {
        set_error("precision must be RANN_FP64 or RANN_MIXED");
        return RANN_EINVAL;
    }
    if (ds->stencil < RANN_STENCIL_SELF || ds->stencil > RANN_STENCIL_FULL ||
        ds->precond < RANN_PRECOND_NONE || ds->precond > RANN_PRECOND_SAS) {
        set_error("invalid stencil or preconditioner");
        return RANN_EINVAL;
    }
    if (ds->n_inner < 0 || ds->n_inner > kMaxInner) {
        set_error("n_inner must be 0..3");
        return RANN_EINVAL;
    }
    for (int i = 0; i < ds->n_inner; ++i)
        if (ds->inner_w[i] < 1 || ds->inner_w[i] > kMaxInnerWidth) {
            set_error("inner layer widths must be 1..64");
            return RANN_EINVAL;
        }
    if (ds->n_inner > 0 && (!ds->R_inner || !ds->b_inner)) {
        set_error("R_inner and b_inner are required when n_inner > 0");
        return RANN_EINVAL;
    }
    {
        int64_t off = 0;
        for (int i = 0; i < d; ++i) {
            for (int c = 0; c < ds->l[i]; ++c) {
                double v = ds->mu[off + c];
                if (!std::isfinite(v) || (c > 0 && !(v > ds->mu[off + c - 1]))) {
                    set_error("centres must be finite and strictly increasing per dimension");
                    return RANN_EINVAL;
                }
            }
            off += ds->l[i];
        }
    }
    for (int64_t j = 0; j < J; ++j) {
        if (ds->m[j] < 1 || ds->m[j] > kMaxWidth) {
            set_error("hidden widths must be 1..1024");
            return RANN_EINVAL;
        }
    }
    Handle* h = new Handle();
    hp = h;
    h->stream = static_cast<hipStream_t>(stream);
    RDD_HIP(hipGetDevice(&h->device));
    Geo& g = h->geo;
    g.d = d;
    g.J = (int)J;
    int off = 0;
    for (int i = 0; i < kMaxDim; ++i) {
        g.l[i] = (i < d) ? ds->l[i] : 1;
        g.mu_off[i] = (i < d) ? off : 0;
        if (i < d) off += ds->l[i];
        g.sigma[i] = (i < d) ? ds->sigma[i] : 1.0;
        g.inv_sigma[i] = 1.0 / g.sigma[i];
    }
    h->lambda_B = ds->lambda_B;
    h->precision = ds->precision;
    h->stencil = ds->stencil;
    h->precond = ds->precond;
    h->n_int = ds->n_int;
    h->n_bnd = ds->n_bnd;
    h->N = ds->n_int + ds->n_bnd;
    h->m.assign(ds->m, ds->m + J);
    h->m_off.assign(J + 1, 0);
    for (int64_t j = 0; j < J; ++j) h->m_off[j + 1] = h->m_off[j] + h->m[j];
    h->sum_m = h->m_off[J];
    RDD_TRY(dev_alloc(*h, &h->d_mu, (size_t)sum_l));
    RDD_TRY(upload(*h, h->d_mu, ds->mu, sizeof(double) * sum_l));
    RDD_TRY(dev_alloc(*h, &h->d_m, (size_t)J));
    RDD_TRY(dev_alloc(*h, &h->d_m_off, (size_t)J + 1));
    RDD_TRY(upload(*h, h->d_m, h->m.data(), sizeof(int32_t) * J));
    RDD_TRY(upload(*h, h->d_m_off, h->m_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(dev_alloc(*h, &h->d_Rf, (size_t)h->sum_m * 4));
    RDD_TRY(dev_alloc(*h, &h->d_bf, (size_t)h->sum_m));
    if (ds->n_inner == 0) {
        hipLaunchKernelGGL(k_pad_features, dim3((unsigned)((h->sum_m + 255) / 256)), dim3(256), 0,
                           h->stream, h->sum_m, d, ds->R, h->d_Rf);
        RDD_HIP(hipGetLastError());
    } else {
        RDD_TRY(deep_setup(*h, ds));
    }
    RDD_HIP(hipMemcpyAsync(h->d_bf, ds->b, sizeof(double) * h->sum_m, hipMemcpyDeviceToDevice,
                           h->stream));
    // points (interior then boundary) and operator coefficients
    double *X = nullptr, *a = nullptr, *be = nullptr, *c = nullptr, *Lf = nullptr;
    RDD_TRY(dev_alloc(*h, &X, (size_t)h->N * d));
    hipLaunchKernelGGL(k_concat_points, dim3((unsigned)((h->N * d + 255) / 256)), dim3(256), 0,
                       h->stream, h->n_int, h->n_bnd, d, ds->X_int, ds->X_bnd, X);
    RDD_HIP(hipGetLastError());
    RDD_TRY(dev_alloc(*h, &a, (size_t)h->n_int * d));
    RDD_TRY(dev_alloc(*h, &be, (size_t)h->n_int * d));
    RDD_TRY(dev_alloc(*h, &c, (size_t)h->n_int));
    RDD_HIP(hipMemcpyAsync(a, ds->a, sizeof(double) * h->n_int * d, hipMemcpyDeviceToDevice, h->stream));
    RDD_HIP(hipMemcpyAsync(be, ds->beta, sizeof(double) * h->n_int * d, hipMemcpyDeviceToDevice,
                           h->stream));
    RDD_HIP(hipMemcpyAsync(c, ds->c, sizeof(double) * h->n_int, hipMemcpyDeviceToDevice, h->stream));
    if (ds->Lfun) {
        RDD_TRY(dev_alloc(*h, &Lf, (size_t)h->N * (1 + 2 * d)));
        RDD_HIP(hipMemcpyAsync(Lf, ds->Lfun, sizeof(double) * h->N * (1 + 2 * d),
                               hipMemcpyDeviceToDevice, h->stream));
    }
    RDD_TRY(bin_points(*h, X, h->N, h->pts));
    RDD_TRY(pair_records(*h, X, h->n_int, a, be, c, Lf, h->N, h->lambda_B, false, nullptr, h->pts));
    RDD_HIP(hipStreamSynchronize(h->stream));
    // the pair records carry everything later phases need
    dev_free(*h, a);
    dev_free(*h, be);
    dev_free(*h, c);
    if (Lf) dev_free(*h, Lf);
    dev_free(*h, X);
    return RANN_OK;
}

static int pca_impl(Handle& h, double tol, int mode, const int32_t* p_force, const double* V_force,
                    int32_t* p_out) {
    if (h.pca_done) {
        set_error("rann_dd_pca was already called on this handle");
        return RANN_EINVAL;
    }
    if (mode < RANN_PCA_REL_EIG || mode > RANN_PCA_OFF || (mode != RANN_PCA_OFF && !(tol > 0.0))) {
        set_error("invalid PCA mode or threshold");
        return RANN_EINVAL;
    }
    if (V_force && !p_force) {
        set_error("V_force requires p_force");
        return RANN_EINVAL;
    }
    const int J = h.geo.J;
    int warn = RANN_OK;
    h.p.assign(J, 0);
    std::vector<int64_t> g_off(J + 1, 0);
    for (int j = 0; j < J; ++j) g_off[j + 1] = g_off[j] + (int64_t)h.m[j] * h.m[j];
    RDD_TRY(dev_alloc(h, &h.d_p, J));
    RDD_TRY(dev_alloc(h, &h.d_eig, (size_t)h.sum_m));
    double* Vfull = nullptr;
    int64_t* d_g_off = nullptr;
    if (mode != RANN_PCA_OFF && !V_force) {
        double *G = nullptr, *Z = nullptr, *Y = nullptr;
        int32_t* flags = nullptr;
        int64_t* d_s_off = nullptr;
        std::vector<int64_t> s_off(J + 1, 0);  // eigensolver scratch per subdomain
        for (int j = 0; j < J; ++j) s_off[j + 1] = s_off[j] + eig_scratch_elems(h.m[j]);
        RDD_TRY(dev_alloc(h, &G, (size_t)g_off[J]));
        RDD_TRY(dev_alloc(h, &Z, (size_t)s_off[J]));
        RDD_TRY(dev_alloc(h, &Y, (size_t)g_off[J]));
        RDD_TRY(dev_alloc(h, &d_g_off, (size_t)J + 1));
        RDD_TRY(dev_alloc(h, &d_s_off, (size_t)J + 1));
        RDD_TRY(dev_alloc(h, &flags, 2));
        RDD_TRY(upload(h, d_g_off, g_off.data(), sizeof(int64_t) * (J + 1)));
        RDD_TRY(upload(h, d_s_off, s_off.data(), sizeof(int64_t) * (J + 1)));
        RDD_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t) * 2, h.stream));
        RDD_TRY(pca_gram(h, G, g_off.data(), d_g_off));
        // the subspace path pays where the direct path is slowest: widths past
        // 480, whose panel reduction no longer fits in LDS
        const int mmin = h.m.empty() ? 0 : *std::min_element(h.m.begin(), h.m.end());
        const int mmax = h.m.empty() ? 0 : *std::max_element(h.m.begin(), h.m.end());
        int rc_e = kSubspaceDecline;
        if (h.tune.pca_subspace && mmin >= 128 && mmax > 480)
            rc_e = eig_subspace(h, G, g_off, d_g_off, tol, mode, h.d_p, h.d_eig, flags, Y);
        if (rc_e == kSubspaceDecline) {  // the direct eigensolver (overwrites G)
            RDD_HIP(hipMemsetAsync(flags, 0, sizeof(int32_t) * 2, h.stream));
            RDD_TRY(eig_batched(h, G, d_g_off, Z, d_s_off, Y, tol, mode, h.d_p, h.d_eig, flags));
        } else {
            RDD_TRY(rc_e);
        }
        dev_free(h, d_s_off);
        int32_t fl[2];
        RDD_TRY(download(h, fl, flags, sizeof(fl)));
        RDD_TRY(download(h, h.p.data(), h.d_p, sizeof(int32_t) * J));
        dev_free(h, Z);
        dev_free(h, G);
        dev_free(h, flags);
        if (fl[0]) {
            dev_free(h, Y);
            set_error("symmetric eigensolver did not converge");
            return RANN_EDEVICE;
        }
        if (fl[1]) warn = RANN_WRANKTIE;
        Vfull = Y;
    } else {
        for (int j = 0; j < J; ++j) h.p[j] = h.m[j];
        RDD_HIP(hipMemsetAsync(h.d_eig, 0, sizeof(double) * h.sum_m, h.stream));
    }
    if (p_force) {
        for (int j = 0; j < J; ++j) {
            if (p_force[j] < 1 || p_force[j] > h.m[j]) {
                set_error("p_force entries must be 1..m_j");
                return RANN_EINVAL;
            }
            h.p[j] = p_force[j];
        }
    }
    RDD_TRY(upload(h, h.d_p, h.p.data(), sizeof(int32_t) * J));
    h.col_off.assign(J + 1, 0);
    h.v_off.assign(J + 1, 0);
    h.h_off.assign(J + 1, 0);
    for (int j = 0; j < J; ++j) {
        h.col_off[j + 1] = h.col_off[j] + h.p[j];
        h.v_off[j + 1] = h.v_off[j] + (int64_t)h.m[j] * h.p[j];
        h.h_off[j + 1] = h.h_off[j] + (h.pts.row_off[j + 1] - h.pts.row_off[j]) * h.p[j];
    }
    h.P = h.col_off[J];
    h.nnz = h.h_off[J];
    RDD_TRY(dev_alloc(h, &h.d_col_off, J + 1));
    RDD_TRY(dev_alloc(h, &h.d_v_off, J + 1));
    RDD_TRY(dev_alloc(h, &h.d_h_off, J + 1));
    RDD_TRY(upload(h, h.d_col_off, h.col_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(upload(h, h.d_v_off, h.v_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(upload(h, h.d_h_off, h.h_off.data(), sizeof(int64_t) * (J + 1)));
    RDD_TRY(dev_alloc(h, &h.d_V, (size_t)h.v_off[J]));
    if (V_force) {
        RDD_HIP(hipMemcpyAsync(h.d_V, V_force, sizeof(double) * h.v_off[J], hipMemcpyDeviceToDevice,
                               h.stream));
    } else if (Vfull) {
        RDD_TRY(compact_V(h, Vfull, d_g_off, h.d_V));
    } else {
        hipLaunchKernelGGL(k_identity_V, dim3(J), dim3(256), 0, h.stream, h.d_m, h.d_v_off, h.d_V);
        RDD_HIP(hipGetLastError());
    }
    RDD_HIP(hipStreamSynchronize(h.stream));
    if (Vfull) dev_free(h, Vfull);
    if (d_g_off) dev_free(h, d_g_off);
    // operator rows in the PCA basis
    RDD_TRY(dev_alloc(h, &h.d_H, (size_t)h.nnz));
    if (h.precision == RANN_MIXED && h.tune.gram32) RDD_TRY(dev_alloc(h, &h.d_H32, (size_t)h.nnz));
    RDD_TRY(feature_rows(h));
    RDD_TRY(plan_products(h));
    RDD_TRY(normal_blocks(h));
    {
        const int rc_s = build_schwarz(h);
        release_gram(h);
        RDD_TRY(rc_s);
    }
    if (p_out) std::copy(h.p.begin(), h.p.end(), p_out);
    h.pca_done = true;
    return warn;
}

}  // namespace rdd

using rdd::Handle;

struct rann_dd_handle {
    Handle h;
};

static int guard_handle(const rann_dd_handle* hh, bool need_pca) {
    if (!hh) {
        rdd::set_error("handle is NULL");
        return RANN_EINVAL;
    }
    if (need_pca && !hh->h.pca_done) {
        rdd::set_error("rann_dd_pca has not been called on this handle");
        return RANN_EINVAL;
    }
    return RANN_OK;
}

extern "C" {

const char* rann_dd_last_error(void) { return rdd::g_last_error.c_str(); }

int rann_dd_ktime_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(rdd::g_ktime_mu);
    rdd::ktime_flush_locked();
    rdd::g_ktime_acc.clear();
    rdd::g_ktime_on.store(on ? 1 : 0);
    return RANN_OK;
}

int rann_dd_ktime_query(const char* name, double* total_ms, int64_t* launches) {
    if (!name || !total_ms || !launches) {
        rdd::set_error("invalid ktime_query arguments");
        return RANN_EINVAL;
    }
    std::lock_guard<std::mutex> lk(rdd::g_ktime_mu);
    rdd::ktime_flush_locked();
    auto it = rdd::g_ktime_acc.find(name);
    *total_ms = (it == rdd::g_ktime_acc.end()) ? 0.0 : it->second.first;
    *launches = (it == rdd::g_ktime_acc.end()) ? 0 : it->second.second;
    return RANN_OK;
}

int rann_dd_assemble(const rann_dd_desc* desc, void* hip_stream, rann_dd_handle** out) {
    if (!out) {
        rdd::set_error("out is NULL");
        return RANN_EINVAL;
    }
    *out = nullptr;
    rdd::g_last_error.clear();
    auto t0 = std::chrono::steady_clock::now();
    Handle* raw = nullptr;
    int rc = rdd::assemble_impl(desc, hip_stream, raw);
    if (rc < 0) {
        if (raw) {
            for (void* p : raw->allocs) (void)hipFree(p);
            delete raw;
        }
        return rc;
    }
    // the handle's device is current here: look up its scratch address once
    rc = rdd::scratch_resolve(raw->device);
    if (rc < 0) {
        for (void* p : raw->allocs) (void)hipFree(p);
        delete raw;
        return rc;
    }
    auto* hh = new rann_dd_handle();
    hh->h = std::move(*raw);
    delete raw;
    hh->h.setup_ms[0] = rdd::ms_since(t0);
    *out = hh;
    return RANN_OK;
}

int rann_dd_pca(rann_dd_handle* hh, double tol, int32_t mode, const int32_t* p_force,
                const double* V_force, int32_t* p_out) {
    RDD_TRY(guard_handle(hh, false));
    auto t0 = std::chrono::steady_clock::now();
    int rc = rdd::pca_impl(hh->h, tol, mode, p_force, V_force, p_out);
    hh->h.setup_ms[1] = rdd::ms_since(t0);
    return rc;
}

int rann_dd_solve(rann_dd_handle* hh, const double* F, int32_t k, const double* W0,
                  const rann_dd_solve_opts* opts, double* W, rann_dd_stats* st) {
    RDD_TRY(guard_handle(hh, true));
    RDD_TRY(rdd::validate_opts(opts));
    Handle& h = hh->h;
    if (!F || !W || k < 1 || k > 256) {
        rdd::set_error("F and W must be given and 1 <= k <= 256");
        return RANN_EINVAL;
    }
    double* Fs = nullptr;
    RDD_TRY(rdd::dev_alloc(h, &Fs, (size_t)h.N * k));
    int rc = rdd::scale_boundary(h, F, k, Fs, h.lambda_B);
    int status = RANN_OK;
    if (rc == RANN_OK) {
        if (opts->method == RANN_METHOD_CG) {
            rc = rdd::krylov_cg(h, Fs, k, W0, *opts, W, st, &status);
        } else if (opts->method == RANN_METHOD_CGS || opts->method == RANN_METHOD_BICG) {
            double* rhs = nullptr;
            double* part = nullptr;
            rc = rdd::dev_alloc(h, &rhs, (size_t)h.P * k);
            if (rc == RANN_OK) rc = rdd::dev_alloc(h, &part, (size_t)h.part_total * k);
            if (rc == RANN_OK) rc = rdd::launch_HTy(h, Fs, k, rhs, part);
            if (rc == RANN_OK) rc = rdd::krylov_lanczos(h, rhs, Fs, k, W0, *opts, W, st, &status);
            if (part) rdd::dev_free(h, part);
            if (rhs) rdd::dev_free(h, rhs);
        } else {
            rc = rdd::krylov_gmres(h, Fs, k, W0, *opts, W, st, &status);
        }
    }
    rdd::dev_free(h, Fs);
    if (rc < 0) return rc;
    return status;
}

int rann_dd_solve_backward(rann_dd_handle* hh, const double* dW, int32_t k,
                           const rann_dd_solve_opts* opts, double* dF, rann_dd_stats* st) {
    RDD_TRY(guard_handle(hh, true));
    RDD_TRY(rdd::validate_opts(opts));
    Handle& h = hh->h;
    if (!dW || !dF || k < 1 || k > 256) {
        rdd::set_error("dW and dF must be given and 1 <= k <= 256");
        return RANN_EINVAL;
    }
    double* z = nullptr;
    RDD_TRY(rdd::dev_alloc(h, &z, (size_t)h.P * k));
    int status = RANN_OK;
    int rc;
    if (opts->method == RANN_METHOD_CG)
        rc = rdd::adjoint_cg(h, dW, k, *opts, z, st, &status);
    else if (opts->method == RANN_METHOD_CGS || opts->method == RANN_METHOD_BICG)
        rc = rdd::krylov_lanczos(h, dW, nullptr, k, nullptr, *opts, z, st, &status);
    else
        rc = rdd::adjoint_gmres(h, dW, k, *opts, z, st, &status);
    if (rc == RANN_OK) rc = rdd::launch_Hx(h, z, k, dF, false);
    if (rc == RANN_OK && h.n_bnd > 0) {
        hipLaunchKernelGGL(rdd::k_scale_tail, dim3((unsigned)((h.n_bnd * k + 255) / 256)), dim3(256), 0,
                           h.stream, h.n_int, h.n_bnd, k, h.lambda_B, dF);
        if (hipGetLastError() != hipSuccess) rc = RANN_EDEVICE;
    }
    if (rc == RANN_OK && st) {
        if (hipStreamSynchronize(h.stream) != hipSuccess) rc = RANN_EDEVICE;
    }
    rdd::dev_free(h, z);
    if (rc < 0) return rc;
    return status;
}

int rann_dd_eval(rann_dd_handle* hh, const double* Xq, int64_t M, const double* Lq, const double* W,
                 int32_t k, double* U) {
    RDD_TRY(guard_handle(hh, true));
    if (!Xq || !W || !U || M < 1 || k < 1 || k > 256) {
        rdd::set_error("invalid eval arguments");
        return RANN_EINVAL;
    }
    return rdd::eval_points(hh->h, Xq, M, Lq, W, k, U, false);
}

int rann_dd_eval_T(rann_dd_handle* hh, const double* Xq, int64_t M, const double* Lq,
                   const double* dU, int32_t k, double* dW) {
    RDD_TRY(guard_handle(hh, true));
    if (!Xq || !dU || !dW || M < 1 || k < 1 || k > 256) {
        rdd::set_error("invalid eval_T arguments");
        return RANN_EINVAL;
    }
    return rdd::eval_points(hh->h, Xq, M, Lq, dU, k, dW, true);
}

int rann_dd_coeffs(rann_dd_handle* hh, const double* W, int32_t k, double* c) {
    RDD_TRY(guard_handle(hh, true));
    if (!W || !c || k < 1) {
        rdd::set_error("invalid coeffs arguments");
        return RANN_EINVAL;
    }
    RDD_TRY(rdd::coeffs_raw(hh->h, W, k, c, false));
    RDD_HIP(hipStreamSynchronize(hh->h.stream));
    return RANN_OK;
}

int rann_dd_matvec(rann_dd_handle* hh, const double* x, int32_t k, double* y) {
    RDD_TRY(guard_handle(hh, true));
    if (!x || !y || k < 1) return (rdd::set_error("invalid matvec arguments"), RANN_EINVAL);
    RDD_TRY(rdd::launch_Hx(hh->h, x, k, y, false));
    RDD_HIP(hipStreamSynchronize(hh->h.stream));
    return RANN_OK;
}

int rann_dd_rmatvec(rann_dd_handle* hh, const double* y, int32_t k, double* x) {
    RDD_TRY(guard_handle(hh, true));
    Handle& h = hh->h;
    if (!x || !y || k < 1) return (rdd::set_error("invalid rmatvec arguments"), RANN_EINVAL);
    double* part = nullptr;
    RDD_TRY(rdd::dev_alloc(h, &part, (size_t)h.part_total * k));
    int rc = rdd::launch_HTy(h, y, k, x, part);
    if (rc == RANN_OK && hipStreamSynchronize(h.stream) != hipSuccess) rc = RANN_EDEVICE;
    rdd::dev_free(h, part);
    return rc;
}

int rann_dd_apply_normal(rann_dd_handle* hh, const double* x, int32_t k, double* s) {
    RDD_TRY(guard_handle(hh, true));
    Handle& h = hh->h;
    if (!x || !s || k < 1) return (rdd::set_error("invalid apply_normal arguments"), RANN_EINVAL);
    double *y = nullptr, *part = nullptr;
    RDD_TRY(rdd::dev_alloc(h, &y, (size_t)h.N * k));
    RDD_TRY(rdd::dev_alloc(h, &part, (size_t)h.part_total * k));
    int rc = rdd::launch_Hx(h, x, k, y, false);
    if (rc == RANN_OK) rc = rdd::launch_HTy(h, y, k, s, part);
    if (rc == RANN_OK && hipStreamSynchronize(h.stream) != hipSuccess) rc = RANN_EDEVICE;
    rdd::dev_free(h, y);
    rdd::dev_free(h, part);
    return rc;
}

int rann_dd_apply_precond(rann_dd_handle* hh, const double* r, int32_t k, double* z) {
    RDD_TRY(guard_handle(hh, true));
    Handle& h = hh->h;
    if (!r || !z || k < 1) return (rdd::set_error("invalid apply_precond arguments"), RANN_EINVAL);
    double* ub = nullptr;
    RDD_TRY(rdd::dev_alloc(h, &ub, (size_t)std::max<int64_t>(2 * h.ub_total + 2 * h.slot_total, 1) * k));
    int rc = rdd::launch_precond(h, r, k, z, ub);
    if (rc == RANN_OK && hipStreamSynchronize(h.stream) != hipSuccess) rc = RANN_EDEVICE;
    rdd::dev_free(h, ub);
    return rc;
}

int rann_dd_get_tuning(const rann_dd_handle* hh, rann_dd_tuning* out) {
    RDD_TRY(guard_handle(hh, false));
    if (!out) return (rdd::set_error("out is NULL"), RANN_EINVAL);
    *out = hh->h.tune;
    return RANN_OK;
}

int rann_dd_set_tuning(rann_dd_handle* hh, const rann_dd_tuning* t) {
    RDD_TRY(guard_handle(hh, false));
    if (!t || t->tile_grid < 64 || t->tile_grid > 4096 || t->red_cap < 32 || t->red_cap > 240 ||
        (t->use_graph != 0 && t->use_graph != 1) || (t->pca_subspace != 0 && t->pca_subspace != 1) ||
        (t->gram32 != 0 && t->gram32 != 1) || t->reserved != 0)
        return (rdd::set_error("tuning outside its ranges (tile_grid 64..4096, red_cap 32..240, use_graph 0/1, "
                               "pca_subspace 0/1, gram32 0/1, reserved 0)"),
                RANN_EINVAL);
    hh->h.tune = *t;
    return RANN_OK;
}

int rann_dd_autotune(rann_dd_handle* hh, int32_t k, int32_t iters, rann_dd_tuning* best, double* best_us) {
    RDD_TRY(guard_handle(hh, true));
    Handle& h = hh->h;
    if (k < 1 || k > 256 || iters < 2 || iters > 1000 || !best)
        return (rdd::set_error("invalid autotune arguments"), RANN_EINVAL);
    double *rhs = nullptr, *W = nullptr;
    RDD_TRY(rdd::dev_alloc(h, &rhs, (size_t)h.P * k));
    int rc = rdd::dev_alloc(h, &W, (size_t)h.P * k);
    const rann_dd_tuning start = h.tune;
    // the persistent grid matters only for the FP64 local solves with 1 or 2
    // right-hand sides
    std::vector<int> grids{start.tile_grid};
    if (h.precision == RANN_FP64 && k <= 2 && h.precond != RANN_PRECOND_NONE) grids = {256, 512, 768, 1024};
    rann_dd_tuning win = start;
    double win_us = 1e300;
    for (int g : grids)
        for (int cap : {64, 128, 240})
            for (int gr : {0, 1}) {
                if (rc != RANN_OK) break;
                h.tune = rann_dd_tuning{g, cap, gr, start.pca_subspace, start.gram32, 0};
                double us = 0.0;
                rc = rdd::time_cg_iterations(h, k, iters, rhs, W, &us);
                if (rc == RANN_OK && us < win_us) {
                    win_us = us;
                    win = h.tune;
                }
            }
    rdd::dev_free(h, rhs);
    rdd::dev_free(h, W);
    h.tune = (rc == RANN_OK) ? win : start;
    RDD_TRY(rc);
    *best = win;
    if (best_us) *best_us = win_us;
    return RANN_OK;
}

int rann_dd_apply_precond_noalloc(rann_dd_handle* hh, const double* r, int32_t k, double* z) {
    RDD_TRY(guard_handle(hh, true));
    Handle& h = hh->h;
    if (!r || !z || k < 1) return (rdd::set_error("invalid apply_precond_noalloc arguments"), RANN_EINVAL);
    const size_t need = (size_t)std::max<int64_t>(2 * h.ub_total + 2 * h.slot_total, 1) * (size_t)k;
    if (need * sizeof(double) > rdd::kScratchBytes) {
        rdd::set_error("apply_precond_noalloc needs " + std::to_string(need * sizeof(double)) +
                       " bytes of scratch, more than its static " + std::to_string(rdd::kScratchBytes) +
                       "; use rann_dd_apply_precond or fewer right-hand sides");
        return RANN_EINVAL;
    }
    double* ub = rdd::scratch_of(h.device);
    if (!ub) return (rdd::set_error("the scratch address of this device was not looked up"), RANN_EDEVICE);
    rdd::KTimeOff no_timers;
    return rdd::launch_precond(h, r, k, z, ub);
}

int rann_dd_linearize(rann_dd_handle* hh, const double* u, const double* c0, const double* f, int64_t n,
                      const double* gamma, int32_t n_gamma, int32_t mode, double* c_out, double* f_out,
                      const double* u_prev, double* inc) {
    if (n < 0 || (n > 0 && (!u || !c0 || !f || !c_out || !f_out)) || !gamma || n_gamma < 1 ||
        n_gamma > RANN_MAX_GAMMA || (mode != RANN_LIN_NEWTON && mode != RANN_LIN_PICARD))
        return (rdd::set_error("invalid linearize arguments"), RANN_EINVAL);
    for (int p = 0; p < n_gamma; ++p)
        if (!std::isfinite(gamma[p])) return (rdd::set_error("gamma must be finite"), RANN_EINVAL);
    if (!hh) {
        if (inc && u_prev) return (rdd::set_error("the increment needs a handle"), RANN_EINVAL);
        Handle tmp;  // default stream, no allocation
        return rdd::linearize(tmp, u, c0, f, n, gamma, n_gamma, mode, c_out, f_out, nullptr, inc);
    }
    return rdd::linearize(hh->h, u, c0, f, n, gamma, n_gamma, mode, c_out, f_out, u_prev, inc);
}

int rann_dd_apply_precond_T(rann_dd_handle* hh, const double* r, int32_t k, double* z) {
    RDD_TRY(guard_handle(hh, true));
    Handle& h = hh->h;
    if (!r || !z || k < 1) return (rdd::set_error("invalid apply_precond_T arguments"), RANN_EINVAL);
    double* ub = nullptr;
    double* tmp = nullptr;
    RDD_TRY(rdd::dev_alloc(h, &ub, (size_t)std::max<int64_t>(2 * h.ub_total + 2 * h.slot_total, 1) * k));
    int rc = rdd::dev_alloc(h, &tmp, (size_t)(h.P + 1) * k);
    if (rc == RANN_OK) rc = rdd::launch_precond_T(h, r, k, z, ub, tmp);
    if (rc == RANN_OK && hipStreamSynchronize(h.stream) != hipSuccess) rc = RANN_EDEVICE;
    if (tmp) rdd::dev_free(h, tmp);
    rdd::dev_free(h, ub);
    return rc;
}

int rann_dd_get_info(const rann_dd_handle* hh, rann_dd_info* out) {
    RDD_TRY(guard_handle(hh, false));
    if (!out) return (rdd::set_error("out is NULL"), RANN_EINVAL);
    const Handle& h = hh->h;
    out->d = h.geo.d;
    out->J = h.geo.J;
    out->N_int = h.n_int;
    out->N_bnd = h.n_bnd;
    out->N = h.N;
    out->P = h.P;
    out->pairs = h.pts.pairs;
    out->nnz = h.nnz;
    out->sum_m = h.sum_m;
    out->factor_elems = h.tile_elems;
    out->max_q = h.max_q;
    out->pca_done = h.pca_done ? 1 : 0;
    out->normal_elems = h.N_elems;
    out->cg_graphs = 0;
    for (const auto& g : h.cg_graph) out->cg_graphs += g.exec ? 1 : 0;
    out->graph_failed = h.graph_broken;
    return RANN_OK;
}

int rann_dd_get_layout(const rann_dd_handle* hh, int64_t* row_off, int32_t* rows, int32_t* p) {
    RDD_TRY(guard_handle(hh, false));
    const Handle& h = hh->h;
    if (row_off) std::copy(h.pts.row_off.begin(), h.pts.row_off.end(), row_off);
    if (rows && h.pts.pairs > 0)
        RDD_HIP(hipMemcpy(rows, h.pts.d_rows, sizeof(int32_t) * h.pts.pairs, hipMemcpyDeviceToHost));
    if (p) {
        if (!h.pca_done) return (rdd::set_error("p is known after rann_dd_pca"), RANN_EINVAL);
        std::copy(h.p.begin(), h.p.end(), p);
    }
    return RANN_OK;
}

int rann_dd_get_arrays(const rann_dd_handle* hh, double* blocks, double* V, double* eig) {
    RDD_TRY(guard_handle(hh, true));
    const Handle& h = hh->h;
    if (blocks) RDD_HIP(hipMemcpy(blocks, h.d_H, sizeof(double) * h.nnz, hipMemcpyDeviceToDevice));
    if (V) RDD_HIP(hipMemcpy(V, h.d_V, sizeof(double) * h.v_off.back(), hipMemcpyDeviceToDevice));
    if (eig) RDD_HIP(hipMemcpy(eig, h.d_eig, sizeof(double) * h.sum_m, hipMemcpyDeviceToDevice));
    return RANN_OK;
}

int rann_dd_get_blocks(const rann_dd_handle* hh, int64_t* q) {
    RDD_TRY(guard_handle(hh, true));
    if (!q) return (rdd::set_error("q is NULL"), RANN_EINVAL);
    const Handle& h = hh->h;
    for (int j = 0; j < h.geo.J; ++j) q[j] = h.q.empty() ? 0 : h.q[j];
    return RANN_OK;
}

size_t rann_dd_trim_cache(void) { return rdd::cache_trim_all(); }

void rann_dd_destroy(rann_dd_handle* hh) {
    if (!hh) return;
    (void)hipStreamSynchronize(hh->h.stream);
    for (auto& g : hh->h.cg_graph)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (hh->h.cap_stream) (void)hipStreamDestroy(hh->h.cap_stream);
    for (void* p : hh->h.allocs) rdd::cache_free(hh->h.device, p, hh->h.stream);
    hh->h.allocs.clear();
    for (auto& c : hh->h.stage) rdd::release_pinned(c.first);
    hh->h.stage.clear();
    delete hh;
}

}  // extern "C"
