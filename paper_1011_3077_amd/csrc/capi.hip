// C ABI entry points (include/sdc.h): argument checks, handle management,
// and translation to the engine's jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "engine.hpp"
#include "engine_util.hpp"
#include "sdc.h"

using sdc::Handle;
using sdc::SplitJob;

struct sdc_handle_s {
    Handle h;
};

// Preallocated device memory of sdc_split_sym_noalloc (layout and use below).
constexpr size_t kScratchBytes = (size_t)SDC_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

using sdc::kMaxN;
using sdc::prec_ok;
using sdc::region_ok;

int use_device(Handle& h) {
    return hipSetDevice(h.device) == hipSuccess ? SDC_OK : SDC_ERR_DEVICE;
}

void resolve_profile(Handle& h) {
    if (!h.prof.on) return;
    (void)hipStreamSynchronize(h.stream);
    h.prof.resolve();
}

sdc_opts_t resolve(const sdc_opts_t* o) {
    sdc_opts_t r;
    if (o) r = *o;
    else sdc_opts_default(&r);
    return r;
}

// ---------------------------------------------------------------------------
// Preallocated memory of the no-allocation entry point (sdc_split_sym_noalloc).
//
// `scratch` is one file-scope device array; every GPU the library runs on
// holds its own copy (at its own address) until the process ends.  In host
// code its name is only a stand-in, so its device address is looked up once
// per device, with that device current, when the first handle on the device
// is created, and kept in scratch_dev[].  The array is carved into the
// descriptor arena, the per-tick norm and result staging buffers, and the
// split's workspace.  Host-side staging (the descriptor mirror and the small
// result buffer) is a static host array per device.  Every call on a device
// shares both, so calls that overlap on one device race; each call ends with
// a stream synchronization, so calls in sequence are safe.
// ---------------------------------------------------------------------------
constexpr size_t kNaDescBytes = 1 << 20;      // descriptor arena
constexpr size_t kNaNormElems = 8 << 10;      // convergence norms (doubles)
constexpr size_t kNaStageElems = 8 << 10;     // gathered results (doubles)
constexpr size_t kNaHostBytes = 64 << 10;     // host copy of the gathered results
constexpr int kNaMaxDevices = 16;
static_assert(kNaDescBytes + (kNaNormElems + kNaStageElems) * sizeof(double) < kScratchBytes, "scratch layout");

char* scratch_dev[kNaMaxDevices] = {};
std::mutex scratch_mu;
alignas(256) char na_host_desc[kNaMaxDevices][kNaDescBytes];
alignas(256) char na_host_res[kNaMaxDevices][kNaHostBytes];

// Device address of this device's scratch (the device must be current).
int init_scratch(int device) {
    if (device < 0 || device >= kNaMaxDevices) return SDC_OK;  // the entry point refuses such devices
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[device]) return SDC_OK;
    char* p = nullptr;
    if (hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return SDC_ERR_DEVICE;
    }
    scratch_dev[device] = p;
    return SDC_OK;
}


}  // namespace

extern "C" {

void sdc_opts_default(sdc_opts_t* o) {
    if (!o) return;
    o->prec = SDC_FP64;
    o->tau = 0.0;
    o->maxit = 60;
    o->seed = 0;
    o->max_retries = 2;
    o->split_tol = 1e-10;
    o->G = nullptr;
    o->diagnostics = 0;
    o->panel_width = 0;
}

const char* sdc_status_string(int s) {
    switch (s) {
    case SDC_OK: return "SDC_OK";
    case SDC_NOT_CONVERGED: return "SDC_NOT_CONVERGED";
    case SDC_NO_SPLIT: return "SDC_NO_SPLIT";
    case SDC_RANK_AMBIGUOUS: return "SDC_RANK_AMBIGUOUS";
    case SDC_ERR_INVALID: return "SDC_ERR_INVALID";
    case SDC_ERR_NOMEM: return "SDC_ERR_NOMEM";
    case SDC_ERR_DEVICE: return "SDC_ERR_DEVICE";
    case SDC_ERR_NONFINITE: return "SDC_ERR_NONFINITE";
    default: return "SDC_UNKNOWN";
    }
}

sdc_status_t sdc_create(sdc_handle_t* handle, int device, size_t budget, void* stream) {
    if (!handle) return SDC_ERR_INVALID;
    *handle = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SDC_ERR_DEVICE;
    sdc_handle_s* p = new (std::nothrow) sdc_handle_s;
    if (!p) return SDC_ERR_NOMEM;
    p->h.device = device;
    p->h.stream = static_cast<hipStream_t>(stream);
    p->h.budget = budget;
    // streams and events are made here, so the entry points that must not
    // allocate find them ready
    if (use_device(p->h) != SDC_OK || init_scratch(device) != SDC_OK || sdc::ensure_streams(p->h) != SDC_OK ||
        hipEventCreateWithFlags(&p->h.ev_sync, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->h.ev_desc, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (p->h.ev_sync) (void)hipEventDestroy(p->h.ev_sync);
        if (p->h.ev_desc) (void)hipEventDestroy(p->h.ev_desc);
        sdc::release_streams(p->h);
        delete p;
        return SDC_ERR_DEVICE;
    }
    *handle = p;
    return SDC_OK;
}

sdc_status_t sdc_destroy(sdc_handle_t handle) {
    if (!handle) return SDC_OK;
    Handle& h = handle->h;
    (void)hipSetDevice(h.device);
    (void)hipStreamSynchronize(h.stream);
    if (h.ws) (void)hipFree(h.ws);
    if (h.desc_d) (void)hipFree(h.desc_d);
    if (h.desc_h) (void)hipHostFree(h.desc_h);
    if (h.host) (void)hipHostFree(h.host);
    if (h.ws2) (void)hipFree(h.ws2);
    if (h.dnorm) (void)hipFree(h.dnorm);
    if (h.dstage) (void)hipFree(h.dstage);
    if (h.ev_sync) (void)hipEventDestroy(h.ev_sync);
    if (h.ev_desc) (void)hipEventDestroy(h.ev_desc);
    sdc::release_graph_stream(h);
    sdc::release_streams(h);
    delete handle;
    return SDC_OK;
}

sdc_status_t sdc_irs(sdc_handle_t hd, int n, const double* A, int lda, const double* B, int ldb, int transpose,
                     sdc_region_t region, const sdc_opts_t* opts, double* Ap, double* Bp, double* R, int ldo,
                     int* p, double* rconv) {
    if (!hd || n < 1 || n > kMaxN || !A || lda < n || (B && ldb < n) || !Ap || !Bp || ldo < n || !p || !rconv ||
        !region_ok(region))
        return SDC_ERR_INVALID;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    const sdc_opts_t o = resolve(opts);
    if (o.prec != SDC_FP64 && o.prec != SDC_FP32_REFINE) return SDC_ERR_INVALID;
    sdc::ProfScope ps(h);
    const int r = sdc::run_irs_only(h, n, A, lda, B, ldb, transpose ? 1 : 0, region, o, Ap, Bp, R, ldo, p, rconv);
    resolve_profile(h);
    return (sdc_status_t)r;
}

sdc_status_t sdc_split_sym(sdc_handle_t hd, int n, const double* A, int lda, sdc_region_t region,
                           const sdc_opts_t* opts, double* Q, int ldq, double* Ahat, int ldah, sdc_info_t* info) {
    if (!hd || n < 0 || n > kMaxN || (n > 0 && (!A || !Q || !Ahat)) || lda < n || ldq < n || ldah < n || !region_ok(region))
        return SDC_ERR_INVALID;
    sdc_info_t dummy;
    if (!info) info = &dummy;
    *info = sdc_info_t{};
    if (n == 0) return SDC_OK;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    std::vector<SplitJob> jobs(1);
    SplitJob& j = jobs[0];
    j.n = n; j.pencil = false; j.A = A; j.lda = lda; j.region = region; j.opts = resolve(opts);
    if (!prec_ok(j.opts, false, region.kind)) return SDC_ERR_INVALID;
    j.Q = Q; j.ldq = ldq; j.Ahat = Ahat; j.ldah = ldah;
    sdc::ProfScope ps(h);
    const int r = sdc::run_split_jobs(h, jobs);
    resolve_profile(h);
    if (r < 0) return (sdc_status_t)r;
    *info = j.info;
    return (sdc_status_t)j.status;
}

sdc_status_t sdc_split_sym_noalloc(sdc_handle_t hd, int n, const double* A, int lda, sdc_region_t region,
                                   const sdc_opts_t* opts, double* Q, int ldq, double* Ahat, int ldah,
                                   sdc_info_t* info) {
    if (!hd || n < 0 || n > SDC_NOALLOC_MAX_N || (n > 0 && (!A || !Q || !Ahat)) || lda < n || ldq < n || ldah < n ||
        !region_ok(region))
        return SDC_ERR_INVALID;
    Handle& h = hd->h;
    if (h.device < 0 || h.device >= kNaMaxDevices || !scratch_dev[h.device]) return SDC_ERR_DEVICE;
    sdc_info_t dummy;
    if (!info) info = &dummy;
    *info = sdc_info_t{};
    if (n == 0) return SDC_OK;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    std::vector<SplitJob> jobs(1);
    SplitJob& j = jobs[0];
    j.n = n; j.pencil = false; j.A = A; j.lda = lda; j.region = region; j.opts = resolve(opts);
    if (!prec_ok(j.opts, false, region.kind)) return SDC_ERR_INVALID;
    j.Q = Q; j.ldq = ldq; j.Ahat = Ahat; j.ldah = ldah;
    // a handle over the preallocated buffers: the caller's stream, streams
    // and events; nothing is allocated (the helpers refuse instead)
    Handle nh;
    nh.device = h.device;
    nh.stream = h.stream;
    nh.budget = 0;
    nh.qs = h.qs;
    nh.ev_sync = h.ev_sync;
    nh.ev_desc = h.ev_desc;
    nh.no_alloc = true;
    char* base = scratch_dev[h.device];
    nh.desc_d = base;
    nh.desc_h = na_host_desc[h.device];
    nh.desc_size = kNaDescBytes;
    nh.dnorm = reinterpret_cast<double*>(base + kNaDescBytes);
    nh.dnorm_cap = kNaNormElems;
    nh.dstage = nh.dnorm + kNaNormElems;
    nh.dstage_cap = kNaStageElems;
    nh.host = na_host_res[h.device];
    nh.host_size = kNaHostBytes;
    const size_t ws_off = kNaDescBytes + (kNaNormElems + kNaStageElems) * sizeof(double);
    nh.ws = base + ws_off;
    nh.ws_size = kScratchBytes - ws_off;
    sdc::ProfScope ps(nh);  // profiling off: its events would be allocations
    const int r = sdc::run_split_jobs(nh, jobs);
    nh.qs = sdc::QrStreams{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    if (r < 0) return (sdc_status_t)r;
    *info = j.info;
    return (sdc_status_t)j.status;
}

sdc_status_t sdc_trevc(sdc_handle_t hd, int n, const double* T, int ldt, const double* S, int lds, double* X,
                       int ldx) {
    if (!hd || n < 0 || n > kMaxN || (n > 0 && (!T || !X)) || ldt < n || ldx < n || (S && lds < n))
        return SDC_ERR_INVALID;
    if (n == 0) return SDC_OK;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    sdc::TrevcArgs a{T, ldt, S, S ? lds : n, X, ldx, n};
    sdc::trevc_launch(a, h.stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h.stream) != hipSuccess) return SDC_ERR_DEVICE;
    return SDC_OK;
}

sdc_status_t sdc_split_nonsym(sdc_handle_t hd, int n, const double* A, int lda, sdc_region_t region,
                              const sdc_opts_t* opts, double* Q, int ldq, double* Ahat, int ldah, sdc_info_t* info) {
    if (!hd || n < 0 || n > kMaxN || (n > 0 && (!A || !Q || !Ahat)) || lda < n || ldq < n || ldah < n || !region_ok(region))
        return SDC_ERR_INVALID;
    sdc_info_t dummy;
    if (!info) info = &dummy;
    *info = sdc_info_t{};
    if (n == 0) return SDC_OK;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    std::vector<SplitJob> jobs(1);
    SplitJob& j = jobs[0];
    j.n = n; j.pencil = false; j.nonsym = true; j.A = A; j.lda = lda; j.region = region; j.opts = resolve(opts);
    if (!prec_ok(j.opts, true, region.kind)) return SDC_ERR_INVALID;  // FP64 only
    j.Q = Q; j.ldq = ldq; j.Ahat = Ahat; j.ldah = ldah;
    sdc::ProfScope ps(h);
    const int r = sdc::run_split_jobs(h, jobs);
    resolve_profile(h);
    if (r < 0) return (sdc_status_t)r;
    *info = j.info;
    return (sdc_status_t)j.status;
}

sdc_status_t sdc_split_pencil(sdc_handle_t hd, int n, const double* A, int lda, const double* B, int ldb,
                              sdc_region_t region, const sdc_opts_t* opts, double* QL, int ldql, double* QR,
                              int ldqr, double* Ahat, int ldah, double* Bhat, int ldbh, sdc_info_t* info) {
    if (!hd || n < 0 || n > kMaxN || (n > 0 && (!A || !B || !QL || !QR || !Ahat || !Bhat)) || lda < n || ldb < n ||
        ldql < n || ldqr < n || ldah < n || ldbh < n || !region_ok(region))
        return SDC_ERR_INVALID;
    sdc_info_t dummy;
    if (!info) info = &dummy;
    *info = sdc_info_t{};
    if (n == 0) return SDC_OK;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    std::vector<SplitJob> jobs(1);
    SplitJob& j = jobs[0];
    j.n = n; j.pencil = true; j.A = A; j.lda = lda; j.B = B; j.ldb = ldb; j.region = region;
    j.opts = resolve(opts);
    if (!prec_ok(j.opts, true, region.kind)) return SDC_ERR_INVALID;
    j.Q = QR; j.ldq = ldqr; j.QL = QL; j.ldql = ldql; j.Ahat = Ahat; j.ldah = ldah; j.Bhat = Bhat; j.ldbh = ldbh;
    sdc::ProfScope ps(h);
    const int r = sdc::run_split_jobs(h, jobs);
    resolve_profile(h);
    if (r < 0) return (sdc_status_t)r;
    *info = j.info;
    return (sdc_status_t)j.status;
}

sdc_status_t sdc_split_sym_batched(sdc_handle_t hd, int count, const int* n, const double* const* A,
                                   const int* lda, const sdc_region_t* regions, const sdc_opts_t* opts,
                                   double* const* Q, const int* ldq, double* const* Ahat, const int* ldah,
                                   sdc_info_t* infos, int* statuses) {
    if (!hd || count < 0) return SDC_ERR_INVALID;
    if (count == 0) return SDC_OK;
    if (!n || !A || !lda || !regions || !Q || !ldq || !Ahat || !ldah || !statuses) return SDC_ERR_INVALID;
    const sdc_opts_t o = resolve(opts);
    if (o.G) return SDC_ERR_INVALID;
    std::vector<SplitJob> jobs;
    std::vector<int> idx;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 0 || n[i] > kMaxN || lda[i] < n[i] || ldq[i] < n[i] || ldah[i] < n[i] || !region_ok(regions[i]) ||
            !prec_ok(o, false, regions[i].kind))
            return SDC_ERR_INVALID;
        if (n[i] > 0 && (!A[i] || !Q[i] || !Ahat[i])) return SDC_ERR_INVALID;
    }
    for (int i = 0; i < count; ++i) {
        if (infos) infos[i] = sdc_info_t{};
        statuses[i] = SDC_OK;
        if (n[i] == 0) continue;
        SplitJob j;
        j.n = n[i]; j.pencil = false; j.A = A[i]; j.lda = lda[i]; j.region = regions[i]; j.opts = o;
        j.opts.seed = o.seed + (uint64_t)i * 1000003ull;
        j.Q = Q[i]; j.ldq = ldq[i]; j.Ahat = Ahat[i]; j.ldah = ldah[i];
        jobs.push_back(j);
        idx.push_back(i);
    }
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    sdc::ProfScope ps(h);
    const int r = sdc::run_split_jobs(h, jobs);
    resolve_profile(h);
    if (r < 0) return (sdc_status_t)r;
    for (size_t q = 0; q < jobs.size(); ++q) {
        statuses[idx[q]] = jobs[q].status;
        if (infos) infos[idx[q]] = jobs[q].info;
    }
    return SDC_OK;
}

sdc_status_t sdc_eig_dc(sdc_handle_t hd, int n, const double* A, int lda, const double* B, int ldb, int symmetric,
                        int leaf_max, const sdc_opts_t* opts, double* T, int ldt, double* S, int lds, double* QL,
                        int ldql, double* QR, int ldqr, int* nblocks, int* block_start, sdc_block_bound_t* bounds,
                        sdc_dc_info_t* info) {
    if (!hd || n < 0 || n > kMaxN || !nblocks || !block_start || leaf_max < 1) return SDC_ERR_INVALID;
    if (n > 0 && (!A || lda < n || !T || ldt < n)) return SDC_ERR_INVALID;
    if (!symmetric && n > 0 && (!B || ldb < n || !S || lds < n)) return SDC_ERR_INVALID;
    if ((QL && ldql < n) || (QR && ldqr < n)) return SDC_ERR_INVALID;
    sdc_dc_info_t dummy;
    if (!info) info = &dummy;
    *info = sdc_dc_info_t{};
    if (n == 0) {
        *nblocks = 0;
        block_start[0] = 0;
        return SDC_OK;
    }
    const sdc_opts_t o = resolve(opts);
    if (o.G || !prec_ok(o, !symmetric, SDC_HALFPLANE)) return SDC_ERR_INVALID;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    sdc::ProfScope ps(h);
    const int r = sdc::run_eig_dc(h, n, A, lda, symmetric ? nullptr : B, ldb, symmetric ? 1 : 0, leaf_max, o, T, ldt,
                                  symmetric ? nullptr : S, lds, symmetric ? nullptr : QL, ldql, QR, ldqr, nblocks,
                                  block_start, bounds, info);
    resolve_profile(h);
    return (sdc_status_t)r;
}

sdc_status_t sdc_profile_enable(sdc_handle_t hd, int on) {
    if (!hd) return SDC_ERR_INVALID;
    hd->h.prof.on = on != 0;
    hd->h.prof.reset();
    return SDC_OK;
}

sdc_status_t sdc_profile_read(sdc_handle_t hd, int kernel, sdc_kernel_stats_t* out) {
    if (!hd || !out || kernel < 0 || kernel >= sdc::PROF_NKERNELS) return SDC_ERR_INVALID;
    const sdc::Profiler& p = hd->h.prof;
    out->launches = p.launches[kernel];
    out->ms = p.ms[kernel];
    out->flops = p.flops[kernel];
    out->bytes = p.bytes[kernel];
    return SDC_OK;
}

sdc_status_t sdc_gaussian(sdc_handle_t hd, int n, uint64_t seed, int tag, double* G, int ldg) {
    if (!hd || n < 0 || (n > 0 && !G) || ldg < n) return SDC_ERR_INVALID;
    if (n == 0) return SDC_OK;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    return (sdc_status_t)sdc::run_gaussian(h, n, seed, tag, G, ldg);
}

// ---------------------------------------------------------------------------
// Panel-width table and its autotuner
// ---------------------------------------------------------------------------
static int tune_to_api(int v) { return v >= sdc::kNb64Never ? SDC_PANEL64_NEVER : v; }
static int tune_from_api(int v) { return v < 0 ? sdc::kNb64Never : v; }

sdc_status_t sdc_graphs_enable(sdc_handle_t hd, int on) {
    if (!hd) return SDC_ERR_INVALID;
    Handle& h = hd->h;
    if (on && h.no_alloc) return SDC_ERR_INVALID;
    if (on) {
        if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
        if (sdc::ensure_graph_stream(h) != SDC_OK) return SDC_ERR_DEVICE;
    }
    h.graphs = on != 0;
    return SDC_OK;
}

sdc_status_t sdc_tree_overlap_enable(sdc_handle_t hd, int on) {
    if (!hd) return SDC_ERR_INVALID;
    hd->h.tree_overlap = on != 0;
    return SDC_OK;
}

sdc_status_t sdc_lookahead_set(sdc_handle_t hd, int min_cols) {
    if (!hd) return SDC_ERR_INVALID;
    hd->h.la_min = min_cols > 0 ? min_cols : sdc::kLookaheadNever;
    return SDC_OK;
}

sdc_status_t sdc_tune_set(sdc_handle_t hd, int nb64_min_fp64, int nb64_min_fp32) {
    if (!hd) return SDC_ERR_INVALID;
    hd->h.nb64_min[0] = tune_from_api(nb64_min_fp64);
    hd->h.nb64_min[1] = tune_from_api(nb64_min_fp32);
    return SDC_OK;
}

sdc_status_t sdc_tune_get(sdc_handle_t hd, int* nb64_min_fp64, int* nb64_min_fp32) {
    if (!hd || !nb64_min_fp64 || !nb64_min_fp32) return SDC_ERR_INVALID;
    *nb64_min_fp64 = tune_to_api(hd->h.nb64_min[0]);
    *nb64_min_fp32 = tune_to_api(hd->h.nb64_min[1]);
    return SDC_OK;
}

sdc_status_t sdc_autotune(sdc_handle_t hd, const int* orders, int count, int reps, sdc_tune_result_t* results) {
    if (!hd || !orders || count < 1 || reps < 1) return SDC_ERR_INVALID;
    for (int i = 0; i < count; ++i)
        if (orders[i] < 1 || orders[i] > kMaxN) return SDC_ERR_INVALID;
    Handle& h = hd->h;
    if (h.no_alloc) return SDC_ERR_INVALID;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    const int nmax = *std::max_element(orders, orders + count);
    const size_t nn = (size_t)nmax * nmax;
    double* buf = nullptr;  // A, then A_p, B_p, R of the timed iteration
    if (hipMalloc(reinterpret_cast<void**>(&buf), 4 * nn * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return SDC_ERR_NOMEM;
    }
    std::vector<sdc_tune_result_t> res;
    int rc = SDC_OK;
    for (int pi = 0; pi < 2 && rc == SDC_OK; ++pi) {
        for (int i = 0; i < count && rc == SDC_OK; ++i) {
            const int n = orders[i];
            sdc_tune_result_t r{n, pi ? SDC_FP32_REFINE : SDC_FP64, INFINITY, INFINITY};
            rc = sdc::run_gaussian(h, n, 0x5dc7u, 0, buf, n);
            for (int w = 0; w < 2 && rc == SDC_OK; ++w) {
                sdc_opts_t o;
                sdc_opts_default(&o);
                o.prec = r.prec;
                o.maxit = 1;  // one iteration: the work of every later one
                o.panel_width = w ? 64 : 32;
                sdc_region_t reg{SDC_HALFPLANE, 0.0, 0.0, 0.0, 1.0};
                for (int k = 0; k <= reps && rc == SDC_OK; ++k) {  // the first run warms up
                    int p = 0;
                    double rconv = 0.0;
                    if (hipStreamSynchronize(h.stream) != hipSuccess) rc = SDC_ERR_DEVICE;
                    const auto t0 = std::chrono::steady_clock::now();
                    const int st = sdc::run_irs_only(h, n, buf, n, nullptr, 0, 0, reg, o, buf + nn, buf + 2 * nn,
                                                     buf + 3 * nn, n, &p, &rconv);
                    if (st < 0) rc = st;
                    if (rc == SDC_OK && hipStreamSynchronize(h.stream) != hipSuccess) rc = SDC_ERR_DEVICE;
                    const double ms =
                        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                    if (k > 0) (w ? r.ms_nb64 : r.ms_nb32) = std::min(w ? r.ms_nb64 : r.ms_nb32, ms);
                }
            }
            res.push_back(r);
        }
    }
    (void)hipFree(buf);
    if (rc != SDC_OK) return (sdc_status_t)rc;
    // per precision: the smallest order from which 64 wins at every larger timed order
    for (int pi = 0; pi < 2; ++pi) {
        std::vector<sdc_tune_result_t> v(res.begin() + pi * count, res.begin() + (pi + 1) * count);
        std::sort(v.begin(), v.end(), [](const sdc_tune_result_t& a, const sdc_tune_result_t& b) { return a.n < b.n; });
        int lim = sdc::kNb64Never;
        for (int i = (int)v.size() - 1; i >= 0 && v[i].ms_nb64 < v[i].ms_nb32; --i) lim = v[i].n;
        h.nb64_min[pi] = lim;
    }
    if (results) std::copy(res.begin(), res.end(), results);
    return SDC_OK;
}

sdc_status_t sdc_tune_save(sdc_handle_t hd, const char* path) {
    if (!hd || !path) return SDC_ERR_INVALID;
    hipDeviceProp_t prop{};
    const bool have = hipGetDeviceProperties(&prop, hd->h.device) == hipSuccess;
    FILE* f = std::fopen(path, "w");
    if (!f) return SDC_ERR_INVALID;
    const int ok = std::fprintf(f, "{\"nb64_min_fp64\": %d, \"nb64_min_fp32\": %d, \"arch\": \"%s\"}\n",
                                tune_to_api(hd->h.nb64_min[0]), tune_to_api(hd->h.nb64_min[1]),
                                have ? prop.gcnArchName : "unknown");
    return (std::fclose(f) == 0 && ok > 0) ? SDC_OK : SDC_ERR_INVALID;
}

// Integer value of "key" in a small JSON object (found: 1, absent: 0, malformed: -1).
static int json_int(const std::string& text, const char* key, int* out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t at = text.find(k);
    if (at == std::string::npos) return 0;
    size_t i = text.find(':', at + k.size());
    if (i == std::string::npos) return -1;
    const char* b = text.c_str() + i + 1;
    char* e = nullptr;
    const long v = std::strtol(b, &e, 10);
    if (e == b || v < INT_MIN || v > INT_MAX) return -1;
    *out = (int)v;
    return 1;
}

sdc_status_t sdc_tune_load(sdc_handle_t hd, const char* path) {
    if (!hd || !path) return SDC_ERR_INVALID;
    FILE* f = std::fopen(path, "r");
    if (!f) return SDC_ERR_INVALID;
    std::string text;
    char chunk[512];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof chunk, f)) > 0 && text.size() < (1u << 16)) text.append(chunk, got);
    std::fclose(f);
    int v64 = 0, v32 = 0;
    const int a = json_int(text, "nb64_min_fp64", &v64), b = json_int(text, "nb64_min_fp32", &v32);
    if (a < 0 || b < 0 || text.find('{') == std::string::npos) return SDC_ERR_INVALID;
    if (a > 0) hd->h.nb64_min[0] = tune_from_api(v64);
    if (b > 0) hd->h.nb64_min[1] = tune_from_api(v32);
    return SDC_OK;
}

sdc_status_t sdc_split_svd(sdc_handle_t hd, int m, int n, const double* A, int lda, sdc_region_t region,
                           const sdc_opts_t* opts, double* U, int ldu, double* V, int ldv, double* S11, int lds11,
                           sdc_info_t* info) {
    const int r = std::min(m, n);
    if (!hd || m < 1 || n < 1 || m + n > kMaxN || !A || !U || !V || !S11 || lda < m || ldu < m || ldv < n ||
        lds11 < r || !region_ok(region) || region.kind != SDC_HALFPLANE || region.shift < 0.0 ||
        (m != n && region.shift == 0.0))  // |m - n| zero eigenvalues of the embedding on the line
        return SDC_ERR_INVALID;
    sdc_info_t dummy;
    if (!info) info = &dummy;
    *info = sdc_info_t{};
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    const sdc_opts_t o = resolve(opts);
    if (!prec_ok(o, false, region.kind)) return SDC_ERR_INVALID;
    int status = 0;
    sdc::ProfScope ps(h);
    const int rc = sdc::run_split_svd(h, m, n, A, lda, region, o, U, ldu, V, ldv, S11, lds11, info, &status);
    resolve_profile(h);
    if (rc < 0) return (sdc_status_t)rc;
    return (sdc_status_t)status;
}

sdc_status_t sdc_block_eigvals(sdc_handle_t hd, int n, const double* T, int ldt, const double* S, int lds,
                               int nblocks, const int* block_start, int symmetric, double* wr, double* wi,
                               double* V, int ldv) {
    if (!hd || n < 1 || !T || ldt < n || (!symmetric && (!S || lds < n)) || nblocks < 1 || nblocks > n ||
        !block_start || !wr || !wi || (V && (!symmetric || ldv < n)))
        return SDC_ERR_INVALID;
    Handle& h = hd->h;
    if (use_device(h) != SDC_OK) return SDC_ERR_DEVICE;
    return (sdc_status_t)sdc::run_block_eigvals(h, n, T, ldt, S, lds, nblocks, block_start, symmetric != 0, wr, wi,
                                                V, ldv);
}

}  // extern "C"
