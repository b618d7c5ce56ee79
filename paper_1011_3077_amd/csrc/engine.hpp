// Host-side engine of the split step: workspace, descriptor staging, and the
// batched drivers behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cmath>
#include <cstdint>
#include <vector>

#include "sdc.h"
#include "profiler.hpp"
#include "sdc_internal.hpp"

namespace sdc {

// Default panel-width table (the smallest number of factored columns that
// takes 64-column panels; kNb64Never: none).  Measured on one MI355X, the
// 64-column panels lose at every order up to 8192 in both precisions: the
// fan-in of their reduction tree drops from 8 to 4, which adds a third more
// rows to the trailing update (a seventh with 32-column panels), and their
// panel and look-ahead kernels each take a CU's whole LDS beside the bulk
// update.  sdc_autotune measures the choice for the device at hand.
constexpr int kNb64Never = 1 << 30;
constexpr int kNb64MinFp64 = kNb64Never;
constexpr int kNb64MinFp32 = kNb64Never;

struct Handle {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    // device workspace (bump-allocated per call)
    char* ws = nullptr;
    size_t ws_size = 0;
    size_t ws_off = 0;
    // descriptor staging: pinned host mirror + device arena, same offsets.
    // desc_dirty: end of the mirror bytes written since the last completed
    // wait (an asynchronous copy still queued may read them); ev_desc: event
    // recorded after the most recent copy
    char* desc_h = nullptr;
    char* desc_d = nullptr;
    size_t desc_size = 0;
    size_t desc_off = 0;
    size_t desc_dirty = 0;
    hipEvent_t ev_desc = nullptr;
    // pinned host buffer for small device-to-host results
    char* host = nullptr;
    size_t host_size = 0;
    // second device workspace, owned by the divide-and-conquer driver
    char* ws2 = nullptr;
    size_t ws2_size = 0;
    // per-tick convergence norms of the repeated squaring (4 per side)
    double* dnorm = nullptr;
    size_t dnorm_cap = 0;
    // device staging of small per-problem results read back in one copy
    double* dstage = nullptr;
    size_t dstage_cap = 0;
    // event polled by sync_spin (created on first use)
    hipEvent_t ev_sync = nullptr;
    // look-ahead stream and events of the QR (created on first use)
    QrStreams qs{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // opt-in kernel timing
    Profiler prof;
    // every buffer above was handed in from preallocated memory: the
    // ensure_* helpers report SDC_ERR_NOMEM instead of allocating
    bool no_alloc = false;
    // replay of the repeated-squaring iterations from a HIP graph
    // (sdc_graphs_enable): graphs on; the capture / replay stream and the
    // events that order it after and before `stream` (created on first use)
    bool graphs = false;
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    // QR panel width table: problems with at least nb64_min[p] factored
    // columns use 64-column panels ([0] FP64 iterates, [1] FP32 iterates);
    // set by sdc_tune_set / sdc_autotune
    int nb64_min[2] = {kNb64MinFp64, kNb64MinFp32};
    // QR schedule (sdc_tree_overlap_enable): the panel tree above the leaves
    // factored in the launch of the leaf-level trailing update
    bool tree_overlap = true;
    // QR schedule (sdc_lookahead_set): problems of at least this many
    // factored columns take the two-stream look-ahead schedule
    int la_min = kLookaheadNever;
};

// Panel width (32 or 64) of a QR with nf factored columns: `forced` (the
// caller's opts.panel_width) if it is 32 or 64, else the handle's table
// (the defaults without a handle).  It depends on the problem alone, never
// on the rest of a batch.
inline int panel_width(const Handle* h, int nf, bool fp32, int forced) {
    if (forced == 32 || forced == 64) return forced;
    const int lim = h ? h->nb64_min[fp32 ? 1 : 0] : (fp32 ? kNb64MinFp32 : kNb64MinFp64);
    return nf >= lim ? 64 : 32;
}

// Installs the handle's profiler (if enabled) for the lifetime of a call.
struct ProfScope {
    Profiler* prev;
    explicit ProfScope(Handle& h) : prev(g_prof) { g_prof = h.prof.on ? &h.prof : nullptr; }
    ~ProfScope() { g_prof = prev; }
};

// Argument checks shared by the entry points.
// Largest order the tree QR supports: 2n rows give at most 128 leaves.
constexpr int kMaxN = 16384;
static_assert(2 * kMaxN <= kMaxPanelRows, "QR tree counters sized for augmented matrices of order kMaxN");
inline bool region_ok(const sdc_region_t& r) {
    if (r.kind == SDC_UNIT_DISK) return true;
    if (r.kind == SDC_DISK) return std::isfinite(r.center) && std::isfinite(r.radius) && r.radius > 0;
    if (r.kind == SDC_HALFPLANE) return std::isfinite(r.shift) && std::isfinite(r.scale) && r.scale >= 0;
    return false;
}
// SDC_FP32_REFINE is for symmetric problems split at a half plane only: its
// refinement solves X A11 - A22 X = E by conjugate gradients, whose operator
// is positive definite only when a point separates the two eigenvalue groups.
inline bool prec_ok(const sdc_opts_t& o, bool pencil, int region_kind) {
    if (o.prec == SDC_FP64) return true;
    return o.prec == SDC_FP32_REFINE && !pencil && region_kind == SDC_HALFPLANE;
}

// One split problem (symmetric or pencil) as the drivers see it.
struct SplitJob {
    int n = 0;
    bool pencil = false;
    bool nonsym = false;  // B = I with a non-symmetric A (RNEP): A_hat not symmetrized
    const double* A = nullptr; int lda = 0;
    const double* B = nullptr; int ldb = 0;
    sdc_region_t region{};
    sdc_opts_t opts{};
    double* Q = nullptr; int ldq = 0;      // Q (symmetric) or Q_R
    double* QL = nullptr; int ldql = 0;
    double* Ahat = nullptr; int ldah = 0;
    double* Bhat = nullptr; int ldbh = 0;
    double* eprof = nullptr;  // optional device output (n doubles): e(k) for k = 1 .. n-1 of the
                              // returned split, at index k (the multi-way splits of the recursion)
    sdc_info_t info{};
    int status = 0;
};

// Runs every job; returns a negative status on argument/device failure,
// else SDC_OK (per-job statuses in job.status).
int run_split_jobs(Handle& h, std::vector<SplitJob>& jobs);
// An SDC_FP32_REFINE split that ended with this status is redone in FP64.
bool fp32_needs_fallback(int status);

// IRS alone for one side; see sdc_irs.
int run_irs_only(Handle& h, int n, const double* A, int lda, const double* B, int ldb, int transpose,
                 const sdc_region_t& region, const sdc_opts_t& opts, double* Ap, double* Bp, double* R,
                 int ldo, int* p, double* rconv);

int run_gaussian(Handle& h, int n, uint64_t seed, int tag, double* G, int ldg);
int run_split_svd(Handle& h, int m, int n, const double* A, int lda, const sdc_region_t& region,
                  const sdc_opts_t& opts, double* U, int ldu, double* V, int ldv, double* S11, int lds11,
                  sdc_info_t* info, int* status);
int run_block_eigvals(Handle& h, int n, const double* T, int ldt, const double* S, int lds, int nblocks,
                      const int* block_start, int symmetric, double* wr, double* wi, double* V, int ldv);

// Incremental driver (continuous batching).  A JobRun holds one split job's
// state in a caller-provided device workspace of job_run_bytes() bytes; each
// job_runs_tick() starts the runs not started yet, advances every run still
// in its repeated squaring by one iteration, and finishes (GRURV, block form,
// split search, refinement) the runs whose squaring ended; done[i] is set for
// runs that finished in this tick.  A run's result does not depend on which
// other runs share its ticks.
struct JobRun;
size_t job_run_bytes(const SplitJob& j);
JobRun* job_run_create(const Handle& h, SplitJob* j, char* ws, size_t bytes);
void job_run_destroy(JobRun* r);
int job_runs_tick(Handle& h, std::vector<JobRun*>& runs, std::vector<char>& done);

// Randomized divide-and-conquer; see sdc_eig_dc.
int run_eig_dc(Handle& h, int n, const double* A, int lda, const double* B, int ldb, int symmetric, int leaf_max,
               const sdc_opts_t& opts, double* T, int ldt, double* S, int lds, double* QL, int ldql, double* QR,
               int ldqr, int* nblocks, int* block_start, sdc_block_bound_t* bounds, sdc_dc_info_t* info);

}  // namespace sdc
