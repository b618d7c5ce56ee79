// Host orchestration of the split step (Alg. 3 IRS -> Alg. 2/1 GRURV ->
// Alg. 4/6 block form and split point) for a batch of independent problems.
//
// All problems of a call advance in lockstep: each IRS iteration is one
// augmented-QR pass plus one epilogue launch for every still-active side, and
// one 8-byte-per-side device-to-host copy feeds the FP64 stopping test.  The
// rank-revealing factorization, block form and split search are likewise
// batched.  Decisions that need the whole problem (rank from the GRURV
// diagonals, accept/retry) are taken on the host from a few numbers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "engine.hpp"
#include "engine_util.hpp"
#include "sdc_aux.hpp"
#include "sdc_internal.hpp"

namespace sdc {

// ---------------------------------------------------------------------------
// Region map (Sec. 3.3): A0 = a1 A + a2 B, B0 = b1 A + b2 B.
// ---------------------------------------------------------------------------
static void region_coeffs(const sdc_region_t& r, double& a1, double& a2, double& b1, double& b2) {
    if (r.kind == SDC_DISK) {
        a1 = 1; a2 = -r.center; b1 = 0; b2 = r.radius;
    } else if (r.kind == SDC_HALFPLANE) {
        const double s = r.scale > 0 ? r.scale : 1.0;
        a1 = 1; a2 = -(r.shift - s); b1 = 1; b2 = -(r.shift + s);
    } else {
        a1 = 1; a2 = 0; b1 = 0; b2 = 1;
    }
}

// ---------------------------------------------------------------------------
// Batched implicit repeated squaring (Alg. 3)
// ---------------------------------------------------------------------------
template <typename T> struct IrsSide {
    int n = 0;
    int ld = 0;  // leading dimension of W: 2n rounded up to 16 elements (aligned columns)
    const double* A = nullptr; int lda = 0;
    const double* B = nullptr; int ldb = 0;
    int trans = 0;
    double a1 = 1, a2 = 0, b1 = 0, b2 = 1;
    double tau = 0;
    int maxit = 60;
    T* W = nullptr; double* Rprev = nullptr; T* diag = nullptr; double* norms = nullptr;
    T* Tm = nullptr; unsigned* counters = nullptr;
    int nb = 32;  // QR panel width of this side (panel_width)
    int p = 0, converged = 0, nonfinite = 0;
    int started = 0, done = 0;
    double rconv = NAN;
};

// Buffers of one IRS side; s.n must be set before the call.
template <typename T> static void irs_layout(Carver& c, IrsSide<T>& s) {
    const size_t n = (size_t)s.n;
    s.ld = (2 * s.n + 15) / 16 * 16;
    s.W = c.take<T>(3 * n * (size_t)s.ld);
    s.Rprev = c.take<double>(n * n);
    s.diag = c.take<T>(n);
    s.Tm = c.take<T>(2 * qr_aux_elems<T>(2 * s.n));
    s.counters = c.take<unsigned>(kMaxInternal);
}

// aux holds 2 * qr_aux_elems<T>(m) elements (one set per panel parity, at
// the same offsets for either panel width).
template <typename T, int NBW> static void qr_desc_aux(QrDesc<T>& d, int m, T* aux) {
    using C = QrCfg<T, NBW>;
    const auto g = tree_geom<T, NBW>(m);
    size_t internal = 0;
    for (int l = 1; l < g.levels; ++l) internal += (size_t)g.L(l);
    const size_t tm = ((size_t)g.L(0) + internal) * C::NB * C::NB;
    const size_t per = qr_aux_elems<T>(m);
    for (int p = 0; p < 2; ++p) {
        d.Tm[p] = aux + p * per;
        d.Vint[p] = aux + p * per + tm;
    }
    d.tm_leaves = g.L(0);
}
template <typename T> static QrDesc<T> qr_desc(T* W, int ld, int m, int nf, int ncols, T* aux, T* diag,
                                               unsigned* counters, int nb, int la_min) {
    QrDesc<T> d;
    d.W = W; d.ld = ld; d.m = m; d.nf = nf; d.ncols = ncols;
    d.nb = nb == 64 ? 64 : 32;
    d.la_min = la_min;
    if (d.nb == 64) qr_desc_aux<T, 64>(d, m, aux);
    else qr_desc_aux<T, 32>(d, m, aux);
    d.diag = diag; d.counters = counters; d.active = 1;
    return d;
}

// Look-ahead streams for a batch of QRs, or none: only problems of at least
// the handle's look-ahead threshold (factored columns; by default none) are
// updated with look-ahead, and a single stream saves the host the event
// calls of every panel.
template <typename T> static const QrStreams* lookahead(Handle& h, const std::vector<QrDesc<T>>& q) {
    for (const QrDesc<T>& d : q)
        if (d.active && d.nf >= d.la_min) return &h.qs;
    return nullptr;
}

// The QRs of a batch, one batched call per panel width (32 first): every
// problem is factored by the kernels of its own width, whatever else is in
// the batch, so it rounds the same alone and in any batch.
template <typename T> static int run_qr_grouped(Handle& h, const std::vector<QrDesc<T>>& qd) {
    for (int nb : {32, 64}) {
        std::vector<QrDesc<T>> g;
        for (const QrDesc<T>& d : qd)
            if (d.nb == nb) g.push_back(d);
        if (g.empty()) continue;
        UPLOAD(dg, g);
        qr_aug_batch<T>(dg, g.data(), (int)g.size(), h.stream, lookahead(h, g), h.tree_overlap);
    }
    return SDC_OK;
}

// Set-up of the sides not started yet: W <- [B0 A0 0; -A0 0 B0] from the
// inputs and the region map; tree counters cleared.
template <typename T> static int irs_start(Handle& h, std::vector<IrsSide<T>*>& sides) {
    std::vector<IrsInit<T>> ini;
    std::vector<ZeroDesc> zd;
    for (IrsSide<T>* sp : sides) {
        IrsSide<T>& s = *sp;
        if (s.started) continue;
        ini.push_back(IrsInit<T>{s.W, s.n, s.ld, s.A, s.lda, s.B, s.ldb, s.a1, s.a2, s.b1, s.b2, s.trans});
        zd.push_back(ZeroDesc{s.counters, (unsigned)kMaxInternal});
        s.p = 0; s.converged = 0; s.nonfinite = 0; s.rconv = NAN; s.done = 0; s.started = 1;
    }
    if (ini.empty()) return SDC_OK;
    UPLOAD(dzd, zd);
    zero_batch(dzd, (int)zd.size(), h.stream);
    UPLOAD(dini, ini);
    irs_init_batch<T>(dini, ini.data(), (int)ini.size(), h.stream);
    return SDC_OK;
}

// One repeated-squaring iteration (QR of the stacked pair, updates, sign
// normalization and convergence test) for every started side that is not
// done, each at its own iteration count.  Sides may join between ticks.
// *left receives the number of sides still iterating.
template <typename T> static int irs_tick(Handle& h, std::vector<IrsSide<T>*>& sides, int* left) {
    std::vector<IrsSide<T>*> act;
    for (IrsSide<T>* sp : sides)
        if (sp->started && !sp->done) act.push_back(sp);
    *left = 0;
    const int cnt = (int)act.size();
    if (!cnt) return SDC_OK;
    CHK(ensure_dnorm(h, 4 * (size_t)cnt));
    CHK(ensure_host(h, sizeof(double) * 4 * cnt));
    std::vector<QrDesc<T>> qd(cnt);
    std::vector<IrsDesc<T>> pd(cnt);
    for (int i = 0; i < cnt; ++i) {
        IrsSide<T>& s = *act[i];
        s.norms = h.dnorm + 4 * i;
        qd[i] = qr_desc<T>(s.W, s.ld, 2 * s.n, s.n, 3 * s.n, s.Tm, s.diag, s.counters, s.nb, h.la_min);
        pd[i] = IrsDesc<T>{s.W, s.n, s.ld, s.Rprev, s.diag, s.norms, 1};
    }
    const size_t mark = h.desc_off;
    UPLOAD(dp, pd);
    fill<double>(h.dnorm, 4 * (size_t)cnt, 0.0, h.stream);
    CHK(ensure_streams(h));
    CHK(run_qr_grouped<T>(h, qd));
    irs_post_batch<T>(dp, pd.data(), cnt, 0, h.stream);
    HIPCHK(hipGetLastError());
    double* hn = reinterpret_cast<double*>(h.host);
    HIPCHK(hipMemcpyAsync(hn, h.dnorm, sizeof(double) * 4 * cnt, hipMemcpyDeviceToHost, h.stream));
    CHK(sync_spin(h));
    h.desc_off = mark;
    for (int i = 0; i < cnt; ++i) {
        IrsSide<T>& s = *act[i];
        const int it = s.p;  // iteration index j of Alg. 3
        const double diff = hn[4 * i], ref = hn[4 * i + 1], cur = hn[4 * i + 2];
        s.p = it + 1;
        bool stop = false;
        if (!std::isfinite(cur) || (it > 0 && !std::isfinite(diff))) {
            s.nonfinite = 1;
            stop = true;
        } else if (it > 0) {
            s.rconv = ref > 0 ? diff / ref : INFINITY;
            if (diff <= s.tau * ref) {
                s.converged = 1;
                stop = true;
            }
        }
        if (!stop && it + 1 > s.maxit) stop = true;
        if (stop) s.done = 1;
        else ++*left;
    }
    return SDC_OK;
}

// ---------------------------------------------------------------------------
// Replay of the repeated squaring from a HIP graph.  One iteration of every
// side not yet done (the fill of the norm staging, the QRs of each panel
// width with their two-stream look-ahead, the post kernel) is captured once
// on the handle's graph stream and replayed per tick.  Everything the graph
// reads stays where it was at capture: the descriptors are uploaded before
// the capture and kept in the arena until the loop ends, the norms go to
// the same staging slots, and nothing inside the capture copies memory,
// records or waits for an event, or synchronizes: it holds kernel launches
// on one stream only.  A side whose test has passed is
// switched off between replays by a four-byte copy of the `active` field of
// its resident descriptors (kernels skip inactive problems), so every
// replay runs the same launches as the direct path over the remaining sides
// and each side's result is bitwise the same.
// ---------------------------------------------------------------------------
template <typename T> struct IrsGraph {
    std::vector<IrsSide<T>*> act;
    std::vector<size_t> qoff;  // arena offset of each uploaded QrDesc (width-32 group first)
    std::vector<int> qside;    // its side (index into act)
    size_t poff = 0;           // arena offset of the IrsDesc array (one per side, act order)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    IrsGraph() = default;
    IrsGraph(const IrsGraph&) = delete;
    IrsGraph& operator=(const IrsGraph&) = delete;
    ~IrsGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

static bool use_graphs(const Handle& h) { return h.graphs && !h.prof.on && !h.no_alloc; }

// Only QRs on one stream are captured: every side below the handle's
// look-ahead threshold.  (Capturing the two-stream look-ahead schedule,
// whose second and third streams join the capture through event waits,
// ended in a host segmentation fault at order 1300, in the runtime; sides
// that take the look-ahead keep the direct launches.)
template <typename T> static bool graphable(const Handle& h, const std::vector<IrsSide<T>*>& sides) {
    for (const IrsSide<T>* sp : sides)
        if (sp->started && !sp->done && sp->n >= h.la_min) return false;
    return true;
}

template <typename T> static int irs_graph_build(Handle& h, std::vector<IrsSide<T>*>& sides, IrsGraph<T>& g) {
    if (!graphable(h, sides)) return SDC_ERR_INVALID;  // never captures the two-stream schedule
    for (IrsSide<T>* sp : sides)
        if (sp->started && !sp->done) g.act.push_back(sp);
    const int cnt = (int)g.act.size();
    if (!cnt) return SDC_OK;
    CHK(ensure_dnorm(h, 4 * (size_t)cnt));
    CHK(ensure_host(h, sizeof(double) * 4 * cnt));
    CHK(ensure_graph_stream(h));
    std::vector<QrDesc<T>> all(cnt);
    std::vector<IrsDesc<T>> pd(cnt);
    for (int i = 0; i < cnt; ++i) {
        IrsSide<T>& s = *g.act[i];
        s.norms = h.dnorm + 4 * i;
        all[i] = qr_desc<T>(s.W, s.ld, 2 * s.n, s.n, 3 * s.n, s.Tm, s.diag, s.counters, s.nb, h.la_min);
        pd[i] = IrsDesc<T>{s.W, s.n, s.ld, s.Rprev, s.diag, s.norms, 1};
    }
    std::vector<QrDesc<T>> grp[2];
    const QrDesc<T>* dgrp[2] = {nullptr, nullptr};
    for (int w = 0; w < 2; ++w) {
        for (int i = 0; i < cnt; ++i)
            if ((all[i].nb == 64) == (w == 1)) {
                grp[w].push_back(all[i]);
                g.qside.push_back(i);
            }
        if (grp[w].empty()) continue;
        UPLOAD(dv, grp[w]);
        dgrp[w] = dv;
        for (size_t j = 0; j < grp[w].size(); ++j)
            g.qoff.push_back((size_t)(reinterpret_cast<const char*>(dv + j) - h.desc_d));
    }
    UPLOAD(dp, pd);
    g.poff = (size_t)(reinterpret_cast<const char*>(dp) - h.desc_d);
    // the uploads have run before the capture starts
    HIPCHK(hipStreamSynchronize(h.stream));
    h.desc_dirty = 0;
    HIPCHK(hipStreamBeginCapture(h.gstream, hipStreamCaptureModeThreadLocal));
    fill<double>(h.dnorm, 4 * (size_t)cnt, 0.0, h.gstream);
    for (int w = 0; w < 2; ++w)
        if (!grp[w].empty())
            qr_aug_batch<T>(dgrp[w], grp[w].data(), (int)grp[w].size(), h.gstream, nullptr, h.tree_overlap);
    irs_post_batch<T>(dp, pd.data(), cnt, 0, h.gstream);
    const hipError_t launch = hipGetLastError();
    const hipError_t end = hipStreamEndCapture(h.gstream, &g.graph);
    if (launch != hipSuccess || end != hipSuccess || !g.graph) return SDC_ERR_DEVICE;
    HIPCHK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
    return SDC_OK;
}

// One replay: the same bookkeeping as irs_tick for the sides not yet done.
template <typename T> static int irs_graph_tick(Handle& h, IrsGraph<T>& g, int* left) {
    *left = 0;
    const int cnt = (int)g.act.size();
    bool any = false;
    for (IrsSide<T>* s : g.act) any = any || !s->done;
    if (!any) return SDC_OK;
    HIPCHK(hipEventRecord(h.gev[0], h.stream));
    HIPCHK(hipStreamWaitEvent(h.gstream, h.gev[0], 0));
    HIPCHK(hipGraphLaunch(g.exec, h.gstream));
    HIPCHK(hipEventRecord(h.gev[1], h.gstream));
    HIPCHK(hipStreamWaitEvent(h.stream, h.gev[1], 0));
    double* hn = reinterpret_cast<double*>(h.host);
    HIPCHK(hipMemcpyAsync(hn, h.dnorm, sizeof(double) * 4 * cnt, hipMemcpyDeviceToHost, h.stream));
    CHK(sync_spin(h));
    std::vector<int> fin;
    for (int i = 0; i < cnt; ++i) {
        IrsSide<T>& s = *g.act[i];
        if (s.done) continue;
        const int it = s.p;  // iteration index j of Alg. 3
        const double diff = hn[4 * i], ref = hn[4 * i + 1], cur = hn[4 * i + 2];
        s.p = it + 1;
        bool stop = false;
        if (!std::isfinite(cur) || (it > 0 && !std::isfinite(diff))) {
            s.nonfinite = 1;
            stop = true;
        } else if (it > 0) {
            s.rconv = ref > 0 ? diff / ref : INFINITY;
            if (diff <= s.tau * ref) {
                s.converged = 1;
                stop = true;
            }
        }
        if (!stop && it + 1 > s.maxit) stop = true;
        if (stop) {
            s.done = 1;
            fin.push_back(i);
        } else {
            ++*left;
        }
    }
    if (*left == 0 || fin.empty()) return SDC_OK;
    // switch the finished sides off before the next replay (it waits for h.stream)
    auto off = [&](size_t at) -> int {
        const int zero = 0;
        std::memcpy(h.desc_h + at, &zero, sizeof zero);
        HIPCHK(hipMemcpyAsync(h.desc_d + at, h.desc_h + at, sizeof zero, hipMemcpyHostToDevice, h.stream));
        h.desc_dirty = std::max(h.desc_dirty, at + sizeof zero);
        return SDC_OK;
    };
    for (int i : fin) {
        CHK(off(g.poff + (size_t)i * sizeof(IrsDesc<T>) + offsetof(IrsDesc<T>, active)));
        for (size_t j = 0; j < g.qside.size(); ++j)
            if (g.qside[j] == i) CHK(off(g.qoff[j] + offsetof(QrDesc<T>, active)));
    }
    return SDC_OK;
}

template <typename T> static int run_irs(Handle& h, std::vector<IrsSide<T>*>& sides) {
    if (sides.empty()) return SDC_OK;
    for (IrsSide<T>* sp : sides) sp->started = 0;
    CHK(irs_start<T>(h, sides));
    for (int left = 1; left;) CHK(irs_tick<T>(h, sides, &left));
    return SDC_OK;
}

// ---------------------------------------------------------------------------
// Rank read off the GRURV diagonals (same rule as the oracle): every ratio
// tiny -> all eigenvalues inside; none tiny -> all outside; otherwise the
// count above the largest gap of the sorted ratios.
// ---------------------------------------------------------------------------
enum Side { SIDE_INSIDE = 0, SIDE_OUTSIDE = 1, SIDE_SPLIT = 2 };
static int rank_from_rho(const std::vector<double>& rho, double& gap, int& side) {
    const int n = (int)rho.size();
    double mx = 0, mn = INFINITY;
    for (double r : rho) {
        mx = std::max(mx, std::fabs(r));
        mn = std::min(mn, std::fabs(r));
    }
    gap = 1.0;
    if (!(mx >= kRhoOneSide)) {
        side = SIDE_INSIDE;
        return 0;
    }
    if (mn > kRhoOneSide) {
        side = SIDE_OUTSIDE;
        return n;
    }
    std::vector<double> s(n);
    for (int i = 0; i < n; ++i) s[i] = std::max(std::fabs(rho[i]), 1e-300);
    std::sort(s.begin(), s.end(), std::greater<double>());
    int best = 0;
    double bg = -1;
    for (int i = 0; i + 1 < n; ++i) {
        const double r = s[i] / s[i + 1];
        if (r > bg) {
            bg = r;
            best = i;
        }
    }
    side = SIDE_SPLIT;
    gap = bg;
    return best + 1;
}

// ---------------------------------------------------------------------------
// Per-problem workspace of the FP64 stages.
// ---------------------------------------------------------------------------
struct JobWs {
    SplitJob* job = nullptr;
    IrsSide<double> sd[2];
    IrsSide<float> sf[2];
    bool fp32 = false;
    const double* Ap[2] = {nullptr, nullptr};
    const double* Bp[2] = {nullptr, nullptr};
    int ldp[2] = {0, 0};
    double* Apd[2] = {nullptr, nullptr};
    double* Bpd[2] = {nullptr, nullptr};
    double *X = nullptr, *Vt = nullptr, *T1 = nullptr, *T2 = nullptr;
    double* qaux = nullptr;
    double* dg[4] = {nullptr, nullptr, nullptr, nullptr};
    unsigned* qcnt = nullptr;
    int qnb = 32;  // panel width of the GRURV / rank-revealing QRs (FP64, n columns)
    double *SA = nullptr, *SB = nullptr, *e = nullptr, *out = nullptr, *nrm = nullptr, *orth = nullptr;
    double* cg = nullptr;  // CG partial sums of the FP64 refinement (5 x kCgMaxBlocks)
    std::vector<double> rho_r, rho_l;
    int attempt = 0, done = 0, best_attempt = -1;
    double best_e = INFINITY;
    int status = 0;
    double tau = 0;
};

static void job_layout(Carver& c, JobWs& w, const Handle* h) {
    const SplitJob& j = *w.job;
    const size_t n = (size_t)j.n;
    const int nsides = j.pencil ? 2 : 1;
    w.qnb = panel_width(h, j.n, false, j.opts.panel_width);
    for (int s = 0; s < nsides; ++s) {
        w.sf[s].n = j.n;
        w.sd[s].n = j.n;
        w.sf[s].nb = panel_width(h, j.n, true, j.opts.panel_width);
        w.sd[s].nb = panel_width(h, j.n, false, j.opts.panel_width);
        if (w.fp32) {
            irs_layout(c, w.sf[s]);
            w.Apd[s] = c.take<double>(n * n);
            w.Bpd[s] = c.take<double>(n * n);
        } else {
            irs_layout(c, w.sd[s]);
        }
    }
    w.X = c.take<double>(2 * n * n);
    w.Vt = c.take<double>(n * n);
    w.T1 = c.take<double>(n * n);
    w.T2 = c.take<double>(n * n);
    w.qaux = c.take<double>(2 * qr_aux_elems<double>((int)n));
    for (int k = 0; k < 4; ++k) w.dg[k] = c.take<double>(n);
    w.qcnt = c.take<unsigned>(kMaxInternal);
    w.SA = c.take<double>(n * n);
    w.SB = j.pencil ? c.take<double>(n * n) : nullptr;
    w.e = c.take<double>(n + 1);
    w.out = c.take<double>(2);
    w.nrm = c.take<double>(2);
    w.orth = c.take<double>(1);
    if (w.fp32 && !j.pencil) w.cg = c.take<double>(5 * (size_t)kCgMaxBlocks);
}

static EwDesc ew_perm(int n, const double* in, int ldi, double* out, int ldo, int trans, int revP, int revQ,
                      const double* sg) {
    EwDesc d{};
    d.op = EW_PERMUTE; d.n = n; d.rows = n; d.in = in; d.ldi = ldi; d.out = out; d.ldo = ldo;
    d.trans = trans; d.revP = revP; d.revQ = revQ; d.sg = sg; d.alpha = 1.0; d.active = 1;
    return d;
}
static EwDesc ew_ident(int n, double* out, int ldo) {
    EwDesc d{};
    d.op = EW_IDENTITY; d.n = n; d.rows = n; d.out = out; d.ldo = ldo; d.alpha = 1.0; d.active = 1;
    return d;
}
static EwDesc ew_add(int n, const double* a, int lda, const double* b, int ldb, double* out, int ldo) {
    EwDesc d{};
    d.op = EW_ADD; d.n = n; d.rows = n; d.in = a; d.ldi = lda; d.in2 = b; d.ld2 = ldb; d.out = out; d.ldo = ldo;
    d.alpha = 1.0; d.active = 1;
    return d;
}
static GemmDesc<double> gemm(int n, const double* A, int lda, int ta, const double* B, int ldb, int tb, double* C,
                             int ldc) {
    GemmDesc<double> g{};
    g.A = A; g.B = B; g.C = C; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.M = n; g.N = n; g.K = n; g.ta = ta; g.tb = tb; g.alpha = 1.0; g.beta = 0.0; g.active = 1;
    return g;
}

static GemmDesc<double> gemm_g(int M, int N, int K, const double* A, int lda, int ta, const double* B, int ldb,
                               int tb, double* C, int ldc, double alpha, double beta) {
    GemmDesc<double> g{};
    g.A = A; g.B = B; g.C = C; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K; g.ta = ta; g.tb = tb; g.alpha = alpha; g.beta = beta; g.active = 1;
    return g;
}
static EwDesc ew_copy(int rows, int cols, const double* in, int ldi, double* out, int ldo) {
    EwDesc d{};
    d.op = EW_PERMUTE; d.n = cols; d.rows = rows; d.in = in; d.ldi = ldi; d.out = out; d.ldo = ldo;
    d.alpha = 1.0; d.active = 1;
    return d;
}

static int run_ew(Handle& h, const std::vector<EwDesc>& v) {
    if (v.empty()) return SDC_OK;
    UPLOAD(d, v);
    ew_batch<double, double>(d, v.data(), (int)v.size(), h.stream);
    return SDC_OK;
}
static int run_gemm(Handle& h, const std::vector<GemmDesc<double>>& v) {
    if (v.empty()) return SDC_OK;
    UPLOAD(d, v);
    gemm_batch<double>(d, v.data(), (int)v.size(), h.stream);
    return SDC_OK;
}
static int run_qr(Handle& h, std::vector<JobWs*>& js, int dgi) {
    std::vector<QrDesc<double>> q;
    for (JobWs* w : js) {
        const int n = w->job->n;
        q.push_back(qr_desc<double>(w->X, n, n, n, 2 * n, w->qaux, w->dg[dgi], w->qcnt, w->qnb, h.la_min));
    }
    if (q.empty()) return SDC_OK;
    CHK(ensure_streams(h));
    return run_qr_grouped<double>(h, q);
}

// X[:, 0:n] <- the Gaussian of (attempt, side); X[:, n:2n] <- I.
static int stage_gaussian(Handle& h, std::vector<JobWs*>& js, int side) {
    std::vector<EwDesc> copies;
    std::vector<GaussDesc> draws;
    std::vector<EwDesc> ids;
    for (JobWs* w : js) {
        const SplitJob& j = *w->job;
        const int n = j.n;
        if (j.opts.G) {
            const double* G = j.opts.G + (size_t)(w->attempt * 2 + side) * n * n;
            copies.push_back(ew_perm(n, G, n, w->X, n, 0, 0, 0, nullptr));
        } else {
            GaussDesc g{};
            g.G = w->X; g.ld = n; g.n = n; g.seed = j.opts.seed + (uint64_t)w->attempt; g.tag = side; g.active = 1;
            draws.push_back(g);
        }
        ids.push_back(ew_ident(n, w->X + (size_t)n * n, n));
    }
    CHK(run_ew(h, copies));
    if (!draws.empty()) {
        UPLOAD(d, draws);
        gauss_batch(d, draws.data(), (int)draws.size(), h.stream);
    }
    CHK(run_ew(h, ids));
    return SDC_OK;
}

// Alg. 2 with k = 2, m = (-1, 1): Q_R = GRURV(2, A_p + B_p, A_p, -1, 1).
// RURV of A_p (V from QR of the Gaussian, sign-fixed; A_p V^T = U R2), then
// RQ of U^T (A_p + B_p) = R1 W by the reversal J, Q_R = W^T.  Writes Q_R to
// job.Q and the diagonals of R2 (dg[1]) and of the reversed R1 (dg[2]).
static int grurv_right(Handle& h, std::vector<JobWs*>& js) {
    CHK(stage_gaussian(h, js, 0));
    CHK(run_qr(h, js, 0));
    std::vector<EwDesc> e1, e2, e3, e4;
    std::vector<GemmDesc<double>> g1;
    for (JobWs* w : js) {
        const int n = w->job->n;
        double* Xr = w->X + (size_t)n * n;
        e1.push_back(ew_perm(n, Xr, n, w->Vt, n, 0, 0, 0, w->dg[0]));              // V^T = diag(s) Q_G^T
        g1.push_back(gemm(n, w->Ap[0], w->ldp[0], 0, w->Vt, n, 0, w->X, n));        // A_p V^T
        e2.push_back(ew_add(n, w->Ap[0], w->ldp[0], w->Bp[0], w->ldp[0], Xr, n));   // A_p + B_p
    }
    CHK(run_ew(h, e1));
    CHK(run_gemm(h, g1));
    CHK(run_ew(h, e2));
    CHK(run_qr(h, js, 1));  // U^T (A_p + B_p) in the right block, R2 diagonal in dg[1]
    for (JobWs* w : js) {
        const int n = w->job->n;
        double* Xr = w->X + (size_t)n * n;
        // Y = J (diag(s2) U^T(A_p+B_p))^T J
        e3.push_back(ew_perm(n, Xr, n, w->X, n, 1, 1, 1, w->dg[1]));
        e4.push_back(ew_ident(n, Xr, n));
    }
    CHK(run_ew(h, e3));
    CHK(run_ew(h, e4));
    CHK(run_qr(h, js, 2));
    std::vector<EwDesc> e5;
    for (JobWs* w : js) {
        const int n = w->job->n;
        // Q_R = J Qt diag(s3) J
        e5.push_back(ew_perm(n, w->X + (size_t)n * n, n, w->job->Q, w->job->ldq, 1, 1, 1, w->dg[2]));
    }
    CHK(run_ew(h, e5));
    return SDC_OK;
}

// Alg. 2 with k = 2, m = (1, -1) on the transposed pencil's iterates:
// Q_L = GRURV(2, A_p'^T, (A_p' + B_p')^T, 1, -1).  RULV of A_p' + B_p'
// (QL through the column reversal: (A_p'+B_p') V^T J = Qt Rt, U = Qt J),
// then QR of A_p'^T U.  Writes Q_L to job.QL, the diagonal of the reversed L
// (dg[1]) and of R1 (dg[2]).
static int grurv_left(Handle& h, std::vector<JobWs*>& js) {
    CHK(stage_gaussian(h, js, 1));
    CHK(run_qr(h, js, 0));
    std::vector<EwDesc> e1, e2, e3;
    std::vector<GemmDesc<double>> g1;
    for (JobWs* w : js) {
        const int n = w->job->n;
        double* Xr = w->X + (size_t)n * n;
        e1.push_back(ew_perm(n, Xr, n, w->Vt, n, 0, 0, 1, w->dg[0]));                  // V^T J
        e2.push_back(ew_add(n, w->Ap[1], w->ldp[1], w->Bp[1], w->ldp[1], w->T1, n));    // A_p' + B_p'
        g1.push_back(gemm(n, w->T1, n, 0, w->Vt, n, 0, w->X, n));                       // (A_p'+B_p') V^T J
        e3.push_back(ew_ident(n, Xr, n));
    }
    CHK(run_ew(h, e1));
    CHK(run_ew(h, e2));
    CHK(run_gemm(h, g1));
    CHK(run_ew(h, e3));
    CHK(run_qr(h, js, 1));
    std::vector<EwDesc> e4, e5;
    std::vector<GemmDesc<double>> g2;
    for (JobWs* w : js) {
        const int n = w->job->n;
        double* Xr = w->X + (size_t)n * n;
        e4.push_back(ew_perm(n, Xr, n, w->Vt, n, 1, 1, 0, w->dg[1]));                   // U = Qt diag(s) J
        g2.push_back(gemm(n, w->Ap[1], w->ldp[1], 1, w->Vt, n, 0, w->X, n));            // A_p'^T U
        e5.push_back(ew_ident(n, Xr, n));
    }
    CHK(run_ew(h, e4));
    CHK(run_gemm(h, g2));
    CHK(run_ew(h, e5));
    CHK(run_qr(h, js, 2));
    std::vector<EwDesc> e6;
    for (JobWs* w : js) {
        const int n = w->job->n;
        e6.push_back(ew_perm(n, w->X + (size_t)n * n, n, w->job->QL, w->job->ldql, 1, 0, 0, w->dg[2]));
    }
    CHK(run_ew(h, e6));
    return SDC_OK;
}

// Block form (Alg. 4 line 5 / Alg. 6 line 3) with the original A, B.
static int block_form(Handle& h, std::vector<JobWs*>& js) {
    std::vector<GemmDesc<double>> g1, g2;
    std::vector<EwDesc> es;
    for (JobWs* w : js) {
        SplitJob& j = *w->job;
        const int n = j.n;
        g1.push_back(gemm(n, j.A, j.lda, 0, j.Q, j.ldq, 0, w->T1, n));
        if (j.pencil) {
            g1.push_back(gemm(n, j.B, j.ldb, 0, j.Q, j.ldq, 0, w->T2, n));
            g2.push_back(gemm(n, j.QL, j.ldql, 1, w->T1, n, 0, j.Ahat, j.ldah));
            g2.push_back(gemm(n, j.QL, j.ldql, 1, w->T2, n, 0, j.Bhat, j.ldbh));
        } else {
            g2.push_back(gemm(n, j.Q, j.ldq, 1, w->T1, n, 0, w->T2, n));
            // symmetric: (A_hat + A_hat^T) / 2 (Alg. 6); RNEP keeps Q^T A Q as is
            EwDesc d{};
            d.op = j.nonsym ? EW_PERMUTE : EW_SYM; d.n = n; d.rows = n; d.in = w->T2; d.ldi = n;
            d.out = j.Ahat; d.ldo = j.ldah;
            d.alpha = 1.0; d.active = 1;
            es.push_back(d);
        }
    }
    CHK(run_gemm(h, g1));
    CHK(run_gemm(h, g2));
    CHK(run_ew(h, es));
    return SDC_OK;
}

static int split_search(Handle& h, std::vector<JobWs*>& js) {
    std::vector<SplitDesc> sd;
    for (JobWs* w : js) {
        SplitJob& j = *w->job;
        SplitDesc d{};
        d.Ah = j.Ahat; d.lda = j.ldah;
        d.Bh = j.pencil ? j.Bhat : nullptr; d.ldb = j.ldbh;
        d.n = j.n; d.SA = w->SA; d.SB = w->SB; d.norms = w->nrm; d.e = w->e; d.out = w->out; d.active = 1;
        sd.push_back(d);
    }
    if (sd.empty()) return SDC_OK;
    UPLOAD(d, sd);
    split_search_batch(d, sd.data(), (int)sd.size(), h.stream);
    return SDC_OK;
}

// Read back the diagonals of the GRURV triangular factors and form the rank
// statistic rho = |diag(R1^{m1} R2^{m2})|.
static int fetch_rho(Handle& h, std::vector<JobWs*>& js, bool left) {
    std::vector<GatherDesc> gd;
    size_t off = 0;
    for (JobWs* w : js) {
        const int n = w->job->n;
        gd.push_back(GatherDesc{w->dg[1], (long long)off, n});
        gd.push_back(GatherDesc{w->dg[2], (long long)(off + n), n});
        off += 2 * (size_t)n;
    }
    double* hb = nullptr;
    CHK(read_back(h, gd, hb));
    off = 0;
    for (JobWs* w : js) {
        const int n = w->job->n;
        const double* d1 = hb + off;
        const double* d2 = d1 + n;
        std::vector<double>& rho = left ? w->rho_l : w->rho_r;
        rho.assign(n, 0.0);
        for (int i = 0; i < n; ++i) {
            // right: |R2_ii| / |R1_ii| with R1_ii = Rt_{n-1-i} (RQ by reversal)
            // left:  |R1_ii| / |L_ii|  with L_ii  = Rt_{n-1-i} (QL by reversal)
            rho[i] = left ? std::fabs(d2[i]) / std::fabs(d1[n - 1 - i])
                          : std::fabs(d1[i]) / std::fabs(d2[n - 1 - i]);
        }
        off += 2 * (size_t)n;
    }
    return SDC_OK;
}

static int fetch_search(Handle& h, std::vector<JobWs*>& js) {
    std::vector<GatherDesc> gd;
    for (size_t q = 0; q < js.size(); ++q) gd.push_back(GatherDesc{js[q]->out, (long long)(2 * q), 2});
    double* hb = nullptr;
    CHK(read_back(h, gd, hb));
    for (size_t q = 0; q < js.size(); ++q) {
        js[q]->job->info.k_lead = (int)hb[2 * q];
        js[q]->job->info.e21_rel = hb[2 * q + 1];
    }
    return SDC_OK;
}

// One GRURV + block form + split search pass for the jobs in js, each at its
// own w->attempt.
static int split_pass(Handle& h, std::vector<JobWs*>& js) {
    if (js.empty()) return SDC_OK;
    CHK(grurv_right(h, js));
    CHK(fetch_rho(h, js, false));
    std::vector<JobWs*> pen;
    for (JobWs* w : js)
        if (w->job->pencil) pen.push_back(w);
    if (!pen.empty()) {
        CHK(grurv_left(h, pen));
        CHK(fetch_rho(h, pen, true));
    }
    CHK(block_form(h, js));
    CHK(split_search(h, js));
    HIPCHK(hipGetLastError());
    CHK(fetch_search(h, js));
    return SDC_OK;
}

static bool sides_converged(const JobWs& w) {
    const int ns = w.job->pencil ? 2 : 1;
    for (int s = 0; s < ns; ++s)
        if (!(w.fp32 ? w.sf[s].converged : w.sd[s].converged)) return false;
    return true;
}

// ---------------------------------------------------------------------------
// FP64 refinement of a symmetric split whose repeated squaring ran in FP32
// (an addition to the paper, which has no mixed precision).
//
// With A_hat = Q^T A Q = [A11 E^T; E A22] (E = A_hat[k:, :k]) and
// U = [I -X^T; X I], the (2,1) block of U^T A_hat U is, to first order in X,
// E + A22 X - X A11; it vanishes when X solves the Sylvester equation
// X A11 - A22 X = E, which CG solves on the device (positive definite when
// A11's eigenvalues lie above A22's, as for a half-plane split).  Since
// U^T U = diag(I + X^T X, I + X X^T), Q U (I + ...)^{-1/2} stays orthogonal;
// the inverse square roots are applied to first order, I - X^T X / 2 and
// I - X X^T / 2 (error O(|X|^4)), followed by one Newton-Schulz step toward
// the polar factor.  Each Newton round squares E's size; the block form and
// split search are then recomputed in FP64.
// ---------------------------------------------------------------------------
constexpr int kRefineRounds = 3;
constexpr int kCgMaxIt = 240;
constexpr int kCgCheck = 8;       // iterations between host convergence checks
constexpr double kCgTol = 1e-6;   // relative residual of each Newton correction
constexpr double kRefineMaxE = 1e-2;

static bool wants_refine(JobWs& w) {
    SplitJob& j = *w.job;
    if (!w.fp32 || j.pencil || !w.cg) return false;
    double gap = 1;
    int side = SIDE_SPLIT;
    const int krho = rank_from_rho(w.rho_r, gap, side);
    const int k = j.info.k_lead;
    const double e = j.info.e21_rel;
    return side == SIDE_SPLIT && k == krho && k > 0 && k < j.n && !(e <= j.opts.split_tol) && e < kRefineMaxE;
}

// Element-wise conversion between FP64 and FP32 copies (rows x cols).
static EwDesc ew_conv(int rows, int cols, const void* in, int ldi, void* out, int ldo) {
    EwDesc d{};
    d.op = EW_PERMUTE; d.n = cols; d.rows = rows; d.in = in; d.ldi = ldi; d.out = out; d.ldo = ldo;
    d.alpha = 1.0; d.active = 1;
    return d;
}

// Conjugate gradients on X A11 - A22 X = E.  The recurrences, inner
// products and the right-hand side are FP64; the operator products
// Z = P A11 - A22 P run on FP32 copies of A11, A22 and P (MFMA FP32 GEMMs at
// half the bytes): a correction only has to be accurate to about the CG
// tolerance, well above the FP32 product error, and the Newton residual
// E is recomputed in FP64 after every round.
static int cg_solve(Handle& h, std::vector<JobWs*>& js) {
    const int count = (int)js.size();
    std::vector<CgDesc> cg;
    std::vector<GemmDesc<float>> g1, g2;
    std::vector<EwDesc> prep, to32, to64;
    for (JobWs* w : js) {
        SplitJob& j = *w->job;
        const int n = j.n, k = j.info.k_lead, m = n - k;
        const size_t mk = (size_t)m * k;
        CgDesc d{};
        d.m = m; d.k = k; d.E = j.Ahat + k; d.lde = j.ldah;
        d.X = w->X; d.R = w->X + mk; d.P = w->X + 2 * mk; d.Z = w->X + 3 * mk;
        d.rr = w->cg; d.rr0 = w->cg + 3 * kCgMaxBlocks; d.pz = w->cg + 4 * kCgMaxBlocks;
        d.tol2 = kCgTol * kCgTol; d.nblk = cg_blocks(m, k); d.active = 1;
        cg.push_back(d);
        // FP32 copies in the second half of X (n^2 doubles hold the
        // (m + k)^2 floats of A11, A22, P and Z; the CG vectors use 4 m k <= n^2)
        float* a11 = reinterpret_cast<float*>(w->X + (size_t)n * n);
        float* a22 = a11 + (size_t)k * k;
        float* pf = a22 + (size_t)m * m;
        float* zf = pf + mk;
        prep.push_back(ew_conv(k, k, j.Ahat, j.ldah, a11, k));
        prep.push_back(ew_conv(m, m, j.Ahat + k + (size_t)k * j.ldah, j.ldah, a22, m));
        to32.push_back(ew_conv(m, k, d.P, m, pf, m));
        to64.push_back(ew_conv(m, k, zf, m, d.Z, m));
        // Z = P A11 - A22 P
        GemmDesc<float> e1{};
        e1.A = pf; e1.lda = m; e1.B = a11; e1.ldb = k; e1.C = zf; e1.ldc = m;
        e1.M = m; e1.N = k; e1.K = k; e1.alpha = 1.0f; e1.beta = 0.0f; e1.active = 1;
        g1.push_back(e1);
        GemmDesc<float> e2{};
        e2.A = a22; e2.lda = m; e2.B = pf; e2.ldb = m; e2.C = zf; e2.ldc = m;
        e2.M = m; e2.N = k; e2.K = m; e2.alpha = -1.0f; e2.beta = 1.0f; e2.active = 1;
        g2.push_back(e2);
    }
    UPLOAD(dcg, cg);
    UPLOAD(dg1, g1);
    UPLOAD(dg2, g2);
    UPLOAD(dprep, prep);
    UPLOAD(d32, to32);
    UPLOAD(d64, to64);
    ew_batch<double, float>(dprep, prep.data(), (int)prep.size(), h.stream);
    size_t need = 0;
    for (const CgDesc& d : cg) need += 2 * (size_t)d.nblk;
    CHK(ensure_host(h, need * sizeof(double) + 64));
    CHK(ensure_dstage(h, need + 1));
    cg_init_batch(dcg, cg.data(), count, h.stream);
    for (int it = 0; it < kCgMaxIt; ++it) {
        ew_batch<double, float>(d32, to32.data(), count, h.stream);
        gemm_batch<float>(dg1, g1.data(), count, h.stream);
        gemm_batch<float>(dg2, g2.data(), count, h.stream);
        ew_batch<float, double>(d64, to64.data(), count, h.stream);
        for (int ph = 0; ph < 3; ++ph) cg_iter_vec(dcg, cg.data(), count, it, ph, h.stream);
        if ((it + 1) % kCgCheck != 0) continue;
        HIPCHK(hipGetLastError());
        // stop launching once every problem is frozen (the device decides;
        // this only saves launches)
        std::vector<GatherDesc> gd;
        size_t off = 0;
        for (const CgDesc& d : cg) {
            gd.push_back(GatherDesc{d.rr + ((it + 1) % 3) * kCgMaxBlocks, (long long)off, d.nblk});
            gd.push_back(GatherDesc{d.rr0, (long long)(off + d.nblk), d.nblk});
            off += 2 * (size_t)d.nblk;
        }
        double* hb = nullptr;
        CHK(read_back(h, gd, hb));
        bool all = true;
        off = 0;
        for (const CgDesc& d : cg) {
            double rr = 0, r0 = 0;
            for (int b = 0; b < d.nblk; ++b) {
                rr += hb[off + b];
                r0 += hb[off + d.nblk + b];
            }
            // slack: the device sums in another order
            if (!(rr <= d.tol2 * r0 * (1 + 1e-9))) all = false;
            off += 2 * (size_t)d.nblk;
        }
        if (all) break;
    }
    HIPCHK(hipGetLastError());
    return SDC_OK;
}

// Q <- Q U with the first-order orthonormalization (see above).
static int apply_correction(Handle& h, std::vector<JobWs*>& js) {
    std::vector<EwDesc> c1, c2;
    std::vector<GemmDesc<double>> u1, u2;
    for (JobWs* w : js) {
        SplitJob& j = *w->job;
        const int n = j.n, k = j.info.k_lead, m = n - k;
        const double* X = w->X;
        double* T1 = w->T1;
        double* S1 = w->T2;
        double* S2 = w->T2 + (size_t)k * k;
        c1.push_back(ew_copy(n, n, j.Q, j.ldq, T1, n));
        u1.push_back(gemm_g(n, k, m, j.Q + (size_t)k * j.ldq, j.ldq, 0, X, m, 0, T1, n, 1.0, 1.0));   // Q1 + Q2 X
        u1.push_back(gemm_g(n, m, k, j.Q, j.ldq, 0, X, m, 1, T1 + (size_t)k * n, n, -1.0, 1.0));      // Q2 - Q1 X^T
        u1.push_back(gemm_g(k, k, m, X, m, 1, X, m, 0, S1, k, 1.0, 0.0));                            // X^T X
        u1.push_back(gemm_g(m, m, k, X, m, 0, X, m, 1, S2, m, 1.0, 0.0));                            // X X^T
        c2.push_back(ew_copy(n, n, T1, n, j.Q, j.ldq));
        u2.push_back(gemm_g(n, k, k, T1, n, 0, S1, k, 0, j.Q, j.ldq, -0.5, 1.0));
        u2.push_back(gemm_g(n, m, m, T1 + (size_t)k * n, n, 0, S2, m, 0, j.Q + (size_t)k * j.ldq, j.ldq, -0.5, 1.0));
    }
    CHK(run_ew(h, c1));
    CHK(run_gemm(h, u1));
    CHK(run_ew(h, c2));
    CHK(run_gemm(h, u2));
    // one Newton-Schulz step toward the polar factor, Q <- Q (I - (Q^T Q - I)/2):
    // removes the O(|X|^4) loss of orthogonality left by the first-order
    // inverse square roots (and any rounding drift), to O(|X|^8)
    std::vector<EwDesc> e1, e2;
    std::vector<GemmDesc<double>> g1, g2;
    for (JobWs* w : js) {
        SplitJob& j = *w->job;
        const int n = j.n;
        e1.push_back(ew_ident(n, w->T1, n));
        g1.push_back(gemm_g(n, n, n, j.Q, j.ldq, 1, j.Q, j.ldq, 0, w->T1, n, 1.0, -1.0));
        e2.push_back(ew_copy(n, n, j.Q, j.ldq, w->T2, n));
        g2.push_back(gemm_g(n, n, n, w->T2, n, 0, w->T1, n, 0, j.Q, j.ldq, -0.5, 1.0));
    }
    CHK(run_ew(h, e1));
    CHK(run_gemm(h, g1));
    CHK(run_ew(h, e2));
    CHK(run_gemm(h, g2));
    return SDC_OK;
}

// FP32 iterates leave ||E21|| at the rank-revealed split of order
// eps32 |A| / gap.  At large n that can exceed e(k) of the trivial splits next
// to k = 1 or k = n - 1 (one border row or column has a small 1-norm), so when
// the split-search minimum k* is such a border split the refinement starts
// from the rank the GRURV diagonals reveal instead: e(k_rho) is read back and
// taken as the candidate.  An interior k* that disagrees with k_rho is left
// alone (the attempt is retried with a new draw).
static int pin_to_rank(Handle& h, std::vector<JobWs*>& js) {
    std::vector<JobWs*> alt;
    std::vector<int> ks;
    for (JobWs* w : js) {
        if (!w->fp32 || w->job->pencil || !w->cg) continue;
        double gap = 1;
        int side = SIDE_SPLIT;
        const int krho = rank_from_rho(w->rho_r, gap, side);
        const int n = w->job->n, kstar = w->job->info.k_lead;
        const int border = std::max(2, n / 64);
        if (side != SIDE_SPLIT || krho == kstar || krho < 1 || krho >= n) continue;
        if (std::min(kstar, n - kstar) > border) continue;
        alt.push_back(w);
        ks.push_back(krho);
    }
    if (alt.empty()) return SDC_OK;
    std::vector<GatherDesc> gd;
    for (size_t q = 0; q < alt.size(); ++q) gd.push_back(GatherDesc{alt[q]->e + ks[q], (long long)q, 1});
    double* hb = nullptr;
    CHK(read_back(h, gd, hb));
    for (size_t q = 0; q < alt.size(); ++q) {
        alt[q]->job->info.k_lead = ks[q];
        alt[q]->job->info.e21_rel = hb[q];
    }
    return SDC_OK;
}

static int refine(Handle& h, std::vector<JobWs*> js) {
    for (int round = 0; round < kRefineRounds && !js.empty(); ++round) {
        const size_t mark = h.desc_off;
        CHK(cg_solve(h, js));
        CHK(apply_correction(h, js));
        CHK(block_form(h, js));
        CHK(split_search(h, js));
        HIPCHK(hipGetLastError());
        CHK(fetch_search(h, js));
        CHK(pin_to_rank(h, js));
        h.desc_off = mark;
        std::vector<JobWs*> next;
        for (JobWs* w : js) {
            w->job->info.refine_rounds = round + 1;
            if (wants_refine(*w)) next.push_back(w);
        }
        js.swap(next);
    }
    return SDC_OK;
}

// GRURV, block form and split search, then the FP64 refinement where the
// repeated squaring ran in FP32.
static int split_pass_refined(Handle& h, std::vector<JobWs*>& js) {
    CHK(split_pass(h, js));
    CHK(pin_to_rank(h, js));
    std::vector<JobWs*> ref;
    for (JobWs* w : js) {
        w->job->info.refine_rounds = 0;
        if (wants_refine(*w)) ref.push_back(w);
    }
    if (!ref.empty()) CHK(refine(h, ref));
    return SDC_OK;
}

// Accept / retry / classify one attempt (Alg. 4: the split point minimizes
// the backward error e(k) and the split is accepted when e(k*) <= split_tol;
// the rank read off the GRURV diagonals decides only whether every
// eigenvalue lies on one side, and is reported).  A pencil whose right and
// left sides disagree about that is retried with a new draw, as a split above
// split_tol is.  Returns true when the job is finished.
static bool decide(JobWs& w, bool& needs_best) {
    SplitJob& j = *w.job;
    const int n = j.n;
    double gap = 1, gapl = 1;
    int side = SIDE_SPLIT, sidel = SIDE_SPLIT;
    const int krho = rank_from_rho(w.rho_r, gap, side);
    if (j.pencil) rank_from_rho(w.rho_l, gapl, sidel);
    else sidel = side;
    const bool conv = sides_converged(w);
    needs_best = false;
    j.info.k_rho = krho;
    j.info.rank_gap = j.pencil ? std::min(gap, gapl) : gap;
    j.info.attempts = w.attempt + 1;
    if (side != SIDE_SPLIT && side == sidel) {
        const int k = side == SIDE_INSIDE ? 0 : n;
        w.status = conv ? SDC_NO_SPLIT : SDC_NOT_CONVERGED;
        j.info.k_lead = k;
        j.info.n_inside = n - k;
        j.info.e21_rel = 0.0;
        return true;
    }
    if (side != sidel) {
        // the two sides disagree about the spectrum being one-sided: a bad
        // draw, or iterates short of convergence
        if (w.attempt < j.opts.max_retries) {
            ++w.attempt;
            return false;
        }
        w.status = conv ? SDC_RANK_AMBIGUOUS : SDC_NOT_CONVERGED;
        needs_best = w.best_attempt >= 0 && w.best_attempt != w.attempt;
        if (!needs_best) {
            j.info.k_lead = -1;
            j.info.n_inside = -1;
            j.info.e21_rel = HUGE_VAL;
        }
        return true;
    }
    const int ks = j.info.k_lead;
    const double es = j.info.e21_rel;
    j.info.n_inside = n - ks;
    if (es < w.best_e) {
        w.best_e = es;
        w.best_attempt = w.attempt;
    }
    if (es <= j.opts.split_tol) {
        w.status = conv ? SDC_OK : SDC_NOT_CONVERGED;
        return true;
    }
    if (w.attempt < j.opts.max_retries) {
        ++w.attempt;
        return false;
    }
    w.status = conv ? SDC_RANK_AMBIGUOUS : SDC_NOT_CONVERGED;
    needs_best = w.best_attempt >= 0 && w.best_attempt != w.attempt;
    return true;
}

static void fill_defaults(sdc_opts_t& o) {
    if (o.maxit <= 0) o.maxit = 60;
    if (o.split_tol <= 0) o.split_tol = 1e-10;
    if (o.max_retries < 0) o.max_retries = 0;
}

// Side parameters of a job (the region map and the tolerances).
static void setup_sides(JobWs& w) {
    SplitJob& j = *w.job;
    double a1, a2, b1, b2;
    region_coeffs(j.region, a1, a2, b1, b2);
    const int ns = j.pencil ? 2 : 1;
    for (int s = 0; s < ns; ++s) {
        auto setup = [&](auto& side, double eps) {
            side.n = j.n; side.A = j.A; side.lda = j.lda;
            side.B = j.pencil ? j.B : nullptr; side.ldb = j.ldb;
            side.trans = s; side.a1 = a1; side.a2 = a2; side.b1 = b1; side.b2 = b2;
            side.tau = j.opts.tau > 0 ? j.opts.tau : std::sqrt(eps);
            side.maxit = j.opts.maxit;
            side.started = 0; side.done = 0;
        };
        if (w.fp32) setup(w.sf[s], (double)std::numeric_limits<float>::epsilon());
        else setup(w.sd[s], std::numeric_limits<double>::epsilon());
    }
}

static void collect_sides(std::vector<JobWs*>& js, std::vector<IrsSide<double>*>& sd,
                          std::vector<IrsSide<float>*>& sf) {
    for (JobWs* w : js) {
        const int ns = w->job->pencil ? 2 : 1;
        for (int s = 0; s < ns; ++s) {
            if (w->fp32) sf.push_back(&w->sf[s]);
            else sd.push_back(&w->sd[s]);
        }
    }
}

static bool irs_finished(const JobWs& w) {
    const int ns = w.job->pencil ? 2 : 1;
    for (int s = 0; s < ns; ++s)
        if (!(w.fp32 ? w.sf[s].done : w.sd[s].done)) return false;
    return true;
}

static int finish_jobs(Handle& h, std::vector<JobWs*>& wsp);

bool fp32_needs_fallback(int status) {
    return status != SDC_OK && status != SDC_NO_SPLIT;
}

int run_split_jobs(Handle& h, std::vector<SplitJob>& jobs) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<JobWs> ws(jobs.size());
    for (size_t i = 0; i < jobs.size(); ++i) {
        fill_defaults(jobs[i].opts);
        ws[i].job = &jobs[i];
        ws[i].fp32 = jobs[i].opts.prec == SDC_FP32_REFINE;
    }
    // workspace: size pass, then carve
    auto layout = [&](Carver& c) {
        for (JobWs& w : ws) job_layout(c, w, &h);
    };
    {
        Carver c0(nullptr);
        layout(c0);
        CHK(ensure_ws(h, c0.off + 4096));
    }
    Carver c(h.ws, h.ws_size);
    layout(c);
    if (c.overflow) return SDC_ERR_NOMEM;
    CHK(ensure_desc(h, (size_t)(64 << 10) + jobs.size() * (size_t)(8 << 10)));
    h.desc_off = 0;

    // IRS on every side: FP64 and FP32 sides advance one iteration per tick,
    // each until its own convergence test passes
    std::vector<JobWs*> wsp;
    for (JobWs& w : ws) {
        setup_sides(w);
        wsp.push_back(&w);
    }
    std::vector<IrsSide<double>*> sd;
    std::vector<IrsSide<float>*> sf;
    collect_sides(wsp, sd, sf);
    CHK(irs_start<double>(h, sd));
    CHK(irs_start<float>(h, sf));
    if (use_graphs(h)) {
        // per precision: replayed from a graph, or launched directly.  The
        // norm staging is sized for both precisions first: a graph keeps the
        // address it was captured with, so nothing may reallocate it while
        // the loop runs (the direct ticks then find it large enough).
        size_t most = 0, c64 = 0, c32 = 0;
        for (IrsSide<double>* sp : sd) c64 += (sp->started && !sp->done) ? 1 : 0;
        for (IrsSide<float>* sp : sf) c32 += (sp->started && !sp->done) ? 1 : 0;
        most = std::max(c64, c32);
        CHK(ensure_dnorm(h, 4 * most));
        CHK(ensure_host(h, sizeof(double) * 4 * most));
        IrsGraph<double> g64;
        IrsGraph<float> g32;
        const bool gr64 = graphable(h, sd), gr32 = graphable(h, sf);
        if (gr64) CHK(irs_graph_build<double>(h, sd, g64));
        if (gr32) CHK(irs_graph_build<float>(h, sf, g32));
        for (int l64 = 1, l32 = 1; l64 || l32;) {
            if (gr64) CHK(irs_graph_tick<double>(h, g64, &l64));
            else CHK(irs_tick<double>(h, sd, &l64));
            if (gr32) CHK(irs_graph_tick<float>(h, g32, &l32));
            else CHK(irs_tick<float>(h, sf, &l32));
        }
    } else {
        for (int l64 = 1, l32 = 1; l64 || l32;) {
            CHK(irs_tick<double>(h, sd, &l64));
            CHK(irs_tick<float>(h, sf, &l32));
        }
    }
    h.desc_off = 0;
    CHK(finish_jobs(h, wsp));
    HIPCHK(hipStreamSynchronize(h.stream));
    // FP32 attempts that all failed: redo those problems in FP64 (the
    // workspace above is free again; every result has reached its outputs)
    std::vector<SplitJob> redo;
    std::vector<size_t> at;
    for (size_t i = 0; i < jobs.size(); ++i)
        if (ws[i].fp32 && fp32_needs_fallback(jobs[i].status)) {
            redo.push_back(jobs[i]);
            redo.back().opts.prec = SDC_FP64;
            redo.back().info = sdc_info_t{};
            at.push_back(i);
        }
    if (!redo.empty()) {
        CHK(run_split_jobs(h, redo));
        for (size_t q = 0; q < redo.size(); ++q) {
            jobs[at[q]].status = redo[q].status;
            jobs[at[q]].info = redo[q].info;
            jobs[at[q]].info.fp64_fallback = 1;
        }
    }
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (JobWs& w : ws) w.job->info.ms = ms;
    return SDC_OK;
}

// Everything after the repeated squaring, for jobs whose sides are all done:
// FP64 views of (A_p, B_p), input norms, GRURV + block form + split search
// with retries (and the FP64 refinement for FP32 jobs), diagnostics, status.
static int finish_jobs(Handle& h, std::vector<JobWs*>& wsp) {
    // views of (A_p, B_p) in FP64; norms of the inputs
    std::vector<EwDesc> conv;
    std::vector<NormDesc> nrm;
    std::vector<ZeroDesc> zd;
    std::vector<JobWs*> live;
    for (JobWs* wp : wsp) {
        JobWs& w = *wp;
        SplitJob& j = *w.job;
        const int n = j.n;
        j.info.n = n;
        const int ns = j.pencil ? 2 : 1;
        bool bad = false;
        for (int s = 0; s < ns; ++s) {
            if (w.fp32) {
                IrsSide<float>& S = w.sf[s];
                bad |= S.nonfinite != 0;
                EwDesc a{}, b{};
                a.op = b.op = EW_PERMUTE; a.n = b.n = n; a.rows = b.rows = n; a.alpha = b.alpha = 1.0;
                a.active = b.active = 1;
                a.in = S.W + (size_t)n * S.ld; a.ldi = S.ld; a.out = w.Apd[s]; a.ldo = n;
                b.in = S.W; b.ldi = S.ld; b.out = w.Bpd[s]; b.ldo = n;
                conv.push_back(a);
                conv.push_back(b);
                w.Ap[s] = w.Apd[s]; w.Bp[s] = w.Bpd[s]; w.ldp[s] = n;
                if (s == 0) { j.info.iters_right = S.p; j.info.rconv_last = S.rconv; }
                else j.info.iters_left = S.p;
            } else {
                IrsSide<double>& S = w.sd[s];
                bad |= S.nonfinite != 0;
                w.Ap[s] = S.W + (size_t)n * S.ld; w.Bp[s] = S.W; w.ldp[s] = S.ld;
                if (s == 0) { j.info.iters_right = S.p; j.info.rconv_last = S.rconv; }
                else j.info.iters_left = S.p;
            }
        }
        if (bad) {
            w.status = SDC_ERR_NONFINITE;
            continue;
        }
        zd.push_back(ZeroDesc{reinterpret_cast<unsigned*>(w.nrm), 4u});
        zd.push_back(ZeroDesc{reinterpret_cast<unsigned*>(w.orth), 2u});
        zd.push_back(ZeroDesc{w.qcnt, (unsigned)kMaxInternal});
        nrm.push_back(NormDesc{j.A, j.lda, n, n, w.nrm, 1});
        if (j.pencil) nrm.push_back(NormDesc{j.B, j.ldb, n, n, w.nrm + 1, 1});
        live.push_back(&w);
    }
    if (!zd.empty()) {
        UPLOAD(dzd, zd);
        zero_batch(dzd, (int)zd.size(), h.stream);
    }
    if (!conv.empty()) {
        UPLOAD(dc, conv);
        ew_batch<float, double>(dc, conv.data(), (int)conv.size(), h.stream);
    }
    if (!nrm.empty()) {
        UPLOAD(dn, nrm);
        norm1_batch(dn, nrm.data(), (int)nrm.size(), h.stream);
    }

    // rank-revealing factorization, block form, split point; retries
    std::vector<JobWs*> redo;
    while (!live.empty()) {
        const size_t mark = h.desc_off;
        CHK(split_pass_refined(h, live));
        h.desc_off = mark;
        std::vector<JobWs*> next;
        for (JobWs* w : live) {
            bool needs_best = false;
            if (!decide(*w, needs_best)) next.push_back(w);
            else if (needs_best) redo.push_back(w);
        }
        live.swap(next);
    }
    if (!redo.empty()) {
        // recompute the attempt with the smallest e(k*) (deterministic draws)
        std::vector<sdc_info_t> keep;
        for (JobWs* w : redo) {
            keep.push_back(w->job->info);
            w->attempt = w->best_attempt;
        }
        CHK(split_pass_refined(h, redo));
        for (size_t q = 0; q < redo.size(); ++q) {
            SplitJob& j = *redo[q]->job;
            const int k = j.info.k_lead, rr = j.info.refine_rounds;
            const double e = j.info.e21_rel;
            j.info = keep[q];
            j.info.k_lead = k;
            j.info.e21_rel = e;
            j.info.refine_rounds = rr;
            j.info.n_inside = j.n - k;
        }
        h.desc_off = 0;
    }

    // the e(k) profile of the returned split, where the caller wants it
    {
        std::vector<EwDesc> ep;
        for (JobWs* w : wsp) {
            SplitJob& j = *w->job;
            if (!j.eprof || w->status != SDC_OK || j.n < 2) continue;
            EwDesc d{};
            d.op = EW_PERMUTE; d.n = 1; d.rows = j.n; d.in = w->e; d.ldi = j.n; d.out = j.eprof; d.ldo = j.n;
            d.alpha = 1.0; d.active = 1;
            ep.push_back(d);
        }
        if (!ep.empty()) {
            UPLOAD(dep, ep);
            ew_batch<double, double>(dep, ep.data(), (int)ep.size(), h.stream);
        }
    }

    // diagnostics: ||Q^T Q - I||_F
    std::vector<GemmDesc<double>> go;
    std::vector<NormDesc> no;
    std::vector<JobWs*> diag_jobs;
    for (JobWs* wp : wsp) {
        JobWs& w = *wp;
        SplitJob& j = *w.job;
        if (!j.opts.diagnostics || w.status < 0) continue;
        go.push_back(gemm(j.n, j.Q, j.ldq, 1, j.Q, j.ldq, 0, w.T1, j.n));
        no.push_back(NormDesc{w.T1, j.n, j.n, j.n, w.orth, 1});
        diag_jobs.push_back(&w);
    }
    if (!go.empty()) {
        CHK(run_gemm(h, go));
        UPLOAD(dno, no);
        orth_err_batch(dno, no.data(), (int)no.size(), h.stream);
        std::vector<GatherDesc> gd;
        for (size_t q = 0; q < diag_jobs.size(); ++q) gd.push_back(GatherDesc{diag_jobs[q]->orth, (long long)q, 1});
        double* hb = nullptr;
        CHK(read_back(h, gd, hb));
        for (size_t q = 0; q < diag_jobs.size(); ++q) diag_jobs[q]->job->info.orth_err = std::sqrt(hb[q]);
    }
    HIPCHK(hipStreamSynchronize(h.stream));
    for (JobWs* w : wsp) w->job->status = w->status;
    return SDC_OK;
}

// ---------------------------------------------------------------------------
// Incremental driver for continuous batching: a job owns its workspace and
// advances by ticks; jobs may start and finish between ticks.
// ---------------------------------------------------------------------------
struct JobRun {
    JobWs w;
    bool finished = false;
};

size_t job_run_bytes(const SplitJob& j0) {
    SplitJob j = j0;
    fill_defaults(j.opts);
    JobWs w;
    w.job = &j;
    w.fp32 = j.opts.prec == SDC_FP32_REFINE;
    Carver c(nullptr);
    job_layout(c, w, nullptr);  // the size does not depend on the panel widths
    return c.off + 256;
}

JobRun* job_run_create(const Handle& h, SplitJob* j, char* ws, size_t bytes) {
    fill_defaults(j->opts);
    JobRun* r = new (std::nothrow) JobRun;
    if (!r) return nullptr;
    r->w.job = j;
    r->w.fp32 = j->opts.prec == SDC_FP32_REFINE;
    Carver c(ws, bytes);
    job_layout(c, r->w, &h);
    if (c.overflow) {
        delete r;
        return nullptr;
    }
    setup_sides(r->w);
    return r;
}

void job_run_destroy(JobRun* r) { delete r; }

int job_runs_tick(Handle& h, std::vector<JobRun*>& runs, std::vector<char>& done) {
    done.assign(runs.size(), 0);
    CHK(ensure_desc(h, (size_t)(64 << 10) + runs.size() * (size_t)(8 << 10)));
    h.desc_off = 0;  // every earlier tick ended with a stream synchronization
    std::vector<JobWs*> wsp;
    for (JobRun* r : runs)
        if (!r->finished) wsp.push_back(&r->w);
    std::vector<IrsSide<double>*> sd;
    std::vector<IrsSide<float>*> sf;
    collect_sides(wsp, sd, sf);
    CHK(irs_start<double>(h, sd));
    CHK(irs_start<float>(h, sf));
    int l64 = 0, l32 = 0;
    CHK(irs_tick<double>(h, sd, &l64));
    CHK(irs_tick<float>(h, sf, &l32));
    std::vector<JobWs*> fin;
    std::vector<size_t> idx;
    for (size_t i = 0; i < runs.size(); ++i)
        if (!runs[i]->finished && irs_finished(runs[i]->w)) {
            fin.push_back(&runs[i]->w);
            idx.push_back(i);
        }
    if (!fin.empty()) {
        h.desc_off = 0;
        CHK(finish_jobs(h, fin));
        for (size_t i : idx) {
            runs[i]->finished = true;
            done[i] = 1;
        }
    }
    HIPCHK(hipStreamSynchronize(h.stream));
    return SDC_OK;
}

int run_irs_only(Handle& h, int n, const double* A, int lda, const double* B, int ldb, int transpose,
                 const sdc_region_t& region, const sdc_opts_t& opts_in, double* Ap, double* Bp, double* R,
                 int ldo, int* p, double* rconv) {
    sdc_opts_t opts = opts_in;
    fill_defaults(opts);
    double a1, a2, b1, b2;
    region_coeffs(region, a1, a2, b1, b2);
    const bool fp32 = opts.prec == SDC_FP32_REFINE;
    IrsSide<double> sdd;
    IrsSide<float> sff;
    auto setup = [&](auto& side, double eps) {
        side.n = n; side.A = A; side.lda = lda; side.B = B; side.ldb = ldb; side.trans = transpose;
        side.a1 = a1; side.a2 = a2; side.b1 = b1; side.b2 = b2;
        side.tau = opts.tau > 0 ? opts.tau : std::sqrt(eps);
        side.maxit = opts.maxit;
    };
    sdd.n = n;
    sff.n = n;
    sdd.nb = panel_width(&h, n, false, opts.panel_width);
    sff.nb = panel_width(&h, n, true, opts.panel_width);
    auto layout = [&](Carver& c) {
        if (fp32) irs_layout(c, sff);
        else irs_layout(c, sdd);
    };
    {
        Carver c0(nullptr);
        layout(c0);
        CHK(ensure_ws(h, c0.off + 4096));
    }
    Carver c(h.ws, h.ws_size);
    layout(c);
    if (c.overflow) return SDC_ERR_NOMEM;
    CHK(ensure_desc(h, 64 << 10));
    h.desc_off = 0;
    int nonfinite, converged;
    const void* W;
    if (fp32) {
        setup(sff, (double)std::numeric_limits<float>::epsilon());
        std::vector<IrsSide<float>*> v{&sff};
        CHK(run_irs<float>(h, v));
        nonfinite = sff.nonfinite; converged = sff.converged; *p = sff.p; *rconv = sff.rconv; W = sff.W;
    } else {
        setup(sdd, std::numeric_limits<double>::epsilon());
        std::vector<IrsSide<double>*> v{&sdd};
        CHK(run_irs<double>(h, v));
        nonfinite = sdd.nonfinite; converged = sdd.converged; *p = sdd.p; *rconv = sdd.rconv; W = sdd.W;
    }
    h.desc_off = 0;
    if (nonfinite) return SDC_ERR_NONFINITE;
    std::vector<EwDesc> cp;
    auto mk = [&](const void* in, int ldi, double* out) {
        EwDesc d{};
        d.op = EW_PERMUTE; d.n = n; d.rows = n; d.in = in; d.ldi = ldi; d.out = out; d.ldo = ldo;
        d.alpha = 1.0; d.active = 1;
        cp.push_back(d);
    };
    const int ldw = fp32 ? sff.ld : sdd.ld;
    const size_t off_a = (size_t)n * ldw;
    if (fp32) {
        mk(static_cast<const float*>(W) + off_a, ldw, Ap);
        mk(W, ldw, Bp);
    } else {
        mk(static_cast<const double*>(W) + off_a, ldw, Ap);
        mk(W, ldw, Bp);
    }
    UPLOAD(dcp, cp);
    if (fp32) ew_batch<float, double>(dcp, cp.data(), (int)cp.size(), h.stream);
    else ew_batch<double, double>(dcp, cp.data(), (int)cp.size(), h.stream);
    if (R) {
        std::vector<EwDesc> rc;
        EwDesc d{};
        d.op = EW_PERMUTE; d.n = n; d.rows = n; d.in = fp32 ? sff.Rprev : sdd.Rprev; d.ldi = n; d.out = R;
        d.ldo = ldo; d.alpha = 1.0; d.active = 1;
        rc.push_back(d);
        UPLOAD(drc, rc);
        ew_batch<double, double>(drc, rc.data(), 1, h.stream);
    }
    HIPCHK(hipStreamSynchronize(h.stream));
    return converged ? SDC_OK : SDC_NOT_CONVERGED;
}

int run_gaussian(Handle& h, int n, uint64_t seed, int tag, double* G, int ldg) {
    CHK(ensure_desc(h, 64 << 10));
    h.desc_off = 0;
    std::vector<GaussDesc> v(1);
    v[0].G = G; v[0].ld = ldg; v[0].n = n; v[0].seed = seed; v[0].tag = tag; v[0].active = 1;
    UPLOAD(d, v);
    gauss_batch(d, v.data(), 1, h.stream);
    HIPCHK(hipStreamSynchronize(h.stream));
    return SDC_OK;
}

}  // namespace sdc
