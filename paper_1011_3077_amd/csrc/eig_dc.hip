// Randomized spectral divide-and-conquer driver (Sec. 3.3-3.5): repeated
// split steps on the diagonal blocks of a block-triangular pencil until every
// block has order <= leaf_max.
//
// Each recursion level is one batched call of the split engine over all the
// blocks still to be divided (the blocks are independent; Sec. 4.3 hands them
// to disjoint processor sets, here they share the GPU's launches).  After a
// block [s, e) is split by (Q_L', Q_R') with leading size k, the global pair
// is updated:   T[s:e, s:e] <- A_hat',   T[s+k:e, s:s+k] <- 0 (E21 dropped),
//               T[s:e, e:n] <- Q_L'^T T[s:e, e:n],  T[0:s, s:e] <- T[0:s, s:e] Q_R',
// likewise S, and the accumulated Q_L[:, s:e] <- Q_L[:, s:e] Q_L',
// Q_R[:, s:e] <- Q_R[:, s:e] Q_R'.
//
// Split curves: symmetric blocks use a random point of the middle half of
// their interval (initially the Gershgorin interval, Sec. 3.4).  Pencils use
// the unit circle first.  When a circle finds every eigenvalue inside, the
// radius shrinks through 2^{-2^k} until a circle splits the spectrum or finds
// it all outside; the last radius with everything inside is then the
// smallest bounding circle, and the block continues with random vertical
// lines through the middle half of that disk.  When everything is outside,
// the radius grows through 2^{2^k} the same way, and the largest circle with
// everything outside (radius r) leads to the swapped pair (B, A), whose
// eigenvalues are the reciprocals and lie inside 1/r (Sec. 3.5).  A circle
// that meets the pseudospectrum (no convergence, no split within split_tol)
// is retried at a randomly perturbed radius; a block whose circles fail
// repeatedly while none has worked is given up and flagged near-singular
// (every curve meets its pseudospectrum, Sec. 3.5).  A block whose lines fail
// repeatedly is given up with the bound the search reached (a block of the
// Schur form with a bound on its pseudospectrum, Sec. 3.6).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <random>
#include <vector>

#include "engine.hpp"
#include "engine_util.hpp"
#include "sdc_aux.hpp"
#include "sdc_internal.hpp"

namespace sdc {

namespace {

enum Mode { MODE_CIRCLE = 0, MODE_LINE = 1 };

struct Block {
    int s = 0, e = 0;
    int swapped = 0;     // pencil split as (S_block, T_block): eigenvalues 1/lambda
    int mode = MODE_LINE;
    double lo = -1, hi = 1;  // interval of real parts (line mode)
    double radius = 1;       // circle mode: the circle tried next; line mode: |mu| bound
    double rprev = 1;        // circle mode: the previous radius of the search
    int dir = 0;             // circle mode: 0 first circle, -1 shrinking, +1 growing
    int tries = 0;           // consecutive failed curves
    int unsplit = 0;
};

constexpr int kMaxTries = 8;         // failed lines before a block is given up
constexpr int kMaxCircleFails = 3;   // failed circles before a block is given up (near-singular)
constexpr double kRadiusMin = 0x1p-1000, kRadiusMax = 0x1p+1000;  // exponent range of the search

// Continue a pencil block with lines inside the disk |mu| <= r (swap: on the
// reciprocal pair).
Block to_lines(Block b, double r, bool swap) {
    b.mode = MODE_LINE;
    b.lo = -r;
    b.hi = r;
    b.radius = r;
    b.swapped ^= swap ? 1 : 0;
    b.tries = 0;
    return b;
}

// Next state of a circle-mode block whose circle found every eigenvalue on
// one side (Sec. 3.5): the search never turns around.
Block circle_no_split(const Block& b, bool all_inside) {
    const double r = b.radius;
    if (all_inside) {
        if (b.dir > 0) return to_lines(b, 1.0 / b.rprev, true);  // growing: rprev had all outside
        const double nr = r >= 1.0 ? 0.5 : r * r;
        if (nr < kRadiusMin) return to_lines(b, r, false);
        Block nb = b;
        nb.radius = nr; nb.rprev = r; nb.dir = -1; nb.tries = 0;
        return nb;
    }
    if (b.dir < 0) return to_lines(b, b.rprev, false);          // shrinking: rprev had all inside
    const double nr = r <= 1.0 ? 2.0 : r * r;
    if (nr > kRadiusMax) return to_lines(b, 1.0 / r, true);
    Block nb = b;
    nb.radius = nr; nb.rprev = r; nb.dir = 1; nb.tries = 0;
    return nb;
}

// The bound on a leaf block's eigenvalues mu (mu = 1/lambda when inverted).
sdc_block_bound_t block_bound(const Block& b, bool symmetric) {
    sdc_block_bound_t o{};
    o.unsplit = b.unsplit;
    if (symmetric) {
        o.re_lo = b.lo; o.re_hi = b.hi; o.radius = std::max(std::fabs(b.lo), std::fabs(b.hi));
        return o;
    }
    if (b.mode == MODE_LINE) {
        o.re_lo = b.lo; o.re_hi = b.hi; o.radius = b.radius; o.inverted = b.swapped;
    } else if (b.dir < 0) {
        o.re_lo = -b.rprev; o.re_hi = b.rprev; o.radius = b.rprev; o.inverted = b.swapped;
    } else if (b.dir > 0) {
        o.re_lo = -1.0 / b.rprev; o.re_hi = 1.0 / b.rprev; o.radius = 1.0 / b.rprev; o.inverted = !b.swapped;
    } else {
        o.re_lo = -INFINITY; o.re_hi = INFINITY; o.radius = INFINITY; o.inverted = b.swapped;
    }
    return o;
}

int ensure_ws2(Handle& h, size_t bytes) {
    if (bytes <= h.ws2_size) return SDC_OK;
    if (h.ws2) {
        HIPCHK(hipStreamSynchronize(h.stream));
        HIPCHK(hipFree(h.ws2));
        h.ws2 = nullptr;
        h.ws2_size = 0;
    }
    const size_t sz = bytes + bytes / 8 + (1 << 20);
    if (hipMalloc(&h.ws2, sz) != hipSuccess) {
        (void)hipGetLastError();
        return SDC_ERR_NOMEM;
    }
    h.ws2_size = sz;
    return SDC_OK;
}

EwDesc copy_desc(int rows, int cols, const double* in, int ldi, double* out, int ldo) {
    EwDesc d{};
    d.op = EW_PERMUTE; d.n = cols; d.rows = rows; d.in = in; d.ldi = ldi; d.out = out; d.ldo = ldo;
    d.alpha = 1.0; d.active = 1;
    return d;
}
EwDesc zero_desc(int rows, int cols, double* out, int ldo) {
    EwDesc d{};
    d.op = EW_ZERO; d.n = cols; d.rows = rows; d.out = out; d.ldo = ldo; d.alpha = 1.0; d.active = 1;
    return d;
}
EwDesc ident_desc(int n, double* out, int ldo) {
    EwDesc d{};
    d.op = EW_IDENTITY; d.n = n; d.rows = n; d.out = out; d.ldo = ldo; d.alpha = 1.0; d.active = 1;
    return d;
}
GemmDesc<double> gemm_desc(int M, int N, int K, const double* A, int lda, int ta, const double* B, int ldb, int tb,
                           double* C, int ldc) {
    GemmDesc<double> g{};
    g.A = A; g.B = B; g.C = C; g.lda = lda; g.ldb = ldb; g.ldc = ldc;
    g.M = M; g.N = N; g.K = K; g.ta = ta; g.tb = tb; g.alpha = 1.0; g.beta = 0.0; g.active = 1;
    return g;
}

int launch_ew(Handle& h, const std::vector<EwDesc>& v) {
    if (v.empty()) return SDC_OK;
    UPLOAD(d, v);
    ew_batch<double, double>(d, v.data(), (int)v.size(), h.stream);
    return SDC_OK;
}
int launch_gemm(Handle& h, const std::vector<GemmDesc<double>>& v) {
    if (v.empty()) return SDC_OK;
    UPLOAD(d, v);
    gemm_batch<double>(d, v.data(), (int)v.size(), h.stream);
    return SDC_OK;
}

}  // namespace

int run_eig_dc(Handle& h, int n, const double* A, int lda, const double* B, int ldb, int symmetric, int leaf_max,
               const sdc_opts_t& opts, double* T, int ldt, double* S, int lds, double* QL, int ldql, double* QR,
               int ldqr, int* nblocks, int* block_start, sdc_block_bound_t* bounds, sdc_dc_info_t* info) {
    const auto t0 = std::chrono::steady_clock::now();
    CHK(ensure_desc(h, (size_t)(256 << 10)));
    h.desc_off = 0;
    std::mt19937_64 rng(opts.seed * 6364136223846793005ull + 1442695040888963407ull);
    std::uniform_real_distribution<double> U(0.0, 1.0);

    // T <- A, S <- B, accumulated factors <- I
    {
        std::vector<EwDesc> init;
        init.push_back(copy_desc(n, n, A, lda, T, ldt));
        if (!symmetric) init.push_back(copy_desc(n, n, B, ldb, S, lds));
        if (QL) init.push_back(ident_desc(n, QL, ldql));
        if (QR) init.push_back(ident_desc(n, QR, ldqr));
        CHK(launch_ew(h, init));
    }
    Block top;
    top.s = 0;
    top.e = n;
    if (symmetric) {
        // Gershgorin interval of A
        CHK(ensure_ws2(h, sizeof(double) * 2 * (size_t)n));
        double* gb = reinterpret_cast<double*>(h.ws2);
        std::vector<GershDesc> gd(1);
        gd[0] = GershDesc{A, lda, n, gb, 1};
        UPLOAD(dg, gd);
        gersh_batch(dg, gd.data(), 1, h.stream);
        CHK(ensure_host(h, sizeof(double) * 2 * (size_t)n));
        HIPCHK(hipMemcpyAsync(h.host, gb, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, h.stream));
        HIPCHK(hipStreamSynchronize(h.stream));
        const double* hb = reinterpret_cast<const double*>(h.host);
        double lo = INFINITY, hi = -INFINITY;
        for (int j = 0; j < n; ++j) {
            lo = std::min(lo, hb[2 * j]);
            hi = std::max(hi, hb[2 * j + 1]);
        }
        if (!std::isfinite(lo) || !std::isfinite(hi)) return SDC_ERR_NONFINITE;
        if (hi <= lo) hi = lo + 1.0;
        top.mode = MODE_LINE;
        top.lo = lo;
        top.hi = hi;
        top.radius = std::max(std::fabs(lo), std::fabs(hi));
    } else {
        top.mode = MODE_CIRCLE;
        top.radius = 1.0;
    }
    h.desc_off = 0;

    std::vector<Block> leaves, work;
    if (n <= leaf_max) leaves.push_back(top);
    else work.push_back(top);
    sdc_dc_info_t st{};
    st.n = n;
    uint64_t split_id = 0;

    while (!work.empty()) {
        ++st.levels;
        // ---- output buffers of this level's split steps
        const int cnt = (int)work.size();
        std::vector<size_t> off(cnt);
        size_t need = 0;
        for (int i = 0; i < cnt; ++i) {
            const size_t m = (size_t)(work[i].e - work[i].s);
            off[i] = need;
            // QR', QL', Ahat', Bhat', row temp (2 x m x (n-e)), col temp (2 x s x m), factor temp (2 x n x m)
            need += 4 * m * m + 2 * m * (size_t)(n - work[i].e) + 2 * (size_t)work[i].s * m + 2 * (size_t)n * m;
            need = (need + 31) & ~size_t(31);
        }
        // e(k) profiles of the split steps, back to back (for multi-way splits)
        std::vector<size_t> poff(cnt);
        const size_t prof0 = need;
        for (int i = 0; i < cnt; ++i) {
            poff[i] = need - prof0;
            need += (size_t)(work[i].e - work[i].s);
        }
        const size_t prof_len = need - prof0;
        need = (need + 31) & ~size_t(31);
        CHK(ensure_ws2(h, need * sizeof(double) + 4096));
        double* base = reinterpret_cast<double*>(h.ws2);
        double* prof = base + prof0;

        std::vector<SplitJob> jobs(cnt);
        std::vector<sdc_region_t> regs(cnt);
        for (int i = 0; i < cnt; ++i) {
            Block& b = work[i];
            const int m = b.e - b.s;
            double* o = base + off[i];
            SplitJob& j = jobs[i];
            j.n = m;
            j.pencil = !symmetric;
            double* Tb = T + b.s + (size_t)b.s * ldt;
            double* Sb = symmetric ? nullptr : S + b.s + (size_t)b.s * lds;
            j.A = b.swapped ? Sb : Tb;
            j.lda = b.swapped ? lds : ldt;
            j.B = b.swapped ? Tb : Sb;
            j.ldb = b.swapped ? ldt : lds;
            sdc_region_t r{};
            if (b.mode == MODE_CIRCLE) {
                r.kind = SDC_DISK;
                r.center = 0.0;
                r.radius = b.radius;
            } else {
                const double c = 0.5 * (b.lo + b.hi), R = 0.5 * (b.hi - b.lo);
                r.kind = SDC_HALFPLANE;
                r.shift = c + (U(rng) - 0.5) * R;
                r.scale = R > 0 ? R : 1.0;
            }
            regs[i] = r;
            j.region = r;
            j.opts = opts;
            j.opts.seed = opts.seed + 7919ull * (++split_id);
            j.Q = o; j.ldq = m;
            j.QL = o + (size_t)m * m; j.ldql = m;
            j.Ahat = o + 2 * (size_t)m * m; j.ldah = m;
            j.Bhat = o + 3 * (size_t)m * m; j.ldbh = m;
            j.eprof = prof + poff[i];
            if (symmetric) j.QL = nullptr;
        }
        CHK(run_split_jobs(h, jobs));
        h.desc_off = 0;
        CHK(ensure_host(h, prof_len * sizeof(double) + 64));
        HIPCHK(hipMemcpyAsync(h.host, prof, prof_len * sizeof(double), hipMemcpyDeviceToHost, h.stream));
        HIPCHK(hipStreamSynchronize(h.stream));
        const std::vector<double> hprof(reinterpret_cast<const double*>(h.host),
                                        reinterpret_cast<const double*>(h.host) + prof_len);

        // ---- classify, and collect the global updates of accepted splits
        std::vector<EwDesc> put, zero, back1, back2;
        std::vector<GemmDesc<double>> rows, cols, facs;
        std::vector<Block> next;
        for (int i = 0; i < cnt; ++i) {
            Block& b = work[i];
            SplitJob& j = jobs[i];
            const int m = b.e - b.s;
            ++st.splits;
            const double m3 = (double)m * m * m;
            st.iters_total += j.info.iters_right + (symmetric ? 0 : j.info.iters_left);
            st.nominal_flops += symmetric ? (40.0 / 3.0 * j.info.iters_right + 16.0) * m3
                                          : (40.0 / 3.0 * (j.info.iters_right + j.info.iters_left) + 32.0) * m3;
            if (j.status < 0 && j.status != SDC_ERR_NONFINITE) return j.status;
            const int k = j.info.k_lead;
            const bool ok = j.status == SDC_OK && k > 0 && k < m;
            if (!ok) {
                Block nb = b;
                if (j.status == SDC_NO_SPLIT) {
                    // progress: the search narrows
                    const bool all_inside = j.info.n_inside == m;
                    if (b.mode == MODE_CIRCLE) {
                        nb = circle_no_split(b, all_inside);
                    } else {
                        // the line missed the spectrum: the interval shrinks (Sec. 3.4)
                        if (all_inside) nb.hi = regs[i].shift;
                        else nb.lo = regs[i].shift;
                        nb.tries = 0;
                        if (!(nb.hi > nb.lo)) nb.tries = kMaxTries;
                    }
                } else {
                    // the curve met the pseudospectrum: perturb the circle, or draw a new line
                    ++nb.tries;
                    if (b.mode == MODE_CIRCLE) nb.radius = b.radius * std::exp2(U(rng) - 0.5);
                }
                if (nb.tries >= (nb.mode == MODE_CIRCLE ? kMaxCircleFails : kMaxTries)) {
                    ++st.unsplit;
                    if (nb.mode == MODE_CIRCLE) ++st.near_singular;
                    nb.unsplit = 1;
                    leaves.push_back(nb);
                } else {
                    next.push_back(nb);
                }
                continue;
            }
            ++st.accepted;
            st.e21_max = std::max(st.e21_max, j.info.e21_rel);
            double* o = base + off[i];
            const double* Qr = j.Q;
            const double* Ql = symmetric ? j.Q : j.QL;
            const double* Ah = b.swapped ? j.Bhat : j.Ahat;
            const double* Bh = b.swapped ? j.Ahat : j.Bhat;
            double* rowt = o + 4 * (size_t)m * m;
            double* colt = rowt + 2 * (size_t)m * (n - b.e);
            double* fact = colt + 2 * (size_t)b.s * m;
            // split points: k, and every other k' whose coupling blocks are as
            // small (e(k') <= split_tol): the step may divide the block into
            // more than two (the remark after Alg. 4)
            std::vector<int> cuts;
            const double* ep = hprof.data() + poff[i];
            for (int kk = 1; kk < m; ++kk)
                if (kk == k || ep[kk] <= j.opts.split_tol) cuts.push_back(kk);
            st.extra_splits += (int)cuts.size() - 1;
            put.push_back(copy_desc(m, m, Ah, m, T + b.s + (size_t)b.s * ldt, ldt));
            if (!symmetric) put.push_back(copy_desc(m, m, Bh, m, S + b.s + (size_t)b.s * lds, lds));
            for (int kk : cuts) {
                zero.push_back(zero_desc(m - kk, kk, T + (b.s + kk) + (size_t)b.s * ldt, ldt));
                if (!symmetric) zero.push_back(zero_desc(m - kk, kk, S + (b.s + kk) + (size_t)b.s * lds, lds));
                // symmetric: the dropped coupling block is E21 and E21^T
                else zero.push_back(zero_desc(kk, m - kk, T + b.s + (size_t)(b.s + kk) * ldt, ldt));
            }
            // For symmetric A both coupling blocks are dropped at every split,
            // so T stays block diagonal and the row/column updates would
            // multiply zero blocks: only the factor is accumulated.
            const int nr = symmetric ? 0 : n - b.e;
            if (nr > 0) {
                rows.push_back(gemm_desc(m, nr, m, Ql, m, 1, T + b.s + (size_t)b.e * ldt, ldt, 0, rowt, m));
                back1.push_back(copy_desc(m, nr, rowt, m, T + b.s + (size_t)b.e * ldt, ldt));
                if (!symmetric) {
                    rows.push_back(gemm_desc(m, nr, m, Ql, m, 1, S + b.s + (size_t)b.e * lds, lds, 0,
                                             rowt + (size_t)m * nr, m));
                    back1.push_back(copy_desc(m, nr, rowt + (size_t)m * nr, m, S + b.s + (size_t)b.e * lds, lds));
                }
            }
            if (b.s > 0 && !symmetric) {
                cols.push_back(gemm_desc(b.s, m, m, T + (size_t)b.s * ldt, ldt, 0, Qr, m, 0, colt, b.s));
                back2.push_back(copy_desc(b.s, m, colt, b.s, T + (size_t)b.s * ldt, ldt));
                if (!symmetric) {
                    cols.push_back(gemm_desc(b.s, m, m, S + (size_t)b.s * lds, lds, 0, Qr, m, 0,
                                             colt + (size_t)b.s * m, b.s));
                    back2.push_back(copy_desc(b.s, m, colt + (size_t)b.s * m, b.s, S + (size_t)b.s * lds, lds));
                }
            }
            if (QR) {
                facs.push_back(gemm_desc(n, m, m, QR + (size_t)b.s * ldqr, ldqr, 0, Qr, m, 0, fact, n));
                back2.push_back(copy_desc(n, m, fact, n, QR + (size_t)b.s * ldqr, ldqr));
            }
            if (QL) {
                facs.push_back(gemm_desc(n, m, m, QL + (size_t)b.s * ldql, ldql, 0, Ql, m, 0,
                                         fact + (size_t)n * m, n));
                back2.push_back(copy_desc(n, m, fact + (size_t)n * m, n, QL + (size_t)b.s * ldql, ldql));
            }
            // children: leading block(s) = eigenvalues outside the curve, the
            // trailing one(s) inside; the pieces of a multi-way split inherit
            // the bound of their side
            Block c1 = b, c2 = b;
            c1.tries = c2.tries = 0;
            if (b.mode == MODE_CIRCLE) {
                // outside the circle r: reciprocals inside 1/r; inside: lines inside r
                c1 = to_lines(c1, 1.0 / b.radius, true);
                c2 = to_lines(c2, b.radius, false);
            } else {
                c1.lo = regs[i].shift;
                c2.hi = regs[i].shift;
            }
            int lo = 0;
            cuts.push_back(m);
            for (int hi : cuts) {
                Block c = hi <= k ? c1 : c2;
                c.s = b.s + lo;
                c.e = b.s + hi;
                if (c.e - c.s <= leaf_max) leaves.push_back(c);
                else next.push_back(c);
                lo = hi;
            }
        }
        // order matters only between the phases: row updates, then column
        // updates and factor accumulation (disjoint within a phase)
        CHK(launch_ew(h, put));
        CHK(launch_ew(h, zero));
        CHK(launch_gemm(h, rows));
        CHK(launch_ew(h, back1));
        CHK(launch_gemm(h, cols));
        CHK(launch_gemm(h, facs));
        CHK(launch_ew(h, back2));
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h.stream));
        h.desc_off = 0;
        work.swap(next);
    }
    std::sort(leaves.begin(), leaves.end(), [](const Block& a, const Block& b) { return a.s < b.s; });
    int nb = 0;
    for (const Block& b : leaves) {
        if (bounds) bounds[nb] = block_bound(b, symmetric != 0);
        block_start[nb++] = b.s;
    }
    block_start[nb] = n;
    *nblocks = nb;
    st.nblocks = nb;
    st.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *info = st;
    return SDC_OK;
}

// RSVD split: one symmetric split step of E = [0 A; A^T 0] (order m + n),
// then U = sqrt(2) Q[:m, :k], V = sqrt(2) Q[m:, :k], S11 = Ahat[:k, :k].
int run_split_svd(Handle& h, int m, int n, const double* A, int lda, const sdc_region_t& region,
                  const sdc_opts_t& opts, double* U, int ldu, double* V, int ldv, double* S11, int lds11,
                  sdc_info_t* info, int* status) {
    const int p = m + n, r = std::min(m, n);
    const size_t pp = (size_t)p * p;
    CHK(ensure_ws2(h, 3 * pp * sizeof(double) + 4096));
    CHK(ensure_desc(h, (size_t)(64 << 10)));
    h.desc_off = 0;
    double* E = reinterpret_cast<double*>(h.ws2);
    double* QE = E + pp;
    double* AE = QE + pp;
    {
        std::vector<EwDesc> z(1);
        z[0] = zero_desc(p, p, E, p);
        CHK(launch_ew(h, z));
        std::vector<EwDesc> c(2);
        c[0] = copy_desc(m, n, A, lda, E + (size_t)m * p, p);  // E[:m, m:] = A
        c[1] = copy_desc(n, m, A, lda, E + m, p);              // E[m:, :m] = A^T
        c[1].trans = 1;
        CHK(launch_ew(h, c));
    }
    std::vector<SplitJob> jobs(1);
    SplitJob& j = jobs[0];
    j.n = p; j.pencil = false; j.A = E; j.lda = p; j.region = region; j.opts = opts;
    j.Q = QE; j.ldq = p; j.Ahat = AE; j.ldah = p;
    CHK(run_split_jobs(h, jobs));
    h.desc_off = 0;
    const int k = std::max(0, std::min(j.info.k_lead, r));
    std::vector<EwDesc> out;
    EwDesc cu = copy_desc(m, k, QE, p, U, ldu);
    cu.alpha = std::sqrt(2.0);
    EwDesc cv = copy_desc(n, k, QE + m, p, V, ldv);
    cv.alpha = std::sqrt(2.0);
    if (k > 0) {
        out.push_back(cu);
        out.push_back(cv);
        out.push_back(copy_desc(k, k, AE, p, S11, lds11));
    }
    if (k < r) {
        out.push_back(zero_desc(m, r - k, U + (size_t)k * ldu, ldu));
        out.push_back(zero_desc(n, r - k, V + (size_t)k * ldv, ldv));
        out.push_back(zero_desc(r, r - k, S11 + (size_t)k * lds11, lds11));
        if (k > 0) out.push_back(zero_desc(r - k, k, S11 + k, lds11));
    }
    CHK(launch_ew(h, out));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h.stream));
    h.desc_off = 0;
    *info = j.info;
    *status = j.status;
    return SDC_OK;
}

int run_block_eigvals(Handle& h, int n, const double* T, int ldt, const double* S, int lds, int nblocks,
                      const int* block_start, int symmetric, double* wr, double* wi, double* V, int ldv) {
    if (nblocks < 1 || block_start[0] != 0 || block_start[nblocks] != n) return SDC_ERR_INVALID;
    for (int b = 0; b < nblocks; ++b)
        if (block_start[b + 1] <= block_start[b]) return SDC_ERR_INVALID;
    CHK(ensure_desc(h, sizeof(BlockEigDesc) * (size_t)nblocks + 4096));
    h.desc_off = 0;
    std::vector<BlockEigDesc> v(nblocks);
    for (int b = 0; b < nblocks; ++b) {
        const int s0 = block_start[b];
        BlockEigDesc& d = v[b];
        d.T = T + s0 + (size_t)s0 * ldt;
        d.ldt = ldt;
        d.S = symmetric ? nullptr : S + s0 + (size_t)s0 * lds;
        d.lds = lds;
        d.m = block_start[b + 1] - s0;
        d.symmetric = symmetric;
        d.wr = wr + s0;
        d.wi = wi + s0;
        d.V = V ? V + s0 + (size_t)s0 * ldv : nullptr;
        d.ldv = ldv;
        d.active = 1;
    }
    UPLOAD(dd, v);
    block_eig_batch(dd, v.data(), nblocks, h.stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h.stream));
    h.desc_off = 0;
    return SDC_OK;
}

}  // namespace sdc
