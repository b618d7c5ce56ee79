// Internal declarations shared by the HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace sdc {

// ---------------------------------------------------------------------------
// Blocked Householder QR geometry (per precision).
//
// The QR of a tall m x nf panel block is computed as a reduction tree of
// Householder QRs (the TSQR panel of the communication-avoiding QR the paper
// costs its algorithms with, Sec. 4.2): leaves of about H rows are factored
// by one workgroup each, then F leaf R factors at a time are stacked and
// factored again, up to a single root.  A panel whose height fits one node
// (<= MT_MAX rows) is a single leaf.  Every node is at most MT_MAX rows by NB
// columns and lives in one workgroup's registers.
// ---------------------------------------------------------------------------
template <typename T, int NBW> struct QrCfg {
    // Panels are NBW = 32 or 64 columns wide.  The wider panel doubles the
    // arithmetic intensity of the trailing update (flops per byte of the
    // trailing matrix moved), at the price of a longer panel factorization
    // per column and a shallower fan-in (F * NB <= MT_MAX).
    static_assert(NBW == 32 || NBW == 64, "panel widths 32 and 64");
    static constexpr int NB = NBW, MT_MAX = 256, H = 256, F = 256 / NBW, PT = 256;
};
// Panel workgroups have PT = 256 threads (four wavefronts, one per SIMD of a
// CU); a node (at most MT_MAX rows, NB columns) is factored in registers
// with each wavefront owning NB/4 columns and each lane up to MT_MAX/64 rows.
// Every node (F * NB <= MT_MAX rows) fits the trailing-update kernels'
// registers (256 rows x 16 columns per wave).

constexpr int kMaxLevels = 5;
// Tree arrival counters per problem (kMaxInternal of them, zero between
// uses: each is reset by its last arrival): the panel factorization counts
// arrivals at internal nodes in the first kPanelCounters, the row-split
// update (k_la, NB/16 column groups of 16) after them, one per (column
// group, internal node) of the panel's tree.
constexpr int kMaxInternal = 320;
constexpr int kPanelCounters = 64;
constexpr int kMaxPanelRows = 2 * 16384;  // augmented matrices of order <= 16384

// Tree shape of a panel with mp rows: L0 leaves, levels levels, and
// L(l) = ceil(L0 / F^l) nodes at level l.  Computed arithmetically (no
// arrays indexed at run time, so kernels keep it in registers).
template <typename T, int NBW> struct TreeGeomT {
    int L0, levels;
    __host__ __device__ int pw(int l) const {
        int p = 1;
        for (int i = 0; i < l; ++i) p *= QrCfg<T, NBW>::F;
        return p;
    }
    __host__ __device__ int L(int l) const {
        if (l >= levels) return 0;
        const int p = pw(l);
        return (L0 + p - 1) / p;
    }
};

template <typename T, int NBW>
__host__ __device__ inline TreeGeomT<T, NBW> tree_geom(int mp) {
    using C = QrCfg<T, NBW>;
    TreeGeomT<T, NBW> g;
    static_assert(C::H % 16 == 0, "leaves are whole 16-row blocks");
    g.L0 = mp <= C::MT_MAX ? 1 : ((mp + 15) / 16 + C::H / 16 - 1) / (C::H / 16);
    g.levels = 1;
    for (int n = g.L0; n > 1 && g.levels < kMaxLevels; n = (n + C::F - 1) / C::F) ++g.levels;
    return g;
}

// First row (relative to the panel's top row) of leaf j among L0 balanced
// leaves.  Leaves are whole runs of 16-row blocks (the last one is cut at
// mp): the panel's top row is a multiple of NB, so (with a leading dimension
// that is a multiple of 16 elements) every 16-row block of a leaf is whole
// cache lines and no line is shared by two leaves' workgroups.  With
// L0 = ceil(ceil(mp/16) / (H/16)) (tree_geom) every leaf has <= H rows.
__host__ __device__ inline int leaf_lo(int j, int mp, int L0) {
    if (j >= L0) return mp;
    const long long blocks = (mp + 15) / 16;
    return (int)((j * blocks) / L0) * 16;
}

// Internal nodes and levels of the tallest supported panel (checked
// against the counters and kMaxLevels).
template <typename T, int NBW> constexpr int max_internal_nodes() {
    using C = QrCfg<T, NBW>;
    int n = ((kMaxPanelRows + 15) / 16 + C::H / 16 - 1) / (C::H / 16), total = 0;
    while (n > 1) {
        n = (n + C::F - 1) / C::F;
        total += n;
    }
    return total;
}
template <typename T, int NBW> constexpr int max_levels() {
    using C = QrCfg<T, NBW>;
    int n = ((kMaxPanelRows + 15) / 16 + C::H / 16 - 1) / (C::H / 16), lv = 1;
    while (n > 1) {
        n = (n + C::F - 1) / C::F;
        ++lv;
    }
    return lv;
}
template <typename T, int NBW> constexpr bool counters_fit() {
    return max_internal_nodes<T, NBW>() <= kPanelCounters &&
           kPanelCounters + (NBW / 16) * max_internal_nodes<T, NBW>() <= kMaxInternal &&
           max_levels<T, NBW>() <= kMaxLevels;
}
static_assert(counters_fit<double, 32>() && counters_fit<float, 32>() && counters_fit<double, 64>() &&
                  counters_fit<float, 64>(),
              "tree counters and levels of the tallest panel");

// Index of an internal node (level >= 1) in per-problem arrays.
template <typename T, int NBW>
__host__ __device__ inline int internal_index(const TreeGeomT<T, NBW>& g, int level, int node) {
    int off = 0;
    for (int l = 1; l < level; ++l) off += g.L(l);
    return off + node;
}
// Which kernel updates which trailing columns after the panel at column c0
// of a QR with nf factored columns: columns [c0 + nbk, c0 + nbk + la) go to
// the row-split kernel (k_la), the rest to the wide kernel (k_update).  With
// nf >= la_min (the handle's look-ahead threshold, sdc_lookahead_set) the
// row-split kernel takes the next panel's columns (look-ahead: they are done
// first, so that the next panel can be factored on a second stream beside
// the bulk update).  By default no problem takes it: with the panel's tree
// above its leaves factored beside the leaf-level update on one stream, the
// one-stream schedule measured faster at every order up to 8192.  The choice
// depends on the problem's own shape and the handle only, so a problem
// rounds the same alone and in any batch of the handle.
constexpr int kLookaheadNever = 1 << 30;
__host__ __device__ inline int row_split_cols(int nb, int nf, int c0, int la_min) {
    const int cb = c0 + (nf - c0 < nb ? nf - c0 : nb);
    if (nf < la_min || cb >= nf) return 0;
    return nf - cb < nb ? nf - cb : nb;
}

// Index of any node in the per-problem T-factor array (leaves first).
template <typename T, int NBW>
__host__ __device__ inline int node_index(const TreeGeomT<T, NBW>& g, int level, int node, int tm_leaves) {
    return level == 0 ? node : tm_leaves + internal_index(g, level, node);
}

// Per-problem descriptor of an augmented QR: factor columns [0, nf) of the
// m x ncols matrix W (column-major, leading dimension ld) and apply Q^T to all
// ncols columns.  The T factors and internal reflectors of a panel live in
// one of two buffers, by panel parity, so that a panel can be factored while
// the previous panel's update is still reading its own.
template <typename T> struct QrDesc {
    T* W;
    int ld, m, nf, ncols;
    T* Tm[2];         // (tm_leaves + internal) * NB * NB: T factors of one panel's nodes
    T* Vint[2];       // internal * MT_MAX * NB: internal-node reflectors (column-major, ld MT_MAX)
    int tm_leaves;    // leaves of the tallest panel (panel 0)
    T* diag;          // nf: diagonal of R as produced (before sign normalization)
    unsigned* counters; // kMaxInternal tree arrival counters (must start at zero)
    int active;
    int nb;           // panel width (32 or 64); every problem of one batched call has the same
    int la_min;       // look-ahead from this many factored columns (row_split_cols)
};

// Elements of one parity's side buffers for an m-row problem and panel
// width NBW, and the most either panel width needs.
template <typename T, int NBW> size_t qr_aux_elems_nb(int m) {
    using C = QrCfg<T, NBW>;
    const auto g = tree_geom<T, NBW>(m);
    size_t internal = 0;
    for (int l = 1; l < g.levels; ++l) internal += (size_t)g.L(l);
    return ((size_t)g.L(0) + internal) * C::NB * C::NB + internal * C::MT_MAX * C::NB;
}
template <typename T> size_t qr_aux_elems(int m) {
    const size_t a = qr_aux_elems_nb<T, 32>(m), b = qr_aux_elems_nb<T, 64>(m);
    return a > b ? a : b;
}

// Streams and events for the look-ahead schedule of the QR (panel k+1
// factored while the rest of panel k's update runs).  crit carries the
// panels and the look-ahead updates, rest the bulk updates.
struct QrStreams {
    hipStream_t crit, rest;
    hipEvent_t evP, evR, evE, evD;
};

// Batched GEMM descriptor: C = alpha op(A) op(B) + beta C, op(X) = X or X^T.
template <typename T> struct GemmDesc {
    const T* A;
    const T* B;
    T* C;
    int lda, ldb, ldc;
    int M, N, K;
    int ta, tb;
    T alpha, beta;
    int active;
};

// Per-problem state of a batched IRS.
template <typename T> struct IrsDesc {
    T* W;              // 2n x 3n, leading dimension ld: [B_j A_j 0; -A_j 0 B_j]
    int n, ld;
    double* Rprev;     // n x n, ld n: previous R (sign-normalized)
    const T* diag;     // R diagonal from the QR (length n)
    double* norms;     // [2]: max column sum of |R_j - R_{j-1}| and of |R_{j-1}|
    int active;
};

// Initialization of an IRS side from the FP64 inputs: A0 = a1 A + a2 B,
// B0 = b1 A + b2 B (the region map), transposed if trans.  B == nullptr
// means the identity.
template <typename T> struct IrsInit {
    T* W;
    int n, ld;
    const double* A; int lda;
    const double* B; int ldb;
    double a1, a2, b1, b2;
    int trans;
};

// Host-side launchers (defined in the .hip files).
// tree_overlap: for panels without a row-split part, factor the tree above
// the leaves in the same launch as the leaf-level trailing update
// (k_update with CLIMB) instead of before it (32-column panels).
template <typename T>
void qr_aug_batch(const QrDesc<T>* d_descs, const QrDesc<T>* h_descs, int count, hipStream_t s,
                  const QrStreams* la = nullptr, bool tree_overlap = true);
template <typename T>
void gemm_batch(const GemmDesc<T>* d_descs, const GemmDesc<T>* h_descs, int count, hipStream_t s);
template <typename T>
void irs_init_batch(const IrsInit<T>* d, const IrsInit<T>* h, int count, hipStream_t s);
template <typename T>
void irs_post_batch(const IrsDesc<T>* d, const IrsDesc<T>* h, int count, int first, hipStream_t s);

}  // namespace sdc
