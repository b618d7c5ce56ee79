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
template <typename T> struct QrCfg;
// Panel workgroups have PT threads = (PT/32) row groups x 32 columns; RPG is
// the register rows per thread for a full MT_MAX-row node.
template <> struct QrCfg<double> {
    static constexpr int NB = 32, MT_MAX = 512, H = 256, F = 16, PT = 512, RPG = MT_MAX / (PT / 32);
};
template <> struct QrCfg<float> {
    static constexpr int NB = 32, MT_MAX = 1024, H = 512, F = 32, PT = 512, RPG = MT_MAX / (PT / 32);
};

constexpr int kMaxLevels = 4;
constexpr int kMaxLeaves = 128;   // per panel and problem
constexpr int kMaxInternal = 16;  // internal tree nodes per panel and problem

struct TreeGeom {
    int L[kMaxLevels];   // nodes per level, L[0] leaves
    int levels;
    int pow[kMaxLevels]; // F^level
};

template <typename T>
__host__ __device__ inline TreeGeom tree_geom(int mp) {
    using C = QrCfg<T>;
    TreeGeom g;
    g.levels = 1;
    g.pow[0] = 1;
    for (int i = 0; i < kMaxLevels; ++i) g.L[i] = 0;
    if (mp <= C::MT_MAX) {
        g.L[0] = 1;
    } else {
        g.L[0] = (mp + C::H - 1) / C::H;
        while (g.L[g.levels - 1] > 1 && g.levels < kMaxLevels) {
            g.L[g.levels] = (g.L[g.levels - 1] + C::F - 1) / C::F;
            g.pow[g.levels] = g.pow[g.levels - 1] * C::F;
            ++g.levels;
        }
    }
    for (int i = g.levels; i < kMaxLevels; ++i) g.pow[i] = g.pow[i - 1] * C::F;
    return g;
}

// First row (relative to the panel's top row) of leaf j among L0 balanced leaves.
__host__ __device__ inline int leaf_lo(int j, int mp, int L0) {
    return (int)(((long long)j * mp) / L0);
}

// Index of an internal node (level >= 1) in per-problem arrays.
__host__ __device__ inline int internal_index(const TreeGeom& g, int level, int node) {
    int off = 0;
    for (int l = 1; l < level; ++l) off += g.L[l];
    return off + node;
}
// Index of any node in the per-problem T-factor array.
__host__ __device__ inline int node_index(const TreeGeom& g, int level, int node) {
    return level == 0 ? node : kMaxLeaves + internal_index(g, level, node);
}

// Per-problem descriptor of an augmented QR: factor columns [0, nf) of the
// m x ncols matrix W (column-major, leading dimension ld) and apply Q^T to all
// ncols columns.  Side buffers live in aux.
template <typename T> struct QrDesc {
    T* W;
    int ld, m, nf, ncols;
    T* Tm;            // (kMaxLeaves + kMaxInternal) * NB * NB, T factors of one panel's nodes
    T* Vint;          // kMaxInternal * MT_MAX * NB, internal-node reflectors (column-major, ld MT_MAX)
    T* diag;          // nf: diagonal of R as produced (before sign normalization)
    unsigned* counters; // kMaxInternal tree arrival counters (must start at zero)
    int active;
};

template <typename T> size_t qr_aux_elems() {
    using C = QrCfg<T>;
    return (size_t)(kMaxLeaves + kMaxInternal) * C::NB * C::NB + (size_t)kMaxInternal * C::MT_MAX * C::NB;
}

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
    T* W;              // 2n x 3n, ld = 2n: [B_j A_j 0; -A_j 0 B_j]
    int n;
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
    int n;
    const double* A; int lda;
    const double* B; int ldb;
    double a1, a2, b1, b2;
    int trans;
};

// Host-side launchers (defined in the .hip files).
template <typename T>
void qr_aug_batch(const QrDesc<T>* d_descs, const QrDesc<T>* h_descs, int count, hipStream_t s);
template <typename T>
void gemm_batch(const GemmDesc<T>* d_descs, const GemmDesc<T>* h_descs, int count, hipStream_t s);
template <typename T>
void irs_init_batch(const IrsInit<T>* d, const IrsInit<T>* h, int count, hipStream_t s);
template <typename T>
void irs_post_batch(const IrsDesc<T>* d, const IrsDesc<T>* h, int count, int first, hipStream_t s);

}  // namespace sdc
