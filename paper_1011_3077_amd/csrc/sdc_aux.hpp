// Descriptors and launchers of the supporting kernels (aux_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sdc {

enum EwOp { EW_PERMUTE = 0, EW_ADD = 1, EW_IDENTITY = 2, EW_SYM = 3, EW_ZERO = 4 };

// Element-wise op on a rows x n output (rows = n for square operands).
struct EwDesc {
    int op, n, rows;
    const void* in; int ldi;
    const void* in2; int ld2;
    void* out; int ldo;
    int trans, revP, revQ;
    const double* sg;  // optional sign source, indexed by the source row
    double alpha;
    int active;
};

struct NormDesc {
    const double* X; int ld, n, rows;
    double* out;
    int active;
};

// Copy n doubles from src to dst + off (collecting small per-problem results
// into one buffer for a single device-to-host copy).
struct GatherDesc {
    const double* src;
    long long off;
    int n;
};

struct SplitDesc {
    const double* Ah; int lda;
    const double* Bh; int ldb;  // null for the symmetric case
    int n;
    double* SA; double* SB;     // n x n suffix-sum scratch
    const double* norms;        // [0] ||A||_1, [1] ||B||_1
    double* e;                  // n
    double* out;                // [0] k*, [1] e(k*)
    int active;
};

struct GaussDesc {
    double* G; int ld, n;
    uint64_t seed;
    int tag;
    int active;
};

// Gershgorin bounds of a symmetric n x n matrix: out[2j] = A_jj - r_j,
// out[2j+1] = A_jj + r_j with r_j = sum_{i != j} |A_ij| (column sums).
struct GershDesc {
    const double* X; int ld, n;
    double* out;
    int active;
};
void gersh_batch(const GershDesc* d, const GershDesc* h, int count, hipStream_t s);

// Eigenvalues of one diagonal block of a block upper-triangular pair
// (leaf_kernels.hip): a symmetric block of order <= kJacobiMax by cyclic
// Jacobi, a pencil block (T, S) of order 1 or 2 in closed form and of order
// <= kPencilMax by the double-shift QR algorithm on S^{-1} T (or on T^{-1} S
// when S is the worse conditioned of the two), NaN for any other block.  T
// and S point at the block's first element (column-major).
constexpr int kJacobiMax = 128;
constexpr int kJacobiVecMax = 64;  // blocks whose eigenvectors are accumulated too
constexpr int kPencilMax = 64;
struct BlockEigDesc {
    const double* T; int ldt;
    const double* S; int lds;   // pencil only
    int m, symmetric;
    double* wr; double* wi;     // m values each
    double* V; int ldv;         // optional: the block's eigenvectors (m x m, columns in the order of wr)
    int active;
};
void block_eig_batch(const BlockEigDesc* d, const BlockEigDesc* h, int count, hipStream_t s);

// Conjugate gradients on X A11 - A22 X = E (refine_kernels.hip).  X, R, P, Z
// are m x k, contiguous (ld m); E has leading dimension lde.  rr is a ring of
// 3 x kCgMaxBlocks partial sums (slot it % 3 holds rr_it), rr0 and pz hold
// kCgMaxBlocks partials each; nblk = cg_blocks(m, k).
constexpr int kCgMaxBlocks = 256;
struct CgDesc {
    int m, k;
    const double* E; int lde;
    double *X, *R, *P, *Z;
    double *rr, *rr0, *pz;
    double tol2;
    int nblk;
    int active;
};
int cg_blocks(int m, int k);
void cg_init_batch(const CgDesc* d, const CgDesc* h, int count, hipStream_t s);
// phase 0: <P, Z>; 1: X, R update; 2: new direction.
void cg_iter_vec(const CgDesc* d, const CgDesc* h, int count, int it, int phase, hipStream_t s);

template <typename Tin, typename Tout>
void ew_batch(const EwDesc* d, const EwDesc* h, int count, hipStream_t s);
template <typename T>
void fill(T* p, size_t n, T v, hipStream_t s);
// Zeroing of many small arrays (counters, norm accumulators) in one launch.
struct ZeroDesc {
    unsigned* p;
    unsigned words;  // 4-byte words
};
void zero_batch(const ZeroDesc* d, int count, hipStream_t s);
void norm1_batch(const NormDesc* d, const NormDesc* h, int count, hipStream_t s);
void split_search_batch(const SplitDesc* d, const SplitDesc* h, int count, hipStream_t s);
void orth_err_batch(const NormDesc* d, const NormDesc* h, int count, hipStream_t s);
void gauss_batch(const GaussDesc* d, const GaussDesc* h, int count, hipStream_t s);

void gather_batch(const GatherDesc* d, int count, double* dst, hipStream_t s);

// Eigenvectors of an upper-triangular matrix or pencil (TREVC, Alg. 8).
struct TrevcArgs {
    const double* T; int ldt;
    const double* S; int lds;   // nullptr: S = I
    double* X; int ldx;
    int n;
};
void trevc_launch(const TrevcArgs& a, hipStream_t s);

}  // namespace sdc
