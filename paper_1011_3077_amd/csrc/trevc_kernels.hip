// Eigenvectors of an upper-triangular matrix or pencil (TREVC, Sec. 5),
// blocked as Alg. 8.
//
// For upper-triangular T (and S) the j-th eigenvalue is lambda_j = T_jj / S_jj
// (S = I if absent) and its eigenvector x_j, with x_j[j] = 1 and zeros below,
// solves (T - lambda_j S) x_j = 0:
//   x_i = -(sum_{k=i+1}^{j} (T_ik - lambda_j S_ik) x_k) / (T_ii - lambda_j S_ii).
// Alg. 8 computes X = [x_0 ... x_{n-1}] by b x b blocks: for block column J
// the diagonal block X[J,J] first, then block rows I = J-1 .. 0, each from
// the product sum over K = I+1 .. J of T[I,K] X[K,J] (and S[I,K] X[K,J])
// followed by a small triangular solve with T[I,I] (and S[I,I]).
//
// Block columns are independent, so one workgroup takes one block column
// (b = 32) and sweeps its block rows upward: the product sums run on the
// FP64 matrix cores (each of the four waves one 16 x 16 quarter of the
// 32 x 32 block, k in steps of 4), the solves run one column per thread from
// LDS.  X is written as it is computed and re-read (L2) by the later
// products of the same workgroup.
#include <cfloat>

#include "mfma.hpp"
#include "sdc_aux.hpp"

namespace sdc {

namespace {

constexpr int kTb = 32;       // block size b of Alg. 8
constexpr int kTls = kTb + 1;  // LDS column stride (conflict-free)

// LAPACK-style guard of the division: a denominator below
// eps (|T_ii| + |lambda S_ii|) + the smallest normal number is replaced by
// that bound with its sign.
__device__ __forceinline__ double guard_den(double den, double t, double ls) {
    const double smin = DBL_EPSILON * (fabs(t) + fabs(ls)) + DBL_MIN;
    return fabs(den) < smin ? (den >= 0.0 ? smin : -smin) : den;
}

__global__ __launch_bounds__(256) void k_trevc(TrevcArgs a) {
    using M = Mfma<double>;
    typedef M::v4 v4;
    __shared__ double sT[kTb * kTls], sS[kTb * kTls];  // diagonal block of T (S), column-major
    __shared__ double sG[kTb * kTls], sH[kTb * kTls];  // product sums of T (S); then the solution
    __shared__ double sLam[kTb];
    const int n = a.n;
    const int J = blockIdx.x;
    const int c0 = J * kTb;
    if (c0 >= n) return;
    const int bw = min(kTb, n - c0);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool pencil = a.S != nullptr;
    const double* T = a.T;
    const double* S = a.S;
    double* X = a.X;
    const size_t ldt = (size_t)a.ldt, lds = (size_t)a.lds, ldx = (size_t)a.ldx;

    if (tid < bw) {
        const double t = T[(size_t)(c0 + tid) * ldt + c0 + tid];
        sLam[tid] = pencil ? t / S[(size_t)(c0 + tid) * lds + c0 + tid] : t;
    }
    // below the diagonal block: zero
    for (int jj = 0; jj < bw; ++jj)
        for (int r = c0 + kTb + tid; r < n; r += 256) X[(size_t)(c0 + jj) * ldx + r] = 0.0;

    // diagonal block: its upper triangle into LDS
    for (int e = tid; e < kTb * kTb; e += 256) {
        const int r = e % kTb, k = e / kTb;
        const bool in = r < bw && k < bw && r <= k;
        sT[k * kTls + r] = in ? T[(size_t)(c0 + k) * ldt + c0 + r] : 0.0;
        sS[k * kTls + r] = in && pencil ? S[(size_t)(c0 + k) * lds + c0 + r] : (in && r == k ? 1.0 : 0.0);
    }
    __syncthreads();
    if (tid < bw) {
        const int jj = tid;
        const double lam = sLam[jj];
        double* x = sG + jj * kTls;
        for (int r = jj + 1; r < kTb; ++r) x[r] = 0.0;
        x[jj] = 1.0;
        for (int r = jj - 1; r >= 0; --r) {
            double acc = 0.0;
            for (int k = r + 1; k <= jj; ++k) acc = fma(sT[k * kTls + r] - lam * sS[k * kTls + r], x[k], acc);
            const double tr = sT[r * kTls + r], ls = lam * sS[r * kTls + r];
            x[r] = -acc / guard_den(tr - ls, tr, ls);
        }
        for (int r = 0; r < bw; ++r) X[(size_t)(c0 + jj) * ldx + c0 + r] = x[r];
    }
    __syncthreads();

    // block rows I = J-1 .. 0
    const int tr = wave >> 1, tc = wave & 1;
    const int gq = lane >> 4, ln = lane & 15;
    const int kend = c0 + bw;
    for (int I = J - 1; I >= 0; --I) {
        const int r0 = I * kTb;
        // G = sum_{k = r0 + b}^{kend - 1} T[r0 + r, k] X[k, c0 + jj] (and S's)
        v4 gt = v4{0, 0, 0, 0}, gs = v4{0, 0, 0, 0};
        const int row = r0 + 16 * tr + ln;           // A operand: T[row, k0 + gq]
        const int col = c0 + 16 * tc + ln;           // B operand: X[k0 + gq, col]
        const bool colok = col < kend;
        for (int k0 = r0 + kTb; k0 < kend; k0 += 4) {
            const int k = k0 + gq;
            const bool kok = k < kend;
            const double ta = kok ? T[(size_t)k * ldt + row] : 0.0;
            const double xb = (kok && colok) ? X[(size_t)col * ldx + k] : 0.0;
            gt = M::mma(ta, xb, gt);
            if (pencil) {
                const double sa = kok ? S[(size_t)k * lds + row] : 0.0;
                gs = M::mma(sa, xb, gs);
            }
        }
        // D layout: lane (gq, ln) holds D[gq + 4 v][ln]
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = 16 * tr + M::row(gq, v), cc = 16 * tc + ln;
            sG[cc * kTls + rr] = gt[v];
            sH[cc * kTls + rr] = pencil ? gs[v] : 0.0;
        }
        // diagonal block of T (S) of block row I
        for (int e = tid; e < kTb * kTb; e += 256) {
            const int r = e % kTb, k = e / kTb;
            const bool in = r <= k;
            sT[k * kTls + r] = in ? T[(size_t)(r0 + k) * ldt + r0 + r] : 0.0;
            sS[k * kTls + r] = in && pencil ? S[(size_t)(r0 + k) * lds + r0 + r] : (r == k ? 1.0 : 0.0);
        }
        __syncthreads();
        if (tid < bw) {
            const int jj = tid;
            const double lam = sLam[jj];
            double* x = sG + jj * kTls;
            const double* h = sH + jj * kTls;
            for (int r = kTb - 1; r >= 0; --r) {
                double acc = x[r] - lam * h[r];
                for (int k = r + 1; k < kTb; ++k) acc = fma(sT[k * kTls + r] - lam * sS[k * kTls + r], x[k], acc);
                const double trr = sT[r * kTls + r], ls = lam * sS[r * kTls + r];
                x[r] = -acc / guard_den(trr - ls, trr, ls);
            }
            for (int r = 0; r < kTb; ++r) X[(size_t)(c0 + jj) * ldx + r0 + r] = x[r];
        }
        __syncthreads();
    }
}

}  // namespace

void trevc_launch(const TrevcArgs& a, hipStream_t s) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_trevc, dim3((a.n + kTb - 1) / kTb), dim3(256), 0, s, a);
}

}  // namespace sdc
