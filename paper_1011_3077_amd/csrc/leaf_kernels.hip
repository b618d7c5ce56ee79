// Eigenvalues of the diagonal blocks that the divide-and-conquer leaves
// (Sec. 3.3-3.5 end the recursion at blocks small enough for a standard dense
// method).  One workgroup per block:
//   * symmetric block of order m <= kJacobiMax: cyclic Jacobi (Jacobi's
//     method for the symmetric eigenproblem, with the round-robin ordering in
//     which the m/2 rotations of a round act on disjoint index pairs and are
//     applied together, rows first, then columns), sweeps of m - 1 rounds
//     until the off-diagonal Frobenius norm is at most 1e-15 of the block's
//     (at most kSweeps sweeps); the eigenvalues are the diagonal, sorted
//     ascending, wi = 0; for a block of order <= kJacobiVecMax the rotations
//     are also accumulated (V <- V J) into the eigenvectors, written in the
//     order of the eigenvalues when the caller asks for them;
//   * pencil block (T, S) of order 1: T/S; of order 2: the roots of
//     det(T - lambda S) = 0, real ones ascending, a complex pair as
//     (re, +im), (re, -im), from the 2 x 2 matrix S'^{-1} T' after a rotation
//     that makes S upper triangular (the shape LAPACK's QZ hands its 2 x 2
//     solver); an infinite eigenvalue (singular S) as +-inf;
//   * any other block: NaN (the recursion can be run to blocks of order <= 2
//     for a pencil; a symmetric block above kJacobiMax is left to the caller).
#include <cmath>

#include "sdc_aux.hpp"

namespace sdc {

namespace {

constexpr int kSweeps = 30;

// Sum over the workgroup (256 threads), the same value in every thread.
__device__ double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ void pencil_small(const BlockEigDesc& d) {
    const double nan = __builtin_nan("");
    if (d.m == 1) {
        d.wr[0] = d.T[0] / d.S[0];
        d.wi[0] = 0.0;
        return;
    }
    if (d.m != 2) {
        for (int i = 0; i < d.m; ++i) d.wr[i] = d.wi[i] = nan;
        return;
    }
    const double t11 = d.T[0], t21 = d.T[1], t12 = d.T[d.ldt], t22 = d.T[d.ldt + 1];
    const double s11 = d.S[0], s21 = d.S[1], s12 = d.S[d.lds], s22 = d.S[d.lds + 1];
    // a rotation from the left makes S upper triangular: (T', S') = G (T, S)
    const double h = hypot(s11, s21);
    const double gc = h > 0.0 ? s11 / h : 1.0, gs = h > 0.0 ? s21 / h : 0.0;
    const double u11 = h, u12 = gc * s12 + gs * s22, u22 = gc * s22 - gs * s12;
    const double v11 = gc * t11 + gs * t21, v12 = gc * t12 + gs * t22;
    const double v21 = gc * t21 - gs * t11, v22 = gc * t22 - gs * t12;
    double r0, r1, i0 = 0.0, i1 = 0.0;
    if (u11 == 0.0 || u22 == 0.0) {
        // singular S: det(T' - l S') = a l^2 + b l + c with a = 0, one
        // infinite eigenvalue and the root of the linear part
        const double b = -(v11 * u22 + v22 * u11 - v12 * 0.0 - v21 * u12);
        const double c = v11 * v22 - v12 * v21;
        r0 = b != 0.0 ? -c / b : nan;
        r1 = (b >= 0.0 ? 1.0 : -1.0) * INFINITY;
        if (u11 == 0.0 && u22 == 0.0) r0 = nan;
    } else {
        // M = S'^{-1} T', whose eigenvalues m22 + p +- sqrt(p^2 + m12 m21),
        // p = (m11 - m22) / 2, are formed without the cancellation of the
        // determinant's coefficients (the larger root first, the other from
        // the product of the two)
        const double m21 = v21 / u22, m22 = v22 / u22;
        const double m11 = (v11 - u12 * m21) / u11, m12 = (v12 - u12 * m22) / u11;
        const double pp = 0.5 * (m11 - m22);
        const double bc = m12 * m21;
        const double disc = pp * pp + bc;
        if (disc >= 0.0) {
            const double z = pp + copysign(sqrt(disc), pp);
            r0 = m22 + z;
            r1 = z != 0.0 ? m22 - bc / z : m22;
            if (r1 < r0) {
                const double t = r0;
                r0 = r1;
                r1 = t;
            }
        } else {
            r0 = r1 = m22 + pp;
            i0 = sqrt(-disc);
            i1 = -i0;
        }
    }
    d.wr[0] = r0; d.wr[1] = r1;
    d.wi[0] = i0; d.wi[1] = i1;
}

__global__ __launch_bounds__(256) void k_block_eig(const BlockEigDesc* __restrict__ descs) {
    constexpr int MX = kJacobiMax, LA = MX + 1;
    __shared__ double s_a[MX * LA];  // row-major, row stride LA
    __shared__ double s_c[MX / 2], s_s[MX / 2];
    __shared__ int s_p[MX / 2], s_q[MX / 2];
    __shared__ double s_red[4];
    const BlockEigDesc d = descs[blockIdx.x];
    if (!d.active || d.m <= 0) return;
    const int m = d.m, tid = threadIdx.x;
    if (!d.symmetric) {
        if (tid == 0) pencil_small(d);
        return;
    }
    if (m > MX) {
        const double nan = __builtin_nan("");
        for (int i = tid; i < m; i += 256) d.wr[i] = d.wi[i] = nan;
        if (d.V)
            for (int e = tid; e < m * m; e += 256) d.V[(e % m) + (size_t)(e / m) * d.ldv] = nan;
        return;
    }
    // the block, symmetrized, padded to even order with an isolated zero row;
    // the eigenvectors (identity at first) use the rows of s_a past MX / 2,
    // which a block of order <= kJacobiVecMax leaves free
    static_assert(2 * kJacobiVecMax <= MX, "eigenvector rows fit after the block's");
    const int mm = m + (m & 1), np = mm / 2;
    const bool vec = d.V != nullptr && m <= kJacobiVecMax;
    double* s_v = s_a + (MX / 2) * LA;  // row-major, row stride LA
    if (vec)
        for (int e = tid; e < mm * mm; e += 256) s_v[(e % mm) * LA + e / mm] = (e % mm) == (e / mm) ? 1.0 : 0.0;
    for (int e = tid; e < mm * mm; e += 256) {
        const int i = e % mm, j = e / mm;
        s_a[i * LA + j] = (i < m && j < m) ? 0.5 * (d.T[i + (size_t)j * d.ldt] + d.T[j + (size_t)i * d.ldt]) : 0.0;
    }
    __syncthreads();
    double f = 0.0;
    for (int e = tid; e < mm * mm; e += 256) {
        const double x = s_a[(e % mm) * LA + e / mm];
        f += x * x;
    }
    const double fro2 = block_sum(f, s_red);
    for (int sweep = 0; sweep < kSweeps; ++sweep) {
        double o = 0.0;
        for (int e = tid; e < mm * mm; e += 256) {
            const int i = e % mm, j = e / mm;
            const double x = i != j ? s_a[i * LA + j] : 0.0;
            o += x * x;
        }
        if (block_sum(o, s_red) <= 1e-30 * fro2) break;
        for (int r = 0; r < mm - 1; ++r) {
            if (tid < np) {
                // round r of the circle method: index mm - 1 stays, the others rotate
                const int p = tid == 0 ? mm - 1 : (r + tid) % (mm - 1);
                const int q = tid == 0 ? r : (r - tid + (mm - 1)) % (mm - 1);
                const double app = s_a[p * LA + p], aqq = s_a[q * LA + q], apq = s_a[p * LA + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    // [c s; -s c]^T [app apq; apq aqq] [c s; -s c] is diagonal
                    const double tau = (aqq - app) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                s_p[tid] = p; s_q[tid] = q; s_c[tid] = c; s_s[tid] = s;
            }
            __syncthreads();
            for (int e = tid; e < np * mm; e += 256) {  // rows p, q of every pair
                const int k = e / mm, j = e % mm;
                const int p = s_p[k], q = s_q[k];
                const double c = s_c[k], s = s_s[k];
                const double x = s_a[p * LA + j], y = s_a[q * LA + j];
                s_a[p * LA + j] = c * x - s * y;
                s_a[q * LA + j] = s * x + c * y;
            }
            __syncthreads();
            for (int e = tid; e < np * mm; e += 256) {  // then columns p, q (of V too)
                const int k = e / mm, i = e % mm;
                const int p = s_p[k], q = s_q[k];
                const double c = s_c[k], s = s_s[k];
                const double x = s_a[i * LA + p], y = s_a[i * LA + q];
                s_a[i * LA + p] = c * x - s * y;
                s_a[i * LA + q] = s * x + c * y;
                if (vec) {
                    const double u = s_v[i * LA + p], w = s_v[i * LA + q];
                    s_v[i * LA + p] = c * u - s * w;
                    s_v[i * LA + q] = s * u + c * w;
                }
            }
            __syncthreads();
        }
    }
    // the diagonal, ranked (ties by index)
    for (int i = tid; i < m; i += 256) {
        const double di = s_a[i * LA + i];
        int rank = 0;
        for (int j = 0; j < m; ++j) {
            const double dj = s_a[j * LA + j];
            rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
        }
        d.wr[rank] = di;
        d.wi[rank] = 0.0;
        if (d.V) {
            const double nan = __builtin_nan("");
            for (int r = 0; r < m; ++r) d.V[r + (size_t)rank * d.ldv] = vec ? s_v[r * LA + i] : nan;
        }
    }
}

}  // namespace

void block_eig_batch(const BlockEigDesc* d, const BlockEigDesc* h, int count, hipStream_t s) {
    (void)h;
    if (count > 0) hipLaunchKernelGGL(k_block_eig, dim3(count), dim3(256), 0, s, d);
}

}  // namespace sdc
