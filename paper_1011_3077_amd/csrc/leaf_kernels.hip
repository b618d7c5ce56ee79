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
//   * pencil block of order 3 .. kPencilMax: the eigenvalues of
//     M = S^{-1} T (Gaussian elimination with partial pivoting on S, applied
//     to T, then back substitution), or of N = T^{-1} S, inverted, when S is
//     the worse conditioned of the two (an infinite eigenvalue of the pencil
//     is a zero one of N); M is reduced to Hessenberg form by Householder
//     reflections and its eigenvalues found by the implicit double-shift QR
//     algorithm (Francis steps on the active window, deflation at a negligible
//     subdiagonal entry, 1 x 1 and 2 x 2 blocks read off, exceptional shifts
//     after 10 and 20 steps without deflation, at most 30 steps per
//     eigenvalue); real eigenvalues ascending, then complex pairs by real part
//     as (re, +im), (re, -im), as for order 2;
//   * any other block: NaN (a symmetric block above kJacobiMax, a pencil
//     block above kPencilMax: the recursion can be run to smaller blocks).
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

// Eigenvalues of the m x m pencil block (3 <= m <= kPencilMax) by the
// whole workgroup; sh holds 2 kPencilMax (kPencilMax + 1) + 3 kPencilMax + 8
// doubles of LDS.  Every scalar decision (pivot, reflector, deflation point)
// is taken by every thread from the same LDS values, so control flow around
// the barriers is uniform.
__device__ void pencil_dense(const BlockEigDesc& d, double* sh, int* ish) {
    constexpr int MX = kPencilMax, LA = MX + 1;
    const int m = d.m, tid = threadIdx.x;
    const double nan = __builtin_nan("");
    const double eps = 2.220446049250313e-16;
    double* sa = sh;             // the matrix being reduced (row-major, stride LA)
    double* sb = sh + MX * LA;   // the one being factored
    double* sv = sb + MX * LA;   // a reflector or the multipliers (MX)
    double* swr = sv + MX;       // eigenvalues found (MX each)
    double* swi = swr + MX;
    double* ssc = swi + MX;      // scalars (8)
    // 1. M = S^{-1} T, or N = T^{-1} S when S is the worse conditioned:
    //    elimination with partial pivoting on the divisor, applied to the
    //    other matrix, then back substitution.  The pivot ratio
    //    min |u_kk| / max |u_kk| serves as the condition estimate.
    int swapped = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool sw = attempt == 1;
        const double* A = sw ? d.S : d.T;   // to be solved for
        const int lda = sw ? d.lds : d.ldt;
        const double* B = sw ? d.T : d.S;   // the divisor
        const int ldb = sw ? d.ldt : d.lds;
        for (int e = tid; e < m * m; e += blockDim.x) {
            const int i = e % m, j = e / m;
            sa[i * LA + j] = A[i + (size_t)j * lda];
            sb[i * LA + j] = B[i + (size_t)j * ldb];
        }
        __syncthreads();
        double umin = INFINITY, umax = 0.0;
        for (int k = 0; k < m; ++k) {
            if (tid == 0) {  // pivot row
                int p = k;
                double best = fabs(sb[k * LA + k]);
                for (int i = k + 1; i < m; ++i) {
                    const double v = fabs(sb[i * LA + k]);
                    if (v > best) {
                        best = v;
                        p = i;
                    }
                }
                ish[0] = p;
            }
            __syncthreads();
            const int p = ish[0];
            if (p != k)
                for (int j = tid; j < m; j += blockDim.x) {
                    double t = sb[k * LA + j];
                    sb[k * LA + j] = sb[p * LA + j];
                    sb[p * LA + j] = t;
                    t = sa[k * LA + j];
                    sa[k * LA + j] = sa[p * LA + j];
                    sa[p * LA + j] = t;
                }
            __syncthreads();
            const double piv = sb[k * LA + k];
            umin = fmin(umin, fabs(piv));
            umax = fmax(umax, fabs(piv));
            for (int i = k + 1 + tid; i < m; i += blockDim.x) sv[i] = piv != 0.0 ? sb[i * LA + k] / piv : 0.0;
            __syncthreads();
            const int rows = m - k - 1;
            for (int e = tid; e < rows * m; e += blockDim.x) {
                const int i = k + 1 + e / m, j = e % m;
                const double l = sv[i];
                if (j > k) sb[i * LA + j] -= l * sb[k * LA + j];
                sa[i * LA + j] -= l * sa[k * LA + j];
            }
            __syncthreads();
        }
        // keep this form if its divisor is the better conditioned one; the
        // second attempt (N) is kept if the first (M) was worse
        const double rc = umax > 0.0 ? umin / umax : 0.0;
        if (attempt == 0) {
            if (tid == 0) ssc[0] = rc;
            __syncthreads();
            if (rc >= 1e-6) break;  // S well enough conditioned: M
        } else {
            const double rc0 = ssc[0];
            if (rc <= rc0) {  // T is no better: back to M
                for (int e = tid; e < m * m; e += blockDim.x) {
                    const int i = e % m, j = e / m;
                    sa[i * LA + j] = d.T[i + (size_t)j * d.ldt];
                    sb[i * LA + j] = d.S[i + (size_t)j * d.lds];
                }
                __syncthreads();
                // redo the elimination of S (same steps as above)
                for (int k = 0; k < m; ++k) {
                    if (tid == 0) {
                        int p = k;
                        double best = fabs(sb[k * LA + k]);
                        for (int i = k + 1; i < m; ++i) {
                            const double v = fabs(sb[i * LA + k]);
                            if (v > best) {
                                best = v;
                                p = i;
                            }
                        }
                        ish[0] = p;
                    }
                    __syncthreads();
                    const int p = ish[0];
                    if (p != k)
                        for (int j = tid; j < m; j += blockDim.x) {
                            double t = sb[k * LA + j];
                            sb[k * LA + j] = sb[p * LA + j];
                            sb[p * LA + j] = t;
                            t = sa[k * LA + j];
                            sa[k * LA + j] = sa[p * LA + j];
                            sa[p * LA + j] = t;
                        }
                    __syncthreads();
                    const double piv = sb[k * LA + k];
                    for (int i = k + 1 + tid; i < m; i += blockDim.x) sv[i] = piv != 0.0 ? sb[i * LA + k] / piv : 0.0;
                    __syncthreads();
                    const int rows = m - k - 1;
                    for (int e = tid; e < rows * m; e += blockDim.x) {
                        const int i = k + 1 + e / m, j = e % m;
                        const double l = sv[i];
                        if (j > k) sb[i * LA + j] -= l * sb[k * LA + j];
                        sa[i * LA + j] -= l * sa[k * LA + j];
                    }
                    __syncthreads();
                }
            } else {
                swapped = 1;
            }
        }
    }
    // a zero pivot left: the pencil is singular (or the block's divisor is): NaN
    if (tid == 0) {
        double mn = INFINITY;
        for (int k = 0; k < m; ++k) mn = fmin(mn, fabs(sb[k * LA + k]));
        ish[1] = mn > 0.0 ? 1 : 0;
    }
    __syncthreads();
    if (!ish[1]) {
        for (int i = tid; i < m; i += blockDim.x) d.wr[i] = d.wi[i] = nan;
        return;
    }
    // back substitution, one column per thread: sa <- U^{-1} sa
    for (int c = tid; c < m; c += blockDim.x)
        for (int i = m - 1; i >= 0; --i) {
            double acc = sa[i * LA + c];
            for (int k = i + 1; k < m; ++k) acc -= sb[i * LA + k] * sa[k * LA + c];
            sa[i * LA + c] = acc / sb[i * LA + i];
        }
    __syncthreads();
    // 2. Householder reduction of sa to upper Hessenberg form
    for (int k = 0; k + 2 < m; ++k) {
        if (tid == 0) {
            double sg = 0.0;
            for (int i = k + 2; i < m; ++i) sg += sa[i * LA + k] * sa[i * LA + k];
            const double x0 = sa[(k + 1) * LA + k];
            double beta = 0.0, tau = 0.0, v0 = 1.0;
            if (sg > 0.0) {
                const double mu = sqrt(x0 * x0 + sg);
                beta = x0 <= 0.0 ? mu : -mu;
                v0 = x0 - beta;
                tau = (beta - x0) / beta;
            } else {
                beta = x0;
            }
            for (int i = k + 2; i < m; ++i) sv[i] = sg > 0.0 ? sa[i * LA + k] / v0 : 0.0;
            sv[k + 1] = 1.0;
            ssc[1] = tau;
            ssc[2] = beta;
        }
        __syncthreads();
        const double tau = ssc[1];
        if (tau != 0.0) {
            // from the left on rows k+1 .. m-1, columns k .. m-1
            for (int j = k + tid; j < m; j += blockDim.x) {
                double w = 0.0;
                for (int i = k + 1; i < m; ++i) w += sv[i] * sa[i * LA + j];
                w *= tau;
                for (int i = k + 1; i < m; ++i) sa[i * LA + j] -= w * sv[i];
            }
            __syncthreads();
            // from the right on columns k+1 .. m-1, every row
            for (int i = tid; i < m; i += blockDim.x) {
                double w = 0.0;
                for (int c = k + 1; c < m; ++c) w += sa[i * LA + c] * sv[c];
                w *= tau;
                for (int c = k + 1; c < m; ++c) sa[i * LA + c] -= w * sv[c];
            }
            __syncthreads();
        }
        if (tid == 0) {
            sa[(k + 1) * LA + k] = ssc[2];
            for (int i = k + 2; i < m; ++i) sa[i * LA + k] = 0.0;
        }
        __syncthreads();
    }
    // 3. implicit double-shift QR on the active window [l, hi]
    int hi = m - 1, its = 0, total = 0, found = 0;
    double hnorm = 0.0;  // a scale for the deflation test of zero diagonals
    for (int e = 0; e < m * m; ++e) hnorm = fmax(hnorm, fabs(sa[(e / m) * LA + e % m]));
    while (hi >= 0) {
        if (hi == 0) {
            if (tid == 0) {
                swr[found] = sa[0];
                swi[found] = 0.0;
            }
            ++found;
            break;
        }
        int l = hi;
        for (; l > 0; --l) {
            double sc = fabs(sa[(l - 1) * LA + l - 1]) + fabs(sa[l * LA + l]);
            if (sc == 0.0) sc = hnorm;
            if (fabs(sa[l * LA + l - 1]) <= eps * sc) break;
        }
        if (l == hi) {  // a 1 x 1 block
            if (tid == 0) {
                swr[found] = sa[hi * LA + hi];
                swi[found] = 0.0;
                sa[hi * LA + hi - 1] = 0.0;
            }
            ++found;
            --hi;
            its = 0;
            __syncthreads();
            continue;
        }
        if (l == hi - 1) {  // a 2 x 2 block
            const double a = sa[(hi - 1) * LA + hi - 1], b = sa[(hi - 1) * LA + hi];
            const double c = sa[hi * LA + hi - 1], dd = sa[hi * LA + hi];
            const double pp = 0.5 * (a - dd), bc = b * c, disc = pp * pp + bc;
            if (tid == 0) {
                if (disc >= 0.0) {
                    const double z = pp + copysign(sqrt(disc), pp);
                    swr[found] = dd + z;
                    swr[found + 1] = z != 0.0 ? dd - bc / z : dd;
                    swi[found] = swi[found + 1] = 0.0;
                } else {
                    swr[found] = swr[found + 1] = dd + pp;
                    swi[found] = sqrt(-disc);
                    swi[found + 1] = -sqrt(-disc);
                }
                if (l > 0) sa[l * LA + l - 1] = 0.0;
            }
            found += 2;
            hi -= 2;
            its = 0;
            __syncthreads();
            continue;
        }
        if (total >= 30 * m) break;  // not converged: the rest stay NaN
        ++its;
        ++total;
        // shifts: the eigenvalues of the trailing 2 x 2 block, or an
        // exceptional pair after 10 and 20 steps without deflation
        double ssum, sprod;
        if (its == 10 || its == 20) {
            const double s = fabs(sa[hi * LA + hi - 1]) + fabs(sa[(hi - 1) * LA + hi - 2]);
            ssum = 1.5 * s;
            sprod = s * s;
        } else {
            const double a = sa[(hi - 1) * LA + hi - 1], dd = sa[hi * LA + hi];
            ssum = a + dd;
            sprod = a * dd - sa[(hi - 1) * LA + hi] * sa[hi * LA + hi - 1];
        }
        const double h00 = sa[l * LA + l], h01 = sa[l * LA + l + 1], h10 = sa[(l + 1) * LA + l];
        const double h11 = sa[(l + 1) * LA + l + 1], h21 = sa[(l + 2) * LA + l + 1];
        double x = h00 * h00 + h01 * h10 - ssum * h00 + sprod;
        double y = h10 * (h00 + h11 - ssum);
        double z = h10 * h21;
        for (int k = l; k <= hi - 1; ++k) {
            const int nr = k < hi - 1 ? 3 : 2;  // the last reflector acts on two rows
            // reflector of [x, y, z] (or [x, y]): v = [1, v1, v2], I - beta v v^T
            const double sg = y * y + (nr == 3 ? z * z : 0.0);
            double beta = 0.0, v1 = 0.0, v2 = 0.0;
            if (sg > 0.0) {
                const double mu = sqrt(x * x + sg);
                const double v0 = x <= 0.0 ? x - mu : -sg / (x + mu);
                beta = 2.0 * v0 * v0 / (sg + v0 * v0);
                v1 = y / v0;
                v2 = nr == 3 ? z / v0 : 0.0;
            }
            if (beta != 0.0) {
                // from the left: rows k .. k+nr-1, columns max(l, k-1) .. hi
                const int j0 = k > l ? k - 1 : l;
                for (int j = j0 + tid; j <= hi; j += blockDim.x) {
                    double w = sa[k * LA + j] + v1 * sa[(k + 1) * LA + j];
                    if (nr == 3) w += v2 * sa[(k + 2) * LA + j];
                    w *= beta;
                    sa[k * LA + j] -= w;
                    sa[(k + 1) * LA + j] -= w * v1;
                    if (nr == 3) sa[(k + 2) * LA + j] -= w * v2;
                }
                __syncthreads();
                // from the right: columns k .. k+nr-1, rows l .. min(k+3, hi)
                const int i1 = k + 3 < hi ? k + 3 : hi;
                for (int i = l + tid; i <= i1; i += blockDim.x) {
                    double w = sa[i * LA + k] + v1 * sa[i * LA + k + 1];
                    if (nr == 3) w += v2 * sa[i * LA + k + 2];
                    w *= beta;
                    sa[i * LA + k] -= w;
                    sa[i * LA + k + 1] -= w * v1;
                    if (nr == 3) sa[i * LA + k + 2] -= w * v2;
                }
                __syncthreads();
            }
            if (k < hi - 1) {
                x = sa[(k + 1) * LA + k];
                y = sa[(k + 2) * LA + k];
                z = k < hi - 2 ? sa[(k + 3) * LA + k] : 0.0;
            }
        }
        __syncthreads();
    }
    // 4. the eigenvalues (inverted for N; NaN for any not found), ordered:
    //    real ascending, then complex pairs by real part, (re, +im), (re, -im)
    if (tid == 0) {
        for (int i = found; i < m; ++i) swr[i] = swi[i] = nan;
        if (swapped)
            for (int i = 0; i < found; ++i) {
                const double a = swr[i], b = swi[i];
                if (b == 0.0) {
                    swr[i] = a != 0.0 ? 1.0 / a : INFINITY;
                } else {
                    const double q = a * a + b * b;
                    swr[i] = a / q;
                    swi[i] = -b / q;
                }
            }
        int o = 0;
        for (int pass = 0; pass < 2; ++pass) {  // the reals, then the pairs
            for (;;) {
                int best = -1;
                for (int i = 0; i < m; ++i) {
                    const bool real = swi[i] == 0.0, cand = pass == 0 ? real : swi[i] > 0.0;
                    if (!cand || swr[i] != swr[i]) continue;
                    if (best < 0 || swr[i] < swr[best] || (swr[i] == swr[best] && swi[i] < swi[best])) best = i;
                }
                if (best < 0) break;
                d.wr[o] = swr[best];
                d.wi[o] = pass == 0 ? 0.0 : swi[best];
                ++o;
                if (pass == 1) {
                    d.wr[o] = swr[best];
                    d.wi[o] = -swi[best];
                    ++o;
                }
                swr[best] = nan;  // taken
            }
        }
        for (; o < m; ++o) d.wr[o] = d.wi[o] = nan;
    }
}

__global__ __launch_bounds__(256) void k_block_eig(const BlockEigDesc* __restrict__ descs) {
    constexpr int MX = kJacobiMax, LA = MX + 1;
    __shared__ double s_a[MX * LA];  // row-major, row stride LA
    __shared__ double s_c[MX / 2], s_s[MX / 2];
    __shared__ int s_p[MX / 2], s_q[MX / 2];
    __shared__ double s_red[4];
    __shared__ int s_i[2];
    const BlockEigDesc d = descs[blockIdx.x];
    if (!d.active || d.m <= 0) return;
    const int m = d.m, tid = threadIdx.x;
    if (!d.symmetric) {
        if (m >= 3 && m <= kPencilMax) {
            static_assert(2 * kPencilMax * (kPencilMax + 1) + 3 * kPencilMax + 8 <= kJacobiMax * (kJacobiMax + 1),
                          "the pencil solver's LDS fits the symmetric block's");
            pencil_dense(d, s_a, s_i);
        } else if (tid == 0) {
            pencil_small(d);
        }
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
