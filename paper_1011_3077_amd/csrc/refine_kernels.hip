// Conjugate gradients for the Sylvester equation of the FP64 refinement of a
// symmetric split:  X A11 - A22 X = E  (X and E are m x k, m = n - k).
//
// With the eigenvalues of A11 above those of A22 (the leading block holds the
// eigenvalues on the far side of the split point), the operator
// X -> X A11 - A22 X is symmetric positive definite in the trace inner
// product, so plain CG converges; its two products run as batched GEMMs
// between these kernels.  The kernels here do the vector work of one CG
// iteration, batched over problems (blockIdx.y).
//
// Determinism: every inner product is reduced in a fixed order.  A problem
// uses nblk blocks (a function of its own size only); block b writes its
// partial sum to slot b, and the consumer kernels re-sum the nblk slots
// themselves.  So a problem's result does not depend on the batch it runs in.
//
// Convergence is decided on the device: once rr_i <= tol2 * rr_0, or the
// curvature p^T M p is not positive, the iteration is frozen and every later
// kernel leaves X untouched, so the host may launch iterations in chunks
// between checks.
#include "sdc_aux.hpp"

namespace sdc {

namespace {

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;  // every lane holds the sum
}

// Sum of the nblk partials at p (all threads get the result).
__device__ inline double sum_partials(const double* p, int nblk, double* sh) {
    double v = 0;
    for (int i = threadIdx.x; i < nblk; i += 256) v += p[i];
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// Block sum written to slot blockIdx.x of out (and of out2 if given).
__device__ inline void put_partial(double v, double* out, double* sh, double* out2 = nullptr) {
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        out[blockIdx.x] = t;
        if (out2) out2[blockIdx.x] = t;
    }
}

}  // namespace

int cg_blocks(int m, int k) {
    const long long mk = (long long)m * k;
    long long b = (mk + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > kCgMaxBlocks) b = kCgMaxBlocks;
    return (int)b;
}

// X = 0, R = P = E; rr_0 partials.
__global__ __launch_bounds__(256) void k_cg_init(const CgDesc* __restrict__ descs) {
    __shared__ double sh[4];
    const CgDesc d = descs[blockIdx.y];
    if (!d.active || (int)blockIdx.x >= d.nblk) return;
    const long long mk = (long long)d.m * d.k;
    double acc = 0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < mk; e += (long long)d.nblk * 256) {
        const int i = (int)(e % d.m), j = (int)(e / d.m);
        const double v = d.E[(size_t)j * d.lde + i];
        d.X[e] = 0.0;
        d.R[e] = v;
        d.P[e] = v;
        acc += v * v;
    }
    put_partial(acc, d.rr0, sh, d.rr);  // ring slot 0 holds rr_0 too
}

// pz_i = <P, Z> unless frozen.
__global__ __launch_bounds__(256) void k_cg_dot(const CgDesc* __restrict__ descs, int it) {
    __shared__ double sh[4];
    const CgDesc d = descs[blockIdx.y];
    if (!d.active || (int)blockIdx.x >= d.nblk) return;
    const double rr = sum_partials(d.rr + (it % 3) * kCgMaxBlocks, d.nblk, sh);
    const double r0 = sum_partials(d.rr0, d.nblk, sh);
    if (rr <= d.tol2 * r0) return;
    const long long mk = (long long)d.m * d.k;
    double acc = 0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < mk; e += (long long)d.nblk * 256) acc += d.P[e] * d.Z[e];
    put_partial(acc, d.pz, sh);
}

// alpha = rr_i / pz_i; X += alpha P; R -= alpha Z; rr_{i+1} partials.
__global__ __launch_bounds__(256) void k_cg_step(const CgDesc* __restrict__ descs, int it) {
    __shared__ double sh[4];
    const CgDesc d = descs[blockIdx.y];
    if (!d.active || (int)blockIdx.x >= d.nblk) return;
    const double* rr_cur = d.rr + (it % 3) * kCgMaxBlocks;
    double* rr_nxt = d.rr + ((it + 1) % 3) * kCgMaxBlocks;
    const double rr = sum_partials(rr_cur, d.nblk, sh);
    const double r0 = sum_partials(d.rr0, d.nblk, sh);
    if (rr <= d.tol2 * r0) {  // converged: carry rr forward
        if (threadIdx.x == 0) rr_nxt[blockIdx.x] = rr_cur[blockIdx.x];
        return;
    }
    const double pz = sum_partials(d.pz, d.nblk, sh);
    if (!(pz > 0.0)) {  // breakdown (operator not definite): freeze
        if (threadIdx.x == 0) rr_nxt[blockIdx.x] = 0.0;
        return;
    }
    const double alpha = rr / pz;
    const long long mk = (long long)d.m * d.k;
    double acc = 0;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < mk; e += (long long)d.nblk * 256) {
        d.X[e] += alpha * d.P[e];
        const double r = d.R[e] - alpha * d.Z[e];
        d.R[e] = r;
        acc += r * r;
    }
    put_partial(acc, rr_nxt, sh);
}

// beta = rr_{i+1} / rr_i; P = R + beta P.
__global__ __launch_bounds__(256) void k_cg_dir(const CgDesc* __restrict__ descs, int it) {
    __shared__ double sh[4];
    const CgDesc d = descs[blockIdx.y];
    if (!d.active || (int)blockIdx.x >= d.nblk) return;
    const double rr = sum_partials(d.rr + (it % 3) * kCgMaxBlocks, d.nblk, sh);
    const double r0 = sum_partials(d.rr0, d.nblk, sh);
    if (rr <= d.tol2 * r0) return;
    const double pz = sum_partials(d.pz, d.nblk, sh);
    if (!(pz > 0.0)) return;
    const double rn = sum_partials(d.rr + ((it + 1) % 3) * kCgMaxBlocks, d.nblk, sh);
    const double beta = rn / rr;
    const long long mk = (long long)d.m * d.k;
    for (long long e = blockIdx.x * 256LL + threadIdx.x; e < mk; e += (long long)d.nblk * 256)
        d.P[e] = d.R[e] + beta * d.P[e];
}

static int max_blocks(const CgDesc* h, int count) {
    int b = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active && h[i].nblk > b) b = h[i].nblk;
    return b;
}

void cg_init_batch(const CgDesc* d, const CgDesc* h, int count, hipStream_t s) {
    const int b = max_blocks(h, count);
    if (b) hipLaunchKernelGGL(k_cg_init, dim3(b, count), dim3(256), 0, s, d);
}
void cg_iter_vec(const CgDesc* d, const CgDesc* h, int count, int it, int phase, hipStream_t s) {
    const int b = max_blocks(h, count);
    if (!b) return;
    if (phase == 0) hipLaunchKernelGGL(k_cg_dot, dim3(b, count), dim3(256), 0, s, d, it);
    else if (phase == 1) hipLaunchKernelGGL(k_cg_step, dim3(b, count), dim3(256), 0, s, d, it);
    else hipLaunchKernelGGL(k_cg_dir, dim3(b, count), dim3(256), 0, s, d, it);
}

}  // namespace sdc
