// Supporting kernels of the split step on gfx950: batched MFMA GEMM, the
// repeated-squaring set-up and per-iteration epilogue, element-wise
// permutations (transposes, reversals J, sign fixes), norms, the split-point
// search and the counter-based Gaussian draw.  Every kernel takes an array of
// per-problem descriptors and uses blockIdx.z (or .y) as the problem index,
// so independent problems of different sizes share one launch.
#include "sdc_internal.hpp"
#include "sdc_aux.hpp"
#include "mfma.hpp"
#include "rawbuf.hpp"
#include "profiler.hpp"

namespace sdc {

// ---------------------------------------------------------------------------
// Reductions (256-thread blocks, wave64)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    return v;
}
// Result valid in thread 0.
__device__ inline double block_sum256(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double r = 0;
    if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
    return r;
}
// Non-negative doubles order like their bit patterns (NaN after +inf).
__device__ inline void atomic_max_nonneg(double* addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// ---------------------------------------------------------------------------
// Batched GEMM on the matrix cores: 64x64 output tile per 256-thread block,
// 2x2 waves of 32x32, K staged through LDS in chunks of 32.  The next chunk
// is loaded into registers while the current one is multiplied, so the
// global loads overlap the MFMAs; the registers go to LDS after the chunk.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc<T>* __restrict__ descs) {
    using M = Mfma<T>;
    typedef typename M::v4 v4;
    constexpr int KC = 32, PER = 64 * KC / 256;  // elements of A (and of B) per thread per chunk
    const GemmDesc<T> d = descs[blockIdx.z];
    if (!d.active) return;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    if (m0 >= d.M || n0 >= d.N) return;
    __shared__ T sA[KC][64 + 4];
    __shared__ T sB[KC][64 + 4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, gq = lane >> 4, ln = lane & 15;
    const int wm = wave >> 1, wn = wave & 1;
    v4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = v4{0, 0, 0, 0};
    T ra[PER], rb[PER];
    // element e (< 64 KC) of a chunk: A as (m, k) with m fastest unless A is
    // transposed, B as (k, n) with k fastest unless B is transposed, so that
    // consecutive threads read consecutive addresses
    auto a_mk = [&](int e, int& m, int& k) {
        if (!d.ta) { m = e & 63; k = e >> 6; } else { k = e & (KC - 1); m = e / KC; }
    };
    auto b_kn = [&](int e, int& k, int& n) {
        if (!d.tb) { k = e & (KC - 1); n = e / KC; } else { n = e & 63; k = e >> 6; }
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + 256 * t;
            int m, k, n;
            a_mk(e, m, k);
            T va = 0;
            if (m0 + m < d.M && k0 + k < d.K)
                va = d.ta ? d.A[(size_t)(m0 + m) * d.lda + k0 + k] : d.A[(size_t)(k0 + k) * d.lda + m0 + m];
            ra[t] = va;
            b_kn(e, k, n);
            T vb = 0;
            if (n0 + n < d.N && k0 + k < d.K)
                vb = d.tb ? d.B[(size_t)(k0 + k) * d.ldb + n0 + n] : d.B[(size_t)(n0 + n) * d.ldb + k0 + k];
            rb[t] = vb;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int e = tid + 256 * t;
            int m, k, n;
            a_mk(e, m, k);
            sA[k][m] = ra[t];
            b_kn(e, k, n);
            sB[k][n] = rb[t];
        }
    };
    load(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < d.K; k0 += KC) {
        const bool more = k0 + KC < d.K;
        if (more) load(k0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const T a0 = sA[kk * 4 + gq][wm * 32 + ln];
            const T a1 = sA[kk * 4 + gq][wm * 32 + 16 + ln];
            const T b0 = sB[kk * 4 + gq][wn * 32 + ln];
            const T b1 = sB[kk * 4 + gq][wn * 32 + 16 + ln];
            acc[0][0] = M::mma(a0, b0, acc[0][0]);
            acc[0][1] = M::mma(a0, b1, acc[0][1]);
            acc[1][0] = M::mma(a1, b0, acc[1][0]);
            acc[1][1] = M::mma(a1, b1, acc[1][1]);
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 32 + j * 16 + ln;
            if (n >= d.N) continue;
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm * 32 + i * 16 + M::row(gq, v);
                if (m >= d.M) continue;
                T* cp = d.C + (size_t)n * d.ldc + m;
                T r = d.alpha * acc[i][j][v];
                if (d.beta != T(0)) r += d.beta * *cp;
                *cp = r;
            }
        }
}

// The same product with a 128 x 128 output tile per 256-thread block (2 x 2
// waves of 64 x 64, sixteen 16x16x4 MFMAs per wave per k-step): each
// element of A and B staged in LDS feeds twice the multiply-adds of the
// 64 x 64 tile, which halves the operand traffic per flop (32 flop/B in
// FP32, 16 in FP64, both above the chip's balance, so the matrix cores
// rather than the memory bound it).  Operands are read through raw buffers
// (32-bit offsets from one scalar resource; an element outside the matrix
// is given the out-of-range offset and reads zero), so the loads need
// neither 64-bit addresses nor branches.  Same k order as k_gemm, so the
// results are the same bits.  For products whose M and N are both large and
// whose operands span less than 2^31 bytes.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_gemm128(const GemmDesc<T>* __restrict__ descs) {
    using M = Mfma<T>;
    typedef typename M::v4 v4;
    // K chunk: 32 (FP32) or 16 (FP64) rows of A and B in LDS, the same bytes
    constexpr int TM = 128, KC = sizeof(T) == 8 ? 16 : 32, PER = TM * KC / 256;
    const GemmDesc<T> d = descs[blockIdx.z];
    if (!d.active) return;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TM;
    if (m0 >= d.M || n0 >= d.N) return;
    __shared__ T sA[KC][TM + 4];
    __shared__ T sB[KC][TM + 4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, gq = lane >> 4, ln = lane & 15;
    const int wm = wave >> 1, wn = wave & 1;
    const RawBuf<T> ba(d.A, (unsigned)((size_t)d.lda * (d.ta ? d.M : d.K) * sizeof(T)));
    const RawBuf<T> bb(d.B, (unsigned)((size_t)d.ldb * (d.tb ? d.K : d.N) * sizeof(T)));
    v4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4{0, 0, 0, 0};
    T ra[PER], rb[PER];
    // Thread tid moves elements e = tid + 256 t (t < PER) of each chunk: A as
    // (m, k) with m fastest unless A is transposed, B as (k, n) with k
    // fastest unless B is transposed, so that consecutive threads read
    // consecutive addresses.  Either way element t sits at a fixed step from
    // element 0 (256 is a multiple of TM and KC), so the geometry is set once.
    int am, ak, adm, adk, bk, bn, bdk, bdn;
    if (!d.ta) { am = tid & (TM - 1); ak = tid / TM; adm = 0; adk = 256 / TM; }
    else { ak = tid & (KC - 1); am = tid / KC; adk = 0; adm = 256 / KC; }
    if (!d.tb) { bk = tid & (KC - 1); bn = tid / KC; bdk = 0; bdn = 256 / KC; }
    else { bn = tid & (TM - 1); bk = tid / TM; bdn = 0; bdk = 256 / TM; }
    // element strides of m and k in A, of k and n in B
    const unsigned a_sm = d.ta ? d.lda : 1, a_sk = d.ta ? 1 : d.lda;
    const unsigned b_sk = d.tb ? d.ldb : 1, b_sn = d.tb ? 1 : d.ldb;
    auto load = [&](int k0) {
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int m = m0 + am + t * adm, ka = k0 + ak + t * adk;
            ra[t] = ba.load(m < d.M && ka < d.K ? ((unsigned)m * a_sm + (unsigned)ka * a_sk) * (unsigned)sizeof(T)
                                                : kOob);
            const int n = n0 + bn + t * bdn, kb = k0 + bk + t * bdk;
            rb[t] = bb.load(n < d.N && kb < d.K ? ((unsigned)kb * b_sk + (unsigned)n * b_sn) * (unsigned)sizeof(T)
                                                : kOob);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            sA[ak + t * adk][am + t * adm] = ra[t];
            sB[bk + t * bdk][bn + t * bdn] = rb[t];
        }
    };
    load(0);
    stash();
    __syncthreads();
    for (int k0 = 0; k0 < d.K; k0 += KC) {
        const bool more = k0 + KC < d.K;
        if (more) load(k0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            T a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = sA[kk * 4 + gq][wm * 64 + i * 16 + ln];
                b[i] = sB[kk * 4 + gq][wn * 64 + i * 16 + ln];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = M::mma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
        if (more) {
            stash();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn * 64 + j * 16 + ln;
            if (n >= d.N) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm * 64 + i * 16 + M::row(gq, v);
                if (m >= d.M) continue;
                T* cp = d.C + (size_t)n * d.ldc + m;
                T r = d.alpha * acc[i][j][v];
                if (d.beta != T(0)) r += d.beta * *cp;
                *cp = r;
            }
        }
}

// Products whose M and N are at least this take the 128 x 128 tile (enough
// tiles to fill the chip at order 2048 and up; smaller ones keep the 64 x 64
// tile's parallelism).
constexpr int kGemmBigMin = 1024;

template <typename T>
void gemm_batch(const GemmDesc<T>* d_descs, const GemmDesc<T>* h, int count, hipStream_t s) {
    int M = 0, N = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) {
            M = M > h[i].M ? M : h[i].M;
            N = N > h[i].N ? N : h[i].N;
        }
    if (M == 0 || N == 0) return;
    Profiler* prof = g_prof;
    double fl = 0, by = 0;
    if (prof)
        for (int i = 0; i < count; ++i)
            if (h[i].active) {
                fl += 2.0 * h[i].M * h[i].N * h[i].K;
                by += ((double)h[i].M * h[i].K + (double)h[i].K * h[i].N + (double)h[i].M * h[i].N) * sizeof(T);
            }
    int mn_min = 1 << 30;
    bool small_span = true;  // every operand within the raw buffers' 2^31-byte range
    for (int i = 0; i < count; ++i)
        if (h[i].active) {
            mn_min = std::min(mn_min, std::min(h[i].M, h[i].N));
            const double sa = (double)h[i].lda * (h[i].ta ? h[i].M : h[i].K) * sizeof(T);
            const double sb = (double)h[i].ldb * (h[i].tb ? h[i].K : h[i].N) * sizeof(T);
            small_span = small_span && sa <= 2147483648.0 && sb <= 2147483648.0;
        }
    const int id = prof ? prof->begin(s) : -1;
    if (mn_min >= kGemmBigMin && small_span)
        hipLaunchKernelGGL(k_gemm128<T>, dim3((N + 127) / 128, (M + 127) / 128, count), dim3(256), 0, s, d_descs);
    else
        hipLaunchKernelGGL(k_gemm<T>, dim3((N + 63) / 64, (M + 63) / 64, count), dim3(256), 0, s, d_descs);
    if (prof) prof->end(id, s, PROF_GEMM, fl, by);
}
template void gemm_batch<double>(const GemmDesc<double>*, const GemmDesc<double>*, int, hipStream_t);
template void gemm_batch<float>(const GemmDesc<float>*, const GemmDesc<float>*, int, hipStream_t);

// ---------------------------------------------------------------------------
// Repeated squaring: set-up of W = [B0 A0 0; -A0 0 B0] (2n x 3n, ld 2n) from
// the FP64 inputs and the region map, and the per-iteration epilogue.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_irs_init(const IrsInit<T>* __restrict__ descs) {
    const IrsInit<T> d = descs[blockIdx.z];
    const int n = d.n;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= n) return;
    const double a = d.trans ? d.A[(size_t)i * d.lda + j] : d.A[(size_t)j * d.lda + i];
    double b;
    if (d.B) b = d.trans ? d.B[(size_t)i * d.ldb + j] : d.B[(size_t)j * d.ldb + i];
    else b = (i == j) ? 1.0 : 0.0;
    const T a0 = (T)(d.a1 * a + d.a2 * b);
    const T b0 = (T)(d.b1 * a + d.b2 * b);
    const size_t ld = (size_t)d.ld;
    T* W = d.W;
    W[(size_t)j * ld + i] = b0;
    W[(size_t)j * ld + n + i] = -a0;
    W[(size_t)(n + j) * ld + i] = a0;
    W[(size_t)(n + j) * ld + n + i] = T(0);
    W[(size_t)(2 * n + j) * ld + i] = T(0);
    W[(size_t)(2 * n + j) * ld + n + i] = b0;
}

template <typename T>
void irs_init_batch(const IrsInit<T>* d, const IrsInit<T>* h, int count, hipStream_t s) {
    int n = 0;
    for (int i = 0; i < count; ++i) n = n > h[i].n ? n : h[i].n;
    if (n == 0) return;
    hipLaunchKernelGGL(k_irs_init<T>, dim3((n + 63) / 64, (n + 3) / 4, count), dim3(256), 0, s, d);
}
template void irs_init_batch<double>(const IrsInit<double>*, const IrsInit<double>*, int, hipStream_t);
template void irs_init_batch<float>(const IrsInit<float>*, const IrsInit<float>*, int, hipStream_t);

// One block per column j.  After the augmented QR, rows [0, n) of the first
// block column hold R_j (diagonal as produced) and rows [n, 2n) of the second
// and third block columns hold A_{j+1} and B_{j+1}.  This kernel
//   * normalizes R_j to a non-negative diagonal (rows times sign(R_ii)),
//   * accumulates max column sums of |R_j - R_{j-1}|, |R_{j-1}| and |R_j|
//     in FP64 (the stopping test of Alg. 3, whatever the iterate precision),
//   * stores R_j as the next R_{j-1},
//   * rewrites W in place as [B_{j+1} A_{j+1} 0; -A_{j+1} 0 B_{j+1}].
template <typename T>
__global__ __launch_bounds__(256) void k_irs_post(const IrsDesc<T>* __restrict__ descs) {
    __shared__ double sh[4];
    const IrsDesc<T> d = descs[blockIdx.y];
    if (!d.active) return;
    const int n = d.n, j = blockIdx.x;
    if (j >= n) return;
    const size_t ld = (size_t)d.ld;
    T* W = d.W;
    double diff = 0, ref = 0, cur = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        double r = 0;
        if (i <= j) {
            r = (double)W[(size_t)j * ld + i];
            if (d.diag[i] < T(0)) r = -r;
        }
        const double rp = d.Rprev[(size_t)j * n + i];
        diff += fabs(r - rp);
        ref += fabs(rp);
        cur += fabs(r);
        d.Rprev[(size_t)j * n + i] = r;
        const T ap = W[(size_t)(n + j) * ld + n + i];
        const T bp = W[(size_t)(2 * n + j) * ld + n + i];
        W[(size_t)j * ld + i] = bp;
        W[(size_t)j * ld + n + i] = -ap;
        W[(size_t)(n + j) * ld + i] = ap;
        W[(size_t)(n + j) * ld + n + i] = T(0);
        W[(size_t)(2 * n + j) * ld + i] = T(0);
    }
    diff = block_sum256(diff, sh);
    ref = block_sum256(ref, sh);
    cur = block_sum256(cur, sh);
    if (threadIdx.x == 0) {
        atomic_max_nonneg(&d.norms[0], diff);
        atomic_max_nonneg(&d.norms[1], ref);
        atomic_max_nonneg(&d.norms[2], cur);
    }
}

template <typename T>
void irs_post_batch(const IrsDesc<T>* d, const IrsDesc<T>* h, int count, int /*first*/, hipStream_t s) {
    int n = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) n = n > h[i].n ? n : h[i].n;
    if (n == 0) return;
    hipLaunchKernelGGL(k_irs_post<T>, dim3(n, count), dim3(256), 0, s, d);
}
template void irs_post_batch<double>(const IrsDesc<double>*, const IrsDesc<double>*, int, int, hipStream_t);
template void irs_post_batch<float>(const IrsDesc<float>*, const IrsDesc<float>*, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Element-wise n x n operations.
// ---------------------------------------------------------------------------
// out[i + j ldo] = alpha * sgn * in[p + q ldi] with (p, q) = trans ? (j, i) : (i, j),
// then p -> n-1-p if revP and q -> n-1-q if revQ; sgn = sign(sg[p]) if sg.
// EW_ADD: out = in + in2.  EW_IDENTITY: out = I.  EW_SYM: out = (in + in^T)/2.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_ew(const EwDesc* __restrict__ descs) {
    const EwDesc d = descs[blockIdx.z];
    const int n = d.n;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (!d.active || i >= d.rows || j >= n) return;
    const Tin* in = static_cast<const Tin*>(d.in);
    Tout* out = static_cast<Tout*>(d.out);
    Tout r;
    switch (d.op) {
    case EW_PERMUTE: {
        int p = d.trans ? j : i, q = d.trans ? i : j;
        if (d.revP) p = (d.trans ? n : d.rows) - 1 - p;
        if (d.revQ) q = (d.trans ? d.rows : n) - 1 - q;
        double v = (double)in[(size_t)q * d.ldi + p];
        if (d.sg && d.sg[p] < 0) v = -v;
        r = (Tout)(d.alpha * v);
        break;
    }
    case EW_ADD: {
        const Tin* in2 = static_cast<const Tin*>(d.in2);
        r = (Tout)((double)in[(size_t)j * d.ldi + i] + (double)in2[(size_t)j * d.ld2 + i]);
        break;
    }
    case EW_IDENTITY:
        r = (i == j) ? Tout(1) : Tout(0);
        break;
    case EW_ZERO:
        r = Tout(0);
        break;
    default: {  // EW_SYM
        r = (Tout)(0.5 * ((double)in[(size_t)j * d.ldi + i] + (double)in[(size_t)i * d.ldi + j]));
        break;
    }
    }
    out[(size_t)j * d.ldo + i] = r;
}

template <typename Tin, typename Tout>
void ew_batch(const EwDesc* d, const EwDesc* h, int count, hipStream_t s) {
    int n = 0, rows = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) {
            n = n > h[i].n ? n : h[i].n;
            rows = rows > h[i].rows ? rows : h[i].rows;
        }
    if (n == 0 || rows == 0) return;
    hipLaunchKernelGGL((k_ew<Tin, Tout>), dim3((rows + 63) / 64, (n + 3) / 4, count), dim3(256), 0, s, d);
}
template void ew_batch<double, double>(const EwDesc*, const EwDesc*, int, hipStream_t);
template void ew_batch<float, double>(const EwDesc*, const EwDesc*, int, hipStream_t);
template void ew_batch<float, float>(const EwDesc*, const EwDesc*, int, hipStream_t);
template void ew_batch<double, float>(const EwDesc*, const EwDesc*, int, hipStream_t);

// Fill a device array (used instead of memset so the calls stay capturable).
template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
template <typename T>
void fill(T* p, size_t n, T v, hipStream_t s) {
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}
template void fill<double>(double*, size_t, double, hipStream_t);
template void fill<float>(float*, size_t, float, hipStream_t);
template void fill<unsigned>(unsigned*, size_t, unsigned, hipStream_t);

// Zero many small device arrays in one launch (one block per array).
__global__ __launch_bounds__(256) void k_zero(const ZeroDesc* __restrict__ descs) {
    const ZeroDesc d = descs[blockIdx.x];
    for (unsigned i = threadIdx.x; i < d.words; i += 256) d.p[i] = 0u;
}
void zero_batch(const ZeroDesc* d, int count, hipStream_t s) {
    if (count > 0) hipLaunchKernelGGL(k_zero, dim3(count), dim3(256), 0, s, d);
}

// ---------------------------------------------------------------------------
// Norms and the split-point search (Alg. 4 line 5; the prefix-sum plus max
// reduction of Sec. 4.2).
// ---------------------------------------------------------------------------
// out[0] = max_j sum_i |X_ij| (matrix 1-norm), one block per column.
__global__ __launch_bounds__(256) void k_norm1(const NormDesc* __restrict__ descs) {
    __shared__ double sh[4];
    const NormDesc d = descs[blockIdx.y];
    if (!d.active || (int)blockIdx.x >= d.n) return;
    const int j = blockIdx.x;
    double s = 0;
    for (int i = threadIdx.x; i < d.rows; i += 256) s += fabs(d.X[(size_t)j * d.ld + i]);
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) atomic_max_nonneg(d.out, s);
}
void norm1_batch(const NormDesc* d, const NormDesc* h, int count, hipStream_t s) {
    int n = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) n = n > h[i].n ? n : h[i].n;
    if (n == 0) return;
    hipLaunchKernelGGL(k_norm1, dim3(n, count), dim3(256), 0, s, d);
}

// Column suffix sums: S[k + c n] = sum_{i >= k} |X_ic| (one block per column c).
__global__ __launch_bounds__(256) void k_suffix(const SplitDesc* __restrict__ descs, int which) {
    __shared__ double part[256];
    const SplitDesc d = descs[blockIdx.y];
    const int n = d.n, c = blockIdx.x;
    if (!d.active || c >= n) return;
    const double* X = which ? d.Bh : d.Ah;
    const int ldx = which ? d.ldb : d.lda;
    if (!X) return;
    double* S = (which ? d.SB : d.SA) + (size_t)c * n;
    const int chunk = (n + 255) / 256;
    const int lo = threadIdx.x * chunk, hi = min(n, lo + chunk);
    double s = 0;
    for (int i = lo; i < hi; ++i) s += fabs(X[(size_t)c * ldx + i]);
    part[threadIdx.x] = s;
    __syncthreads();
    // suffix offset of this chunk: sum of later chunks
    double off = 0;
    for (int t = threadIdx.x + 1; t < 256; ++t) off += part[t];
    double run = off;
    for (int i = hi - 1; i >= lo; --i) {
        run += fabs(X[(size_t)c * ldx + i]);
        S[i] = run;
    }
}

// e[k] = max_{c<k} SA[k + c n]/normA (+ max_{c<k} SB[k + c n]/normB), k = 1..n-1.
__global__ __launch_bounds__(256) void k_emax(const SplitDesc* __restrict__ descs) {
    const SplitDesc d = descs[blockIdx.y];
    const int n = d.n;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (!d.active || k < 1 || k >= n) return;
    double ea = 0, eb = 0;
    for (int c = 0; c < k; ++c) ea = fmax(ea, d.SA[(size_t)c * n + k]);
    double e = ea / d.norms[0];
    if (d.Bh) {
        for (int c = 0; c < k; ++c) eb = fmax(eb, d.SB[(size_t)c * n + k]);
        e += eb / d.norms[1];
    }
    d.e[k] = e;
}

// argmin over k = 1..n-1 (smallest k on ties); out[0] = k*, out[1] = e(k*).
__global__ __launch_bounds__(256) void k_argmin(const SplitDesc* __restrict__ descs) {
    __shared__ double sv[256];
    __shared__ int sk[256];
    const SplitDesc d = descs[blockIdx.x];
    if (!d.active) return;
    double best = INFINITY;
    int bk = 0;
    for (int k = 1 + threadIdx.x; k < d.n; k += 256) {
        const double v = d.e[k];
        if (bk == 0 || v < best || best != best) {  // k increases: ties keep the first
            best = v;
            bk = k;
        }
    }
    sv[threadIdx.x] = best;
    sk[threadIdx.x] = bk;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const double v2 = sv[threadIdx.x + o];
            const int k2 = sk[threadIdx.x + o];
            const double v1 = sv[threadIdx.x];
            const int k1 = sk[threadIdx.x];
            bool take = false;
            if (k2 != 0) {
                if (k1 == 0) take = true;
                else if (v2 < v1) take = true;
                else if (v2 == v1 && k2 < k1) take = true;
                else if (v1 != v1 && v2 == v2) take = true;  // prefer a number over NaN
            }
            if (take) { sv[threadIdx.x] = v2; sk[threadIdx.x] = k2; }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.out[0] = (double)sk[0];
        d.out[1] = sv[0];
    }
}

void split_search_batch(const SplitDesc* d, const SplitDesc* h, int count, hipStream_t s) {
    int n = 0, pencil = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) {
            n = n > h[i].n ? n : h[i].n;
            pencil |= h[i].Bh != nullptr;
        }
    if (n == 0) return;
    hipLaunchKernelGGL(k_suffix, dim3(n, count), dim3(256), 0, s, d, 0);
    if (pencil) hipLaunchKernelGGL(k_suffix, dim3(n, count), dim3(256), 0, s, d, 1);
    hipLaunchKernelGGL(k_emax, dim3((n + 255) / 256, count), dim3(256), 0, s, d);
    hipLaunchKernelGGL(k_argmin, dim3(count), dim3(256), 0, s, d);
}

__global__ __launch_bounds__(256) void k_gersh(const GershDesc* __restrict__ descs) {
    __shared__ double sh[4];
    const GershDesc d = descs[blockIdx.y];
    if (!d.active || (int)blockIdx.x >= d.n) return;
    const int j = blockIdx.x;
    double s = 0;
    for (int i = threadIdx.x; i < d.n; i += 256)
        if (i != j) s += fabs(d.X[(size_t)j * d.ld + i]);
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) {
        const double c = d.X[(size_t)j * d.ld + j];
        d.out[2 * j] = c - s;
        d.out[2 * j + 1] = c + s;
    }
}
void gersh_batch(const GershDesc* d, const GershDesc* h, int count, hipStream_t s) {
    int n = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) n = n > h[i].n ? n : h[i].n;
    if (n == 0) return;
    hipLaunchKernelGGL(k_gersh, dim3(n, count), dim3(256), 0, s, d);
}

// ||X^T X - I||_F^2 accumulated into out (X n x n), one block per column of E.
__global__ __launch_bounds__(256) void k_orth_err(const NormDesc* __restrict__ descs) {
    __shared__ double sh[4];
    const NormDesc d = descs[blockIdx.y];
    if (!d.active || (int)blockIdx.x >= d.n) return;
    const int j = blockIdx.x;
    double s = 0;
    for (int i = threadIdx.x; i < d.n; i += 256) {
        const double e = d.X[(size_t)j * d.ld + i] - (i == j ? 1.0 : 0.0);
        s += e * e;
    }
    s = block_sum256(s, sh);
    if (threadIdx.x == 0) atomicAdd(d.out, s);
}
void orth_err_batch(const NormDesc* d, const NormDesc* h, int count, hipStream_t s) {
    int n = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) n = n > h[i].n ? n : h[i].n;
    if (n == 0) return;
    hipLaunchKernelGGL(k_orth_err, dim3(n, count), dim3(256), 0, s, d);
}

// ---------------------------------------------------------------------------
// Gaussian draw: Philox4x32-10 (Salmon et al., SC'11) + Box-Muller.
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__global__ __launch_bounds__(256) void k_gauss(const GaussDesc* __restrict__ descs) {
    const GaussDesc d = descs[blockIdx.z];
    const int n = d.n;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (!d.active || i >= n || j >= n) return;
    const uint64_t e = (uint64_t)i + (uint64_t)j * (uint64_t)n;
    uint32_t c[4] = {(uint32_t)e, (uint32_t)(e >> 32), (uint32_t)d.tag, 0u};
    philox4x32_10(c, (uint32_t)d.seed, (uint32_t)(d.seed >> 32));
    const uint64_t x1 = (((uint64_t)c[1] << 32) | c[0]) >> 11;
    const uint64_t x2 = (((uint64_t)c[3] << 32) | c[2]) >> 11;
    const double u1 = ((double)x1 + 0.5) * 0x1.0p-53;
    const double u2 = (double)x2 * 0x1.0p-53;
    d.G[(size_t)j * d.ld + i] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}
void gauss_batch(const GaussDesc* d, const GaussDesc* h, int count, hipStream_t s) {
    int n = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) n = n > h[i].n ? n : h[i].n;
    if (n == 0) return;
    hipLaunchKernelGGL(k_gauss, dim3((n + 63) / 64, (n + 3) / 4, count), dim3(256), 0, s, d);
}

__global__ __launch_bounds__(256) void k_gather(const GatherDesc* __restrict__ descs, double* __restrict__ dst) {
    const GatherDesc d = descs[blockIdx.x];
    for (int i = threadIdx.x; i < d.n; i += 256) dst[d.off + i] = d.src[i];
}

void gather_batch(const GatherDesc* d, int count, double* dst, hipStream_t s) {
    if (count > 0) hipLaunchKernelGGL(k_gather, dim3(count), dim3(256), 0, s, d, dst);
}

}  // namespace sdc
