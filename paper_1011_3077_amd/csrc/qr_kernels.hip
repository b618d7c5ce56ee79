// Augmented blocked Householder QR on gfx950.
//
// For an m x ncols column-major matrix W, the leading nf columns are reduced
// to upper-triangular form by Householder reflectors, and the transpose of
// the accumulated orthogonal factor is applied to ALL ncols columns.  The
// repeated squaring step (Alg. 3) uses it on W = [B_j A_j 0; -A_j 0 B_j]:
// the QR of the first block column [B_j; -A_j] leaves R_j in the top rows and
// turns the bottom halves of the two extra block columns into
// Q12^T A_j = A_{j+1} and Q22^T B_j = B_{j+1}, so no explicit Q is formed.
//
// Panels are NB columns wide.  A panel's QR is a reduction tree of Householder
// QRs over row blocks (the TSQR panel of communication-avoiding QR, which the
// paper uses for its QR costs, Sec. 4.2): leaves of about H rows, then nodes
// stacking up to F child R factors.  One kernel launch factors every node of
// a panel; the last workgroup to finish among a node's children (counted with
// an atomic) factors the parent, so no grid-wide barrier is needed.  The
// trailing update applies the tree level by level: each node's block
// reflector I - V T V^T is applied to its rows of every trailing column tile
// on the matrix cores (MFMA), keeping the tile in registers.
#include "sdc_internal.hpp"
#include "mfma.hpp"
#include "rawbuf.hpp"
#include "profiler.hpp"

namespace sdc {

// ---------------------------------------------------------------------------
// Cross-lane moves inside one wavefront (T = float or double).
// ---------------------------------------------------------------------------
// Every control used here (quad permutes and row mirrors, all rows and banks
// enabled) writes every lane from a valid source lane, so the move needs no
// old value: a plain DPP move per 32-bit half, without the register
// initialisation (and its hazard wait) that an update with an old value of
// zero costs.
template <int CTRL, typename T> __device__ __forceinline__ T lane_dpp(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
        const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
    }
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]: lane ^ 1
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]: lane ^ 2
constexpr int kDppHalfMirror = 0x141; // lane ^ 7 within each 8 lanes
constexpr int kDppMirror = 0x140;     // lane ^ 15 within each 16 lanes

// v(lane) + v(lane ^ 16) (R16) or v(lane) + v(lane ^ 32) (R32) in every lane,
// with the gfx950 row swaps: swapping a value with itself across 16-lane
// (32-lane) rows leaves one copy of the pair in each result, so their sum is
// the pair sum, in the same order in both lanes of a pair.
template <bool R32> __device__ __forceinline__ void row_swap(unsigned& x, unsigned& y) {
    if constexpr (R32) {
        const auto p = __builtin_amdgcn_permlane32_swap(x, y, false, false);
        x = p[0];
        y = p[1];
    } else {
        const auto p = __builtin_amdgcn_permlane16_swap(x, y, false, false);
        x = p[0];
        y = p[1];
    }
}
template <bool R32, typename T> __device__ __forceinline__ T pair_sum(T v) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        unsigned lo0 = (unsigned)b, lo1 = lo0, hi0 = (unsigned)(b >> 32), hi1 = hi0;
        row_swap<R32>(lo0, lo1);
        row_swap<R32>(hi0, hi1);
        const T u = __builtin_bit_cast(T, ((unsigned long long)hi0 << 32) | lo0);
        const T w = __builtin_bit_cast(T, ((unsigned long long)hi1 << 32) | lo1);
        return u + w;
    } else {
        unsigned x = __builtin_bit_cast(unsigned, v), y = x;
        row_swap<R32>(x, y);
        return __builtin_bit_cast(T, x) + __builtin_bit_cast(T, y);
    }
}

// Value of v in lane `lane` (a wave-uniform index), for every lane.
template <typename T> __device__ __forceinline__ T lane_read(T v, int lane) {
    if constexpr (sizeof(T) == 8) {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_readlane((int)b, lane);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __builtin_bit_cast(T, ((long long)hi << 32) | (long long)(unsigned)lo);
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
    }
}

// Sum of v over the 64 lanes, in every lane (each stage adds the partner's
// value, a + b in one lane and b + a in the other, so all lanes agree bitwise).
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
    v += lane_dpp<kDppXor1>(v);
    v += lane_dpp<kDppXor2>(v);
    v += lane_dpp<kDppHalfMirror>(v);
    v += lane_dpp<kDppMirror>(v);
    v = pair_sum<false>(v);
    return pair_sum<true>(v);
}

// Sum of x over lanes l and l ^ 32 (R32) or l ^ 16 (R16) in the lanes with
// that lane bit clear, and of y in the lanes with it set: one gfx950 row swap
// exchanges x's upper rows with y's lower ones, so x + y holds both pair sums
// (an exchange stage of a transposed reduction, without selects).
template <bool R32, typename T> __device__ __forceinline__ T swap_sum(T x, T y) {
    if constexpr (sizeof(T) == 8) {
        const unsigned long long bx = __builtin_bit_cast(unsigned long long, x);
        const unsigned long long by = __builtin_bit_cast(unsigned long long, y);
        unsigned xl = (unsigned)bx, xh = (unsigned)(bx >> 32), yl = (unsigned)by, yh = (unsigned)(by >> 32);
        row_swap<R32>(xl, yl);
        row_swap<R32>(xh, yh);
        return __builtin_bit_cast(T, ((unsigned long long)xh << 32) | xl) +
               __builtin_bit_cast(T, ((unsigned long long)yh << 32) | yl);
    } else {
        unsigned a = __builtin_bit_cast(unsigned, x), b = __builtin_bit_cast(unsigned, y);
        row_swap<R32>(a, b);
        return __builtin_bit_cast(T, a) + __builtin_bit_cast(T, b);
    }
}

// Sums over the 64 lanes of eight values q[0..7] at once, as a transposed
// reduction: each exchange stage pairs two of a lane's values with a
// partner lane, keeps one of them summed over both lanes and hands the other
// over, halving the values a lane carries.  The first two stages exchange
// across 32-lane halves and 16-lane rows by row swaps (bits 5 and 4 of the
// lane pick the value kept), the third within each row over the DPP mirror
// (bit 3, with selects); three plain stages finish the sum over the eight
// lanes that carry the same value.  Lane l ends with the total of column
// c(l) = (l >> 3) & 7, so column c's total is in lane 8 c (among others).
template <typename T> __device__ __forceinline__ T wave_sum8(const T (&q)[8], int lane) {
    const bool b3 = (lane >> 3) & 1;
    T h[4], g[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) h[k] = swap_sum<true>(q[k], q[k + 4]);  // column k, or k + 4 if bit 5
#pragma unroll
    for (int k = 0; k < 2; ++k) g[k] = swap_sum<false>(h[k], h[k + 2]);  // + 2 if bit 4
    const T keep = b3 ? g[1] : g[0], send = b3 ? g[0] : g[1];          // partner lane ^ 15: + 1 if bit 3
    T f = keep + lane_dpp<kDppMirror>(send);
    f += lane_dpp<kDppHalfMirror>(f);
    f += lane_dpp<kDppXor2>(f);
    f += lane_dpp<kDppXor1>(f);
    return f;
}

// ---------------------------------------------------------------------------
// Householder QR of one tree node held in registers, row-owner layout: wave
// wv = tid / 64 owns columns [8 wv, 8 wv + 8) and lane l its rows l + 64 i
// (i < NRW), so a wave holds whole columns and the dot products of a step
// are summed inside the wave by lane exchanges, not through LDS.  Only
// column j crosses waves: its owner publishes it to LDS, with its squared
// norm below the diagonal and its diagonal entry alpha, before the step's
// single barrier.
//
// Step j (H_j = I - tau v v^T, v_j = 1, beta = -sign(alpha) ||x||,
// d = alpha - beta, v = x / d below the diagonal, tau = -d / beta): with
// xh = x below the diagonal, xh_j = d and 0 above, v = xh / d on rows >= j, so
//   S_c = sum_r xh_r a_rc   (one eight-column wave sum),
//   w_c = v^T a_c = S_c / d (for c < j this is v_c^T v_j),
//   a_c <- a_c - (tau w_c / d) xh   for c > j,
// and column j becomes beta on the diagonal and v below it.  Rows beyond the
// node and columns >= nbk are zero and stay zero.
//
// The compact-WY factor (H_0 ... H_{nbk-1} = I - V T V^T, T upper
// triangular) follows the forward recurrence
//   T[i][j] = -tau_j sum_{l=i}^{j-1} T[i][l] (v_l^T v_j),  T[j][j] = tau_j,
// built alongside: lanes i < NB of wave wv keep T[i][l] for the wave's
// columns l; at step j each wave adds up its columns' share of the sum with
// the w_l it already has, leaves it in LDS, and the owner of column j
// finishes that column after the next barrier.
// ---------------------------------------------------------------------------
template <typename T, int NRW, int CW, int CC>
__device__ __forceinline__ void qr_publish(const T (&a)[NRW][CW], int jn, T* xs, T* sc) {
    const int l = threadIdx.x & 63;
    T nsq = 0;
#pragma unroll
    for (int i = 0; i < NRW; ++i) {
        const int r = l + 64 * i;
        const T v = a[i][CC];
        xs[r] = v;
        nsq += r > jn ? v * v : T(0);
    }
    nsq = wave_sum(nsq);
    const T al = lane_read(a[0][CC], jn);  // row jn < 64 is register 0 of lane jn
    if (l == 0) {
        sc[0] = nsq;
        sc[1] = al;
    }
}

// T column j of the node from the waves' partial sums p[4][NB] (lanes i < NB).
template <typename T, int NB>
__device__ __forceinline__ T qr_tcol(const T* p, int j, T tauj) {
    const int i = threadIdx.x & (NB - 1), l = threadIdx.x & 63;
    const T s = (p[i] + p[NB + i]) + (p[2 * NB + i] + p[3 * NB + i]);
    return l < j ? -tauj * s : (l == j ? tauj : T(0));
}

// One column step; CW = NB / 4 columns per wave (8 or 16).
template <typename T, int NRW, int CW, int JJ>
__device__ __forceinline__ bool qr_step(T (&a)[NRW][CW], T (&tc)[CW], T& tau_prev, int jw, int nbk, T* s_x, T* s_sc,
                                        T* s_P, T* s_tau, T* s_beta) {
    constexpr int NB = 4 * CW;
    const int j = CW * jw + JJ;
    if (j >= nbk) return false;
    const int tid = threadIdx.x, l = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: scalar branches below
    const int par = j & 1;
    const T* xs = s_x + par * 256;
    const T xn2 = s_sc[par * 2], alpha = s_sc[par * 2 + 1];
    T xh[NRW];
#pragma unroll
    for (int i = 0; i < NRW; ++i) {
        const int r = l + 64 * i;
        const T x = xs[r];
        xh[i] = r > j ? x : T(0);
    }
    // finish T column j - 1 (its owner, register (JJ + CW - 1) % CW)
    if (j > 0 && wv == (j - 1) / CW) tc[(JJ + CW - 1) % CW] = qr_tcol<T, NB>(s_P + (par ^ 1) * 4 * NB, j - 1, tau_prev);
    // reflector scalars, without branches (the zero-norm case selected at the end)
    const T nrm = sqrt(alpha * alpha + xn2);
    const T b0 = alpha >= T(0) ? -nrm : nrm;
    const T d0 = alpha - b0;
    // one division: rr = 1 / (beta d) gives 1 / d = beta rr, tau = -d / beta = -d^2 rr
    const T rr = T(1) / (b0 * d0);
    const bool zero = xn2 == T(0);
    const T beta = zero ? alpha : b0;
    const T scale = zero ? T(0) : b0 * rr;
    const T tau = zero ? T(0) : -(d0 * d0) * rr;
    const T dd = zero ? T(0) : d0;
    // products over the rows below the diagonal, then row j's term (row j < 64:
    // register 0 of lane j) once d is known
    T q[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        T s = xh[0] * a[0][c];
#pragma unroll
        for (int i = 1; i < NRW; ++i) s = fma(xh[i], a[i][c], s);
        q[c] = s;
    }
    const bool rowj = l == j;
    const T dj = rowj ? dd : T(0);
#pragma unroll
    for (int c = 0; c < CW; ++c) q[c] = fma(dj, a[0][c], q[c]);
    xh[0] = rowj ? dd : xh[0];
    // S_c (wave-uniform), eight columns per wave sum; w_c = scale S_c
    T sc8[CW];
#pragma unroll
    for (int h = 0; h < CW / 8; ++h) {
        T q8[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) q8[c] = q[8 * h + c];
        const T f = wave_sum8(q8, l);
#pragma unroll
        for (int c = 0; c < 8; ++c) sc8[8 * h + c] = lane_read(f, 8 * c);
    }
    // this wave's share of T column j, scale sum_c T[i][c] S_c (tc is zero
    // for columns >= j)
    T pj = tc[0] * sc8[0];
#pragma unroll
    for (int c = 1; c < CW; ++c) pj = fma(tc[c], sc8[c], pj);
    if (l < NB) s_P[par * 4 * NB + wv * NB + l] = scale * pj;
    // a_c <- a_c - (tau w_c / d) xh = a_c - S_c (tau scale^2 xh) for the
    // columns after j: all of a later wave's, those after JJ in j's own wave
    const T g = tau * scale * scale;
    T u[NRW];
#pragma unroll
    for (int i = 0; i < NRW; ++i) u[i] = g * xh[i];
    // (selects on wave-uniform conditions: no branches, whose register
    // copies would cost more than the products they skip)
    const bool later = wv > jw, own = wv == jw;
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        const T cf = (later || (own && c > JJ)) ? sc8[c] : T(0);
#pragma unroll
        for (int i = 0; i < NRW; ++i) a[i][c] = fma(-cf, u[i], a[i][c]);
    }
#pragma unroll
    for (int i = 0; i < NRW; ++i) {
        const int r = l + 64 * i;
        const T vj = r > j ? xh[i] * scale : (r == j ? beta : a[i][JJ]);
        a[i][JJ] = own ? vj : a[i][JJ];
    }
    if (tid == 0) {
        s_tau[j] = tau;
        s_beta[j] = beta;
    }
    tau_prev = tau;
    if (j + 1 < nbk) {
        if (wv == (j + 1) / CW)
            qr_publish<T, NRW, CW, (JJ + 1) % CW>(a, j + 1, s_x + ((j + 1) & 1) * 256, s_sc + ((j + 1) & 1) * 2);
        __syncthreads();
    }
    return true;
}

// The CW column steps of wave-block jw, JJ = J0 .. CW - 1 (false once past nbk).
template <typename T, int NRW, int CW, int J0>
__device__ __forceinline__ bool qr_steps(T (&a)[NRW][CW], T (&tc)[CW], T& tau_prev, int jw, int nbk, T* s_x,
                                         T* s_sc, T* s_P, T* s_tau, T* s_beta) {
    if constexpr (J0 >= CW) {
        return true;
    } else {
        if (!qr_step<T, NRW, CW, J0>(a, tc, tau_prev, jw, nbk, s_x, s_sc, s_P, s_tau, s_beta)) return false;
        return qr_steps<T, NRW, CW, J0 + 1>(a, tc, tau_prev, jw, nbk, s_x, s_sc, s_P, s_tau, s_beta);
    }
}

// Factor the node; T (NB x NB, column-major) goes to Tg.  s_P holds 8 NB
// elements of scratch.
template <typename T, int NRW, int CW>
__device__ __forceinline__ void node_qr_rows(T (&a)[NRW][CW], int nbk, T* s_x, T* s_sc, T* s_P, T* s_tau, T* s_beta,
                                             T* Tg) {
    constexpr int NB = 4 * CW;
    static_assert(QrCfg<T, NB>::PT == 256, "four waves of NB / 4 columns");
    const int tid = threadIdx.x, wv = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
    T tc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) tc[c] = 0;
    T tau_prev = 0;
    if (tid < 64) qr_publish<T, NRW, CW, 0>(a, 0, s_x, s_sc);
    __syncthreads();
    for (int jw = 0; jw < 4; ++jw)
        if (!qr_steps<T, NRW, CW, 0>(a, tc, tau_prev, jw, nbk, s_x, s_sc, s_P, s_tau, s_beta)) break;
    __syncthreads();
    // last column of T
    const int jl = nbk - 1;
    if (wv == jl / CW) {
        const T t = qr_tcol<T, NB>(s_P + (jl & 1) * 4 * NB, jl, tau_prev);
#pragma unroll
        for (int c = 0; c < CW; ++c) tc[c] = c == (jl % CW) ? t : tc[c];
    }
    if (l < NB) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int col = CW * wv + c;
            Tg[col * NB + l] = (l <= col && col < nbk) ? tc[c] : T(0);
        }
    }
}

// Factor the mt x nbk node staged column-major in s_tile (stride LDT) with
// NRW register rows per lane (64 NRW >= mt): load, QR, write T (NB x NB,
// column-major) to Tg, and put R/V back into s_tile.  The start of s_tile
// serves as scratch while the node is in registers.
template <typename T, int NRW, int NB>
__device__ __forceinline__ void factor_tile_rows(T* s_tile, int mt, int nbk, T* s_x, T* s_sc, T* s_tau, T* s_beta,
                                                 T* Tg) {
    constexpr int LDT = QrCfg<T, NB>::MT_MAX + 1, CW = NB / 4;
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    T a[NRW][CW];
#pragma unroll
    for (int i = 0; i < NRW; ++i)
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int r = l + 64 * i;
            a[i][c] = r < mt ? s_tile[(CW * wv + c) * LDT + r] : T(0);
        }
    __syncthreads();
    node_qr_rows<T, NRW, CW>(a, nbk, s_x, s_sc, s_tile, s_tau, s_beta, Tg);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NRW; ++i)
#pragma unroll
        for (int c = 0; c < CW; ++c) s_tile[(CW * wv + c) * LDT + l + 64 * i] = a[i][c];
    __syncthreads();
}

template <typename T, int NB>
__device__ __forceinline__ void factor_node(T* s_tile, int mt, int nbk, T* s_x, T* s_sc, T* s_tau, T* s_beta, T* Tg) {
    if (mt <= 64) factor_tile_rows<T, 1, NB>(s_tile, mt, nbk, s_x, s_sc, s_tau, s_beta, Tg);
    else if (mt <= 128) factor_tile_rows<T, 2, NB>(s_tile, mt, nbk, s_x, s_sc, s_tau, s_beta, Tg);
    else factor_tile_rows<T, 4, NB>(s_tile, mt, nbk, s_x, s_sc, s_tau, s_beta, Tg);
}

// LDS of one panel workgroup: the node tile (column-major, stride
// MT_MAX + 1), the published column (two steps in flight), the step scalars
// and the reflector scalars.
template <typename T> struct PanelSmem {
    T* tile;
    T* x;
    T* sc;
    T* tau;
    T* beta;
};

// Internal node `node` at tree level `level` (>= 1), whose nch children are
// factored: their stacked upper-triangular R factors are factored in place,
// its T goes to the T buffer, its explicit reflectors to the internal
// reflector buffer and its R into the first child's top rows.
template <typename T, int NBW>
__device__ __forceinline__ void panel_internal_node(const QrDesc<T>& d, const RawBuf<T>& bw,
                                                    const TreeGeomT<T, NBW>& g, int c0, int mp, int nbk, int level,
                                                    int node, int nch, const PanelSmem<T>& sm) {
    using C = QrCfg<T, NBW>;
    constexpr int NB = C::NB, LDT = C::MT_MAX + 1;
    T* const s_tile = sm.tile;
    const int tid = threadIdx.x;
    const int ld = d.ld;
    const int par = (c0 / NB) & 1;
    const int iidx = internal_index(g, level, node);
    const int mt = nch * NB;
    // stacked upper-triangular R factors of the children (row s of the
    // stack is row s % NB of child s / NB)
    {
        const int s = tid, t = s / NB, r = s % NB;
        const int rb = s < mt ? c0 + leaf_lo((node * C::F + t) * g.pw(level - 1), mp, g.L(0)) : 0;
        const unsigned vo = s < mt ? (unsigned)((rb + r) * sizeof(T)) : kOob;
        T v[NB];
#pragma unroll
        for (int col = 0; col < NB; ++col) {
            const T x = bw.load(vo + (unsigned)(col * ld * sizeof(T)));
            v[col] = r <= col ? x : T(0);
        }
#pragma unroll
        for (int col = 0; col < NB; ++col) s_tile[col * LDT + s] = v[col];
    }
    __syncthreads();
    factor_node<T, NBW>(s_tile, mt, nbk, sm.x, sm.sc, sm.tau, sm.beta,
                        (par ? d.Tm[1] : d.Tm[0]) + (size_t)node_index(g, level, node, d.tm_leaves) * NB * NB);
    // explicit reflectors of this node, and its R into the top rows
    const RawBuf<T> bvi((par ? d.Vint[1] : d.Vint[0]) + (size_t)iidx * C::MT_MAX * NB,
                        (unsigned)(C::MT_MAX * NB * sizeof(T)));
    const int rbase = c0 + leaf_lo(node * g.pw(level), mp, g.L(0));
    {
        const int s = tid;
#pragma unroll
        for (int col = 0; col < NB; ++col) {
            const T x = s_tile[col * LDT + s];
            const T v = (s < mt && col < nbk) ? (s > col ? x : (s == col ? T(1) : T(0))) : T(0);
            bvi.store(v, (unsigned)((col * C::MT_MAX + s) * sizeof(T)));
            // R: the upper triangle into the first child's top rows
            if (s < NB) bw.store(x, s <= col ? (unsigned)(((size_t)col * ld + rbase + s) * sizeof(T)) : kOob);
        }
    }
}

// Climb from a node factored by this workgroup at `level`: the last child
// to arrive at each parent (counted with an atomic) factors it; the
// workgroup that factors the root writes the diagonal of R.
template <typename T, int NBW>
__device__ __forceinline__ void panel_climb(const QrDesc<T>& d, const RawBuf<T>& bw, const TreeGeomT<T, NBW>& g,
                                            int c0, int mp, int nbk, int level, int node, const PanelSmem<T>& sm,
                                            int* s_last) {
    using C = QrCfg<T, NBW>;
    const int tid = threadIdx.x;
    for (++level; level < g.levels; ++level) {
        __threadfence();
        __syncthreads();
        const int parent = node / C::F;
        const int iidx = internal_index(g, level, parent);
        const int nch = min(C::F, g.L(level - 1) - parent * C::F);
        if (tid == 0) {
            const unsigned old = atomicAdd(&d.counters[iidx], 1u);
            *s_last = (old == (unsigned)(nch - 1));
            if (*s_last) d.counters[iidx] = 0u;
        }
        __syncthreads();
        if (!*s_last) return;
        __threadfence();
        node = parent;
        panel_internal_node<T, NBW>(d, bw, g, c0, mp, nbk, level, node, nch, sm);
    }
    if (tid < nbk) d.diag[c0 + tid] = sm.beta[tid];
}

// Panel factorization of columns [c0, c0 + NB): one workgroup per leaf
// (blockIdx.x) and problem (blockIdx.y).  With leaves_only set and a tree of
// more than one level, the workgroups stop after their leaves and the
// levels above are left to the leaf-level trailing update's launch
// (k_update with CLIMB), which factors them beside the update.
template <typename T, int NBW>
__global__ __launch_bounds__(256) void k_panel(const QrDesc<T>* __restrict__ descs, int c0, int leaves_only) {
    using C = QrCfg<T, NBW>;
    constexpr int NB = C::NB, LDT = C::MT_MAX + 1, PT = C::PT;
    __shared__ T s_tile[LDT * NB];
    __shared__ T s_x[2 * C::MT_MAX];  // published column, two steps in flight
    __shared__ T s_sc[4];
    __shared__ T s_tau[NB], s_beta[NB];
    __shared__ int s_last;
    const PanelSmem<T> sm{s_tile, s_x, s_sc, s_tau, s_beta};

    const QrDesc<T> d = descs[blockIdx.y];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(NB, d.nf - c0);
    const int mp = d.m - c0;
    const auto g = tree_geom<T, NBW>(mp);
    const int node = blockIdx.x;
    if (node >= g.L(0)) return;
    const int par = (c0 / NB) & 1;
    T* const Tm = (par ? d.Tm[1] : d.Tm[0]);
    const int tid = threadIdx.x;
    const int ld = d.ld;
    static_assert(C::MT_MAX <= PT, "one node row per thread");
    // the panel's columns as a raw buffer (reads outside it give zero,
    // writes there are dropped: no branches for the columns >= nbk or the
    // rows beyond a node)
    const RawBuf<T> bw(d.W + (size_t)c0 * ld, (unsigned)(nbk * ld * sizeof(T)));

    // ---- leaf: rows [row0, row0 + mt) of the panel columns
    // Each thread moves one whole row (all NB columns), so its global
    // accesses are independent and in flight together; across threads every
    // column access is a contiguous run of rows.
    const int row0 = c0 + leaf_lo(node, mp, g.L(0));
    const int mt = c0 + leaf_lo(node + 1, mp, g.L(0)) - row0;
    {
        const unsigned vo = tid < mt ? (unsigned)((row0 + tid) * sizeof(T)) : kOob;
        T v[NB];
#pragma unroll
        for (int col = 0; col < NB; ++col) v[col] = bw.load(vo + (unsigned)(col * ld * sizeof(T)));
#pragma unroll
        for (int col = 0; col < NB; ++col) s_tile[col * LDT + tid] = v[col];
        __syncthreads();
        factor_node<T, NBW>(s_tile, mt, nbk, s_x, s_sc, s_tau, s_beta,
                            Tm + (size_t)node_index(g, 0, node, d.tm_leaves) * NB * NB);
#pragma unroll
        for (int col = 0; col < NB; ++col) bw.store(s_tile[col * LDT + tid], vo + (unsigned)(col * ld * sizeof(T)));
    }
    if (leaves_only && g.levels > 1) return;
    // ---- climb the tree: the last child to arrive factors the parent
    panel_climb<T, NBW>(d, bw, g, c0, mp, nbk, 0, node, sm, &s_last);
}

// The climbing role of k_update (climb set): level-1 node `node` of problem
// descs[z], then the levels above it.  Not inlined, so that its registers
// are allocated apart from the trailing update's (which uses the whole
// budget of two workgroups per CU).
template <typename T>
__device__ __noinline__ void panel_tree_from_level1(const QrDesc<T>* __restrict__ descs, int z, int c0, int node,
                                                    T* s_v, T* s_xs, int* s_i) {
    using C = QrCfg<T, 32>;
    const QrDesc<T> d = descs[z];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(C::NB, d.nf - c0);
    const int mp = d.m - c0;
    const auto g = tree_geom<T, 32>(mp);
    if (g.levels < 2 || node >= g.L(1)) return;
    // the node tile in the update's reflector array, the rest in its staging
    // tiles
    const PanelSmem<T> sm{s_v, s_xs, s_xs + 2 * C::MT_MAX, s_xs + 2 * C::MT_MAX + 4, s_xs + 2 * C::MT_MAX + 4 + C::NB};
    const RawBuf<T> bw(d.W + (size_t)c0 * d.ld, (unsigned)(nbk * d.ld * sizeof(T)));
    panel_internal_node<T, 32>(d, bw, g, c0, mp, nbk, 1, node, min(C::F, g.L(0) - node * C::F), sm);
    panel_climb<T, 32>(d, bw, g, c0, mp, nbk, 1, node, sm, s_i);
}

// Apply the transpose of one tree level's block reflectors to a 64-column
// tile of the trailing matrix: C <- C - V (T^T (V^T C)) for the node's rows.
//
// Each wave owns 16 columns and keeps its slice of C in registers in the
// accumulator layout of C^T (MFMA 16x16x4): in row block rb, lane (gq, ln)
// holds column row(gq, v) and row 16 rb + ln, so every global load and store
// instruction moves whole runs of 16 consecutive rows of a few columns.
//   W = V^T C   : B operand = C, re-read from a per-wave 16x16 LDS tile
//                 (rows on the lane group, columns on the lane);
//   Y = T^T W   : W's accumulator registers are the B operand (k-slices
//                 {row(gq, v) : gq});
//   C^T -= Y^T V^T : Y's accumulator registers are the A operand with the
//                 same k-slices, V^T read from LDS, C^T accumulated in place.
// Row blocks per group of the update phase of k_update (1, 2 and 4 were
// measured; 2 was fastest, 1 spills)
constexpr int kUpdGroup = 2;
// One workgroup's share of k_update: node `node` of tree level `level`
// applied to trailing column tile `tile` of problem d.
// With CLIMB (leaf level only), the workgroups of blockIdx.y = 0 factor
// the panel's tree above its leaves instead (level-1 node blockIdx.x, then
// the levels above; k_panel ran with leaves_only) and blockIdx.y = t + 1
// updates column tile t.  The two touch disjoint data: the update reads the
// leaves' reflectors below their diagonals and the leaves' T factors and
// writes only trailing columns; the climb reads and writes the upper
// triangles of the leaves' top rows, the internal nodes' T factors and
// reflectors and the tree counters.  The climb works in this kernel's LDS
// arrays, so two workgroups still fit a CU.
template <typename T, int RB, bool CLIMB>
__global__ __launch_bounds__(256, (sizeof(T) == 4 && CLIMB) ? 3 : 2) void k_update(const QrDesc<T>* __restrict__ descs, int c0, int level) {
    using C = QrCfg<T, 32>;
    using M = Mfma<T>;
    typedef typename M::v4 v4;
    constexpr int NB = C::NB, VS = NB + 1, XS = 17;  // odd strides: conflict-free LDS access
    __shared__ T s_V[RB * 16 * VS];
    __shared__ T s_X[4 * 16 * XS];
    __shared__ int s_rb[32];
    static_assert((C::MT_MAX + 1) * C::NB <= RB * 16 * VS && 2 * C::MT_MAX + 4 + 2 * C::NB <= 4 * 16 * XS,
                  "the panel's LDS fits the update's");
    if constexpr (CLIMB) {
        if (blockIdx.y == 0) {
            panel_tree_from_level1<T>(descs, blockIdx.z, c0, blockIdx.x, s_V, s_X, s_rb);
            return;
        }
    }

    const QrDesc<T> d = descs[blockIdx.z];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(NB, d.nf - c0);
    // column range: the trailing columns after those of the row-split kernel
    const int cb = c0 + nbk + row_split_cols(NB, d.nf, c0, d.la_min);
    const int ce = d.ncols;
    const int col0 = cb + (blockIdx.y - (CLIMB ? 1 : 0)) * 64;
    if (col0 >= ce) return;
    const int par = (c0 / NB) & 1;
    const int mp = d.m - c0;
    const auto g = tree_geom<T, 32>(mp);
    if (level >= g.levels) return;
    const int node = blockIdx.x;
    if (node >= g.L(level)) return;
    const int tid = threadIdx.x;
    const size_t ld = (size_t)d.ld;
    T* W = d.W;

    int mt, lo = 0;
    if (level == 0) {
        lo = c0 + leaf_lo(node, mp, g.L(0));
        mt = c0 + leaf_lo(node + 1, mp, g.L(0)) - lo;
    } else {
        const int nch = min(C::F, g.L(level - 1) - node * C::F);
        mt = nch * NB;
        if (tid < nch) s_rb[tid] = c0 + leaf_lo((node * C::F + tid) * g.pw(level - 1), mp, g.L(0));
        __syncthreads();
    }
    const int rows_pad = ((mt + 15) >> 4) << 4;
    const int wave = tid >> 6, lane = tid & 63, gq = lane >> 4, ln = lane & 15;
    const int cbase = col0 + wave * 16;
    // FP32 leaf level: the node's rows are taken in row-block pairs (rows
    // 32 p + 2 j and 32 p + 2 j + 1 at position j of blocks 2 p and 2 p + 1),
    // so that a lane moves both with one 8-byte access, whole 128-byte lines
    // per column as in FP64; the reflectors are staged with the same
    // permutation (the sum over rows only changes its order).  Only nodes of
    // even height (every leaf but possibly the last of an odd-height panel),
    // so that a pair's rows are both in the node or both out of it.
    const bool pair = sizeof(T) == 4 && level == 0 && (mt & 1) == 0;
    const int rbe = pair ? ((mt + 31) >> 5) * 2 : rows_pad >> 4;
    // Global traffic goes through raw buffers (reads outside a range give
    // zero, writes there are dropped), so it has no branches: the compiler
    // counts the loads exactly and each consumer waits only for its own
    // data.  The C slice streams in while the reflectors go to LDS and while
    // the first row blocks are multiplied.
    // Reflectors: thread s holds row s of the node (explicit: unit diagonal,
    // zero above it and beyond the node).
    static_assert(C::MT_MAX <= 256, "one reflector row per thread");
    const int s = tid;
    T v[NB];
    if (level == 0) {
        const RawBuf<T> bv(W + (size_t)c0 * ld, (unsigned)(nbk * ld * sizeof(T)));
        const unsigned vo = s < mt ? (unsigned)((lo + s) * sizeof(T)) : kOob;
#pragma unroll
        for (int col = 0; col < NB; ++col) {
            const T x = bv.load(vo + (unsigned)(col * ld * sizeof(T)));
            v[col] = s > col ? x : ((s == col && s < mt && col < nbk) ? T(1) : T(0));
        }
    } else {
        const T* Vi = (par ? d.Vint[1] : d.Vint[0]) + (size_t)internal_index(g, level, node) * C::MT_MAX * NB;
        const RawBuf<T> bv(Vi, (unsigned)(nbk * C::MT_MAX * sizeof(T)));
        const unsigned vo = s < mt ? (unsigned)(s * sizeof(T)) : kOob;
#pragma unroll
        for (int col = 0; col < NB; ++col) v[col] = bv.load(vo + (unsigned)(col * C::MT_MAX * sizeof(T)));
    }
    // C^T slice: row block rb, lane (gq, ln), register q <-> node row 16 rb + ln,
    // column cbase + row(gq, q) (row(g, q) = row(g, 0) + row(0, q)); the
    // wave's buffer covers its valid columns only.  The first half of the
    // row blocks is requested before the reflectors go to LDS, the second
    // half after (registers: the reflector row and half the slice).
    const RawBuf<T> bc(W + (size_t)cbase * ld, (unsigned)(max(0, min(16, ce - cbase)) * ld * sizeof(T)));
    auto c_off = [&](int rb) -> unsigned {
        const int sr = rb * 16 + ln;
        const int wr = (rb >= rbe || sr >= mt) ? -1
                       : level == 0 ? lo + sr
                       : ((sr & (NB - 1)) < nbk ? s_rb[sr / NB] + (sr & (NB - 1)) : -1);
        return wr >= 0 ? (unsigned)((M::row(gq, 0) * ld + wr) * sizeof(T)) : kOob;
    };
    // the pair (2 p, 2 p + 1) of the FP32 leaf level: rows lo + 32 p + 2 ln
    // and the next (the height is even, so both or neither are in the node)
    auto c_off2 = [&](int p) -> unsigned {
        const int sr = p * 32 + 2 * ln;
        return 2 * p < rbe && sr < mt ? (unsigned)((M::row(gq, 0) * ld + lo + sr) * sizeof(T)) : kOob;
    };
    v4 cr[RB];
    if constexpr (sizeof(T) == 4) {
        auto load_half = [&](int rb0) {
            if (pair) {
#pragma unroll
                for (int p = rb0 / 2; p < (rb0 + RB / 2) / 2; ++p) {
                    const unsigned o = c_off2(p);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const auto x = bc.load2(o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
                        cr[2 * p][q] = x[0];
                        cr[2 * p + 1][q] = x[1];
                    }
                }
            } else {
#pragma unroll
                for (int rb = rb0; rb < rb0 + RB / 2; ++rb) {
                    const unsigned o = c_off(rb);
#pragma unroll
                    for (int q = 0; q < 4; ++q) cr[rb][q] = bc.load(o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
                }
            }
        };
        load_half(0);
        // every row of s_V (zero beyond the node), without a branch; in pair
        // mode row s goes to position (s mod 32) / 2 of block 2 (s / 32) + s mod 2
        const int sv = pair ? ((s >> 5) * 2 + (s & 1)) * 16 + ((s & 31) >> 1) : s;
#pragma unroll
        for (int col = 0; col < NB; ++col) s_V[sv * VS + col] = v[col];
        __syncthreads();
        load_half(RB / 2);
    } else {
#pragma unroll
        for (int rb = 0; rb < RB / 2; ++rb) {
            const unsigned o = c_off(rb);
#pragma unroll
            for (int q = 0; q < 4; ++q) cr[rb][q] = bc.load(o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
        }
        // every row of s_V (zero beyond the node), without a branch
#pragma unroll
        for (int col = 0; col < NB; ++col) s_V[s * VS + col] = v[col];
        __syncthreads();
#pragma unroll
        for (int rb = RB / 2; rb < RB; ++rb) {
            const unsigned o = c_off(rb);
#pragma unroll
            for (int q = 0; q < 4; ++q) cr[rb][q] = bc.load(o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
        }
    }
    // T factor of this node, as the A operand of Y = T^T W: lane (gq, ln)
    // needs T[k][ln] for k = kb * 16 + row(gq, j); through a buffer (a
    // generic-pointer load would be a flat access, which the wait counters
    // cannot tell apart from the LDS traffic).
    const RawBuf<T> bt((par ? d.Tm[1] : d.Tm[0]) + (size_t)node_index(g, level, node, d.tm_leaves) * NB * NB,
                       (unsigned)(NB * NB * sizeof(T)));
    T ta[2][2][4];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kb * 16 + M::row(gq, j);
            ta[0][kb][j] = bt.load((unsigned)((ln * NB + k) * sizeof(T)));
            ta[1][kb][j] = bt.load((unsigned)(((16 + ln) * NB + k) * sizeof(T)));
        }

    // W = V^T C (NB x 16): per row block, C goes through the wave's LDS tile
    // into the B-operand layout.  Software pipelined: the LDS traffic of row
    // block rb + 1 (tile write, operand reads) is issued before the MFMAs of
    // rb.  A wave's LDS operations complete in issue order, so the tile can be
    // rewritten after the previous block's reads without a barrier.  Two
    // accumulator chains per half (even / odd row blocks).
    T* X = s_X + wave * 16 * XS;
    v4 w0 = v4{0, 0, 0, 0}, w1 = v4{0, 0, 0, 0}, w2 = v4{0, 0, 0, 0}, w3 = v4{0, 0, 0, 0};
    T ob[2][4], ova[2][4], ovb[2][4];
#define SDC_STAGE_W(RBI, BUF)                                                     \
    {                                                                             \
        _Pragma("unroll") for (int v = 0; v < 4; ++v) X[ln * XS + M::row(gq, v)] = cr[RBI][v]; \
        _Pragma("unroll") for (int kk = 0; kk < 4; ++kk) {                        \
            ob[BUF][kk] = X[(4 * kk + gq) * XS + ln];                             \
            const T* vr = s_V + ((RBI) * 16 + 4 * kk + gq) * VS;                  \
            ova[BUF][kk] = vr[ln];                                                \
            ovb[BUF][kk] = vr[16 + ln];                                           \
        }                                                                         \
    }
    if (rbe > 0) SDC_STAGE_W(0, 0)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        if (rb < rbe) {
            if (rb + 1 < RB && rb + 1 < rbe) SDC_STAGE_W(rb + 1 < RB ? rb + 1 : rb, (rb + 1) & 1)
            __builtin_amdgcn_sched_barrier(0);
            const int bf = rb & 1;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                if (rb & 1) {
                    w2 = M::mma(ova[bf][kk], ob[bf][kk], w2);
                    w3 = M::mma(ovb[bf][kk], ob[bf][kk], w3);
                } else {
                    w0 = M::mma(ova[bf][kk], ob[bf][kk], w0);
                    w1 = M::mma(ovb[bf][kk], ob[bf][kk], w1);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#undef SDC_STAGE_W
    w0 += w2;
    w1 += w3;
    // Y = T^T W
    v4 y0 = v4{0, 0, 0, 0}, y1 = v4{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T bw = kb ? w1[j] : w0[j];
            y0 = M::mma(ta[0][kb][j], bw, y0);
            y1 = M::mma(ta[1][kb][j], bw, y1);
        }
    }
    // C^T -= Y^T V^T, kUpdGroup row blocks at a time (one accumulator chain
    // each over the eight k-steps, in the same k order as a whole-slice
    // pass, so the result does not depend on the grouping); each group is
    // stored as soon as it is done, so its stores drain while later groups
    // are multiplied
    constexpr int G = kUpdGroup;
    static_assert(RB % G == 0, "whole groups of row blocks");
    T ya[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) ya[t] = -((t >> 2) ? y1[t & 3] : y0[t & 3]);
#pragma unroll
    for (int rb = 0; rb < RB; rb += G) {
        if (rb < rbe) {
            T vb[G][8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int kcol = (t >> 2) * 16 + M::row(gq, t & 3);
#pragma unroll
                for (int g = 0; g < G; ++g) vb[g][t] = rb + g < rbe ? s_V[((rb + g) * 16 + ln) * VS + kcol] : T(0);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int g = 0; g < G; ++g) cr[rb + g] = M::mma(ya[t], vb[g][t], cr[rb + g]);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (sizeof(T) == 4) {
                static_assert(G == 2, "a group is one row-block pair");
                if (pair) {
                    const unsigned o = c_off2(rb / 2);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        typename RawBuf<T>::f2 x;
                        x[0] = cr[rb][q];
                        x[1] = cr[rb + 1][q];
                        bc.store2(x, o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const unsigned o = c_off(rb + g);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            bc.store(cr[rb + g][q], o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
                    }
                }
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const unsigned o = c_off(rb + g);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        bc.store(cr[rb + g][q], o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
                }
            }
        }
    }
}

// The trailing update for 64-column panels (twice the flops per byte of
// the trailing matrix: above the FP64 machine balance, so the matrix cores
// bound it).  Same layouts as k_update; the 64 reflector columns go through
// LDS 32 at a time, so that two workgroups still fit a CU:
//   stage V[:, 32:64], W_b = V_b^T C;  stage V[:, 0:32], W_a = V_a^T C;
//   Y = T^T W (T upper triangular: the blocks below its diagonal skipped);
//   C^T -= Y_a^T V_a^T;  stage V[:, 32:64] again, C^T -= Y_b^T V_b^T, store.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_update64(const QrDesc<T>* __restrict__ descs, int c0, int level) {
    using C = QrCfg<T, 64>;
    using M = Mfma<T>;
    typedef typename M::v4 v4;
    constexpr int NB = C::NB, RB = C::MT_MAX / 16, VS = 33, XS = 17, NKB = NB / 16;
    __shared__ T s_V[C::MT_MAX * VS];
    __shared__ T s_X[4 * 16 * XS];
    __shared__ int s_rb[C::F];

    const QrDesc<T> d = descs[blockIdx.z];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(NB, d.nf - c0);
    const int cb = c0 + nbk + row_split_cols(NB, d.nf, c0, d.la_min);
    const int ce = d.ncols;
    const int col0 = cb + blockIdx.y * 64;
    if (col0 >= ce) return;
    const int par = (c0 / NB) & 1;
    const int mp = d.m - c0;
    const auto g = tree_geom<T, NB>(mp);
    if (level >= g.levels) return;
    const int node = blockIdx.x;
    if (node >= g.L(level)) return;
    const int tid = threadIdx.x;
    const size_t ld = (size_t)d.ld;
    T* W = d.W;

    int mt, lo = 0;
    if (level == 0) {
        lo = c0 + leaf_lo(node, mp, g.L(0));
        mt = c0 + leaf_lo(node + 1, mp, g.L(0)) - lo;
    } else {
        const int nch = min(C::F, g.L(level - 1) - node * C::F);
        mt = nch * NB;
        if (tid < nch) s_rb[tid] = c0 + leaf_lo((node * C::F + tid) * g.pw(level - 1), mp, g.L(0));
        __syncthreads();
    }
    const int rbe = (mt + 15) >> 4;
    const int wave = tid >> 6, lane = tid & 63, gq = lane >> 4, ln = lane & 15;
    const int cbase = col0 + wave * 16;
    static_assert(C::MT_MAX <= 256, "one reflector row per thread");
    const int s = tid;
    // reflector columns [32 h, 32 h + 32) into s_V, row s by thread s
    // (explicit: unit diagonal, zero above it and beyond the node)
    auto stage = [&](int h) {
        T v[32];
        if (level == 0) {
            const RawBuf<T> bv(W + (size_t)c0 * ld, (unsigned)(nbk * ld * sizeof(T)));
            const unsigned vo = s < mt ? (unsigned)((lo + s) * sizeof(T)) : kOob;
#pragma unroll
            for (int c = 0; c < 32; ++c) {
                const int col = 32 * h + c;
                const T x = bv.load(vo + (unsigned)(col * ld * sizeof(T)));
                v[c] = s > col ? x : ((s == col && s < mt && col < nbk) ? T(1) : T(0));
            }
        } else {
            const T* Vi = (par ? d.Vint[1] : d.Vint[0]) + (size_t)internal_index(g, level, node) * C::MT_MAX * NB;
            const RawBuf<T> bv(Vi, (unsigned)(nbk * C::MT_MAX * sizeof(T)));
            const unsigned vo = s < mt ? (unsigned)(s * sizeof(T)) : kOob;
#pragma unroll
            for (int c = 0; c < 32; ++c) v[c] = bv.load(vo + (unsigned)((32 * h + c) * C::MT_MAX * sizeof(T)));
        }
#pragma unroll
        for (int c = 0; c < 32; ++c) s_V[s * VS + c] = v[c];
    };
    const RawBuf<T> bc(W + (size_t)cbase * ld, (unsigned)(max(0, min(16, ce - cbase)) * ld * sizeof(T)));
    auto c_off = [&](int rb) -> unsigned {
        const int sr = rb * 16 + ln;
        const int wr = (rb >= rbe || sr >= mt) ? -1
                       : level == 0 ? lo + sr
                       : ((sr & (NB - 1)) < nbk ? s_rb[sr / NB] + (sr & (NB - 1)) : -1);
        return wr >= 0 ? (unsigned)((M::row(gq, 0) * ld + wr) * sizeof(T)) : kOob;
    };
    v4 cr[RB];
#pragma unroll
    for (int rb = 0; rb < RB / 2; ++rb) {
        const unsigned o = c_off(rb);
#pragma unroll
        for (int q = 0; q < 4; ++q) cr[rb][q] = bc.load(o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
    }
    stage(1);
    __syncthreads();
#pragma unroll
    for (int rb = RB / 2; rb < RB; ++rb) {
        const unsigned o = c_off(rb);
#pragma unroll
        for (int q = 0; q < 4; ++q) cr[rb][q] = bc.load(o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
    }
    // W for the staged half h: rows [32 h, 32 h + 32) of W = V^T C (16
    // columns per wave), C through the wave's LDS tile into the B layout
    T* X = s_X + wave * 16 * XS;
    v4 w[NKB];
    auto wphase = [&](int h) {
        v4 a0 = v4{0, 0, 0, 0}, a1 = v4{0, 0, 0, 0};
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            if (rb < rbe) {
                T ob[4], ova[4], ovb[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) X[ln * XS + M::row(gq, v)] = cr[rb][v];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    ob[kk] = X[(4 * kk + gq) * XS + ln];
                    const T* vr = s_V + (rb * 16 + 4 * kk + gq) * VS;
                    ova[kk] = vr[ln];
                    ovb[kk] = vr[16 + ln];
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    a0 = M::mma(ova[kk], ob[kk], a0);
                    a1 = M::mma(ovb[kk], ob[kk], a1);
                }
            }
        }
        w[2 * h] = a0;
        w[2 * h + 1] = a1;
    };
    wphase(1);
    __syncthreads();
    stage(0);
    __syncthreads();
    wphase(0);
    // Y = T^T W: output block o from the k-blocks kb <= o (T[k][m] = 0 for k > m)
    const RawBuf<T> bt((par ? d.Tm[1] : d.Tm[0]) + (size_t)node_index(g, level, node, d.tm_leaves) * NB * NB,
                       (unsigned)(NB * NB * sizeof(T)));
    T ya[NKB][4];
#pragma unroll
    for (int o = 0; o < NKB; ++o) {
        v4 y = v4{0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb <= o; ++kb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kb * 16 + M::row(gq, j);
                y = M::mma(bt.load((unsigned)(((16 * o + ln) * NB + k) * sizeof(T))), w[kb][j], y);
            }
#pragma unroll
        for (int j = 0; j < 4; ++j) ya[o][j] = -y[j];
    }
    // C^T -= Y_h^T V_h^T for the staged half h, two row blocks at a time;
    // the last pass stores each pair as soon as it is done
    auto uphase = [&](int h, bool store) {
#pragma unroll
        for (int rb = 0; rb < RB; rb += 2) {
            if (rb < rbe) {
                T vb[2][8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int kcol = (t >> 2) * 16 + M::row(gq, t & 3);
#pragma unroll
                    for (int g2 = 0; g2 < 2; ++g2)
                        vb[g2][t] = rb + g2 < rbe ? s_V[((rb + g2) * 16 + ln) * VS + kcol] : T(0);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int g2 = 0; g2 < 2; ++g2)
                        cr[rb + g2] = M::mma(ya[2 * h + (t >> 2)][t & 3], vb[g2][t], cr[rb + g2]);
                __builtin_amdgcn_sched_barrier(0);
                if (store) {
#pragma unroll
                    for (int g2 = 0; g2 < 2; ++g2) {
                        const unsigned o = c_off(rb + g2);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            bc.store(cr[rb + g2][q], o + (unsigned)(M::row(0, q) * ld * sizeof(T)));
                    }
                }
            }
        }
    };
    uphase(0, false);
    __syncthreads();
    stage(1);
    __syncthreads();
    uphase(1, true);
}

// Row-split (look-ahead) update: the transpose of panel c0's orthogonal
// factor (every tree level) applied, in one launch, to the next panel's
// columns (row_split_cols).  A workgroup owns one node and one 16-column
// group of them; its four
// waves split the node's rows (row blocks [RBW w, RBW w + RBW) of wave w),
// each forms its share of W = V^T C, the shares are summed through LDS, and
// each wave applies C <- C - V (T^T W) to its rows.  The last workgroup to
// finish among a node's children (counted per column group) goes on to the
// parent, as in the panel factorization, so the tree levels need no further
// launches.  The MFMA layouts are those of k_update.
template <typename T>
__global__ __launch_bounds__(256) void k_la(const QrDesc<T>* __restrict__ descs, int c0) {
    using C = QrCfg<T, 32>;
    using M = Mfma<T>;
    typedef typename M::v4 v4;
    constexpr int NB = C::NB, VS = NB + 1, XS = 17, RBW = C::MT_MAX / 64;
    __shared__ T s_V[C::MT_MAX * VS];
    __shared__ T s_X[4 * 16 * XS];  // per-wave transpose tiles, then the W / Y exchange
    __shared__ int s_rb[C::F];
    __shared__ int s_last;
    static_assert(4 * 16 * XS >= 1024, "exchange space for two 32 x 16 partial sums per lane set");

    const QrDesc<T> d = descs[blockIdx.z];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(NB, d.nf - c0);
    const int cb = c0 + nbk;
    const int ce = cb + row_split_cols(NB, d.nf, c0, d.la_min);
    const int cgrp = blockIdx.y;
    if (ce - cb <= 16 * cgrp) return;  // no columns in this group (for every node alike)
    const int cbase = cb + 16 * cgrp;
    const int mp = d.m - c0;
    const auto g = tree_geom<T, 32>(mp);
    int node = blockIdx.x;
    if (node >= g.L(0)) return;
    // arrival counters of column group cgrp: after the panel factorization's
    // kPanelCounters, one per internal node of this panel's tree
    const int nint = internal_index(g, g.levels, 0);
    const int par = (c0 / NB) & 1;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, gq = lane >> 4, ln = lane & 15;
    const int ld = d.ld;
    T* W = d.W;
    int level = 0;
    const int lo = c0 + leaf_lo(node, mp, g.L(0));
    int mt = c0 + leaf_lo(node + 1, mp, g.L(0)) - lo;
    for (;;) {
        const int rows_pad = ((mt + 15) >> 4) << 4;
        const int rbe = rows_pad >> 4;
        // explicit reflectors of the node (unit diagonal, zero above it and
        // beyond the node), one row per thread
        // (raw buffers: reads outside a range give zero, so no branches and
        // exact wait counts; a generic-pointer load would be a flat access)
        {
            const int s = tid;
            T v[NB];
            if (level == 0) {
                const RawBuf<T> bv(W + (size_t)c0 * ld, (unsigned)(nbk * ld * sizeof(T)));
                const unsigned vo = s < mt ? (unsigned)((lo + s) * sizeof(T)) : kOob;
#pragma unroll
                for (int col = 0; col < NB; ++col) {
                    const T x = bv.load(vo + (unsigned)(col * ld * sizeof(T)));
                    v[col] = s > col ? x : ((s == col && s < mt && col < nbk) ? T(1) : T(0));
                }
            } else {
                const T* Vi = (par ? d.Vint[1] : d.Vint[0]) + (size_t)internal_index(g, level, node) * C::MT_MAX * NB;
                const RawBuf<T> bv(Vi, (unsigned)(nbk * C::MT_MAX * sizeof(T)));
                const unsigned vo = s < mt ? (unsigned)(s * sizeof(T)) : kOob;
#pragma unroll
                for (int col = 0; col < NB; ++col) v[col] = bv.load(vo + (unsigned)(col * C::MT_MAX * sizeof(T)));
            }
#pragma unroll
            for (int col = 0; col < NB; ++col) s_V[s * VS + col] = v[col];
        }
        const RawBuf<T> bt((par ? d.Tm[1] : d.Tm[0]) + (size_t)node_index(g, level, node, d.tm_leaves) * NB * NB,
                           (unsigned)(NB * NB * sizeof(T)));
        T ta[2][2][4];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int k = kb * 16 + M::row(gq, j);
                ta[0][kb][j] = bt.load((unsigned)((ln * NB + k) * sizeof(T)));
                ta[1][kb][j] = bt.load((unsigned)(((16 + ln) * NB + k) * sizeof(T)));
            }
        // this wave's rows of C^T (layout of k_update); the buffer covers the
        // group's valid columns only
        const RawBuf<T> bc(W + (size_t)cbase * ld, (unsigned)(max(0, min(16, ce - cbase)) * ld * sizeof(T)));
        unsigned co[RBW];
        v4 cr[RBW];
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
            const int rb = wave * RBW + i;
            const int sr = rb * 16 + ln;
            const int wr = (rb >= rbe || sr >= mt) ? -1
                           : level == 0 ? lo + sr
                           : ((sr & (NB - 1)) < nbk ? s_rb[sr / NB] + (sr & (NB - 1)) : -1);
            co[i] = wr >= 0 ? (unsigned)((M::row(gq, 0) * ld + wr) * sizeof(T)) : kOob;
#pragma unroll
            for (int q = 0; q < 4; ++q) cr[i][q] = bc.load(co[i] + (unsigned)(M::row(0, q) * ld * sizeof(T)));
        }
        __syncthreads();  // s_V complete
        // this wave's share of W = V^T C (rows: V's columns; two accumulator
        // chains per half)
        T* X = s_X + wave * 16 * XS;
        v4 w0 = v4{0, 0, 0, 0}, w1 = v4{0, 0, 0, 0}, w2 = v4{0, 0, 0, 0}, w3 = v4{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
            const int rb = wave * RBW + i;
            if (rb < rbe) {
                T ob[4], ova[4], ovb[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) X[ln * XS + M::row(gq, v)] = cr[i][v];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    ob[kk] = X[(4 * kk + gq) * XS + ln];
                    const T* vr = s_V + (rb * 16 + 4 * kk + gq) * VS;
                    ova[kk] = vr[ln];
                    ovb[kk] = vr[16 + ln];
                }
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    if (i & 1) {
                        w2 = M::mma(ova[kk], ob[kk], w2);
                        w3 = M::mma(ovb[kk], ob[kk], w3);
                    } else {
                        w0 = M::mma(ova[kk], ob[kk], w0);
                        w1 = M::mma(ovb[kk], ob[kk], w1);
                    }
                }
            }
        }
        w0 += w2;
        w1 += w3;
        // sum of the four shares, (P0 + P2) + (P1 + P3), then Y = T^T W by
        // wave 0, handed to every wave
        T* E = s_X;
        __syncthreads();  // transpose tiles free
        if (wave >= 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                E[(wave - 2) * 512 + lane * 8 + v] = w0[v];
                E[(wave - 2) * 512 + lane * 8 + 4 + v] = w1[v];
            }
        }
        __syncthreads();
        if (wave < 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                w0[v] += E[wave * 512 + lane * 8 + v];
                w1[v] += E[wave * 512 + lane * 8 + 4 + v];
            }
        }
        __syncthreads();
        if (wave == 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                E[lane * 8 + v] = w0[v];
                E[lane * 8 + 4 + v] = w1[v];
            }
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                w0[v] += E[lane * 8 + v];
                w1[v] += E[lane * 8 + 4 + v];
            }
            v4 y0 = v4{0, 0, 0, 0}, y1 = v4{0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const T bw = kb ? w1[j] : w0[j];
                    y0 = M::mma(ta[0][kb][j], bw, y0);
                    y1 = M::mma(ta[1][kb][j], bw, y1);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                E[512 + lane * 8 + v] = y0[v];
                E[512 + lane * 8 + 4 + v] = y1[v];
            }
        }
        __syncthreads();
        T yv[2][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            yv[0][v] = E[512 + lane * 8 + v];
            yv[1][v] = E[512 + lane * 8 + 4 + v];
        }
        // C^T -= Y^T V^T on this wave's rows
#pragma unroll
        for (int pb = 0; pb < 2; ++pb) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T a = -yv[pb][j];
                const int kcol = pb * 16 + M::row(gq, j);
                T vb[RBW];
#pragma unroll
                for (int i = 0; i < RBW; ++i) {
                    const int rb = wave * RBW + i;
                    vb[i] = rb < rbe ? s_V[(rb * 16 + ln) * VS + kcol] : T(0);
                }
#pragma unroll
                for (int i = 0; i < RBW; ++i)
                    if (wave * RBW + i < rbe) cr[i] = M::mma(a, vb[i], cr[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < RBW; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) bc.store(cr[i][q], co[i] + (unsigned)(M::row(0, q) * ld * sizeof(T)));
        // climb: the last child to arrive updates the parent's rows
        if (level + 1 >= g.levels) return;
        __threadfence();
        __syncthreads();
        const int parent = node / C::F;
        const int iidx = internal_index(g, level + 1, parent);
        const int nch = min(C::F, g.L(level) - parent * C::F);
        if (tid == 0) {
            unsigned* cnt = d.counters + kPanelCounters + cgrp * nint + iidx;
            const unsigned old = atomicAdd(cnt, 1u);
            s_last = (old == (unsigned)(nch - 1));
            if (s_last) *cnt = 0u;
        }
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        node = parent;
        ++level;
        mt = nch * NB;
        if (tid < nch) s_rb[tid] = c0 + leaf_lo((node * C::F + tid) * g.pw(level - 1), mp, g.L(0));
        __syncthreads();
    }
}

// Row-split (look-ahead) update for 64-column panels: as k_la, with the
// node's 64 reflector columns in LDS at once (one workgroup per CU), W in
// four 16-row blocks, and Y = T^T W formed one 16-row block per wave
// (T upper triangular: the blocks below its diagonal skipped).
template <typename T>
__global__ __launch_bounds__(256) void k_la64(const QrDesc<T>* __restrict__ descs, int c0) {
    using C = QrCfg<T, 64>;
    using M = Mfma<T>;
    typedef typename M::v4 v4;
    constexpr int NB = C::NB, VS = NB + 1, XS = 17, RBW = C::MT_MAX / 64, NKB = NB / 16;
    constexpr int SH = 64 * 4 * NKB;  // one wave's W (or all of Y) in the exchange buffer
    __shared__ T s_V[C::MT_MAX * VS];
    __shared__ T s_X[4 * 16 * XS];
    __shared__ T s_E[2 * SH];
    __shared__ int s_rb[C::F];
    __shared__ int s_last;

    const QrDesc<T> d = descs[blockIdx.z];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(NB, d.nf - c0);
    const int cb = c0 + nbk;
    const int ce = cb + row_split_cols(NB, d.nf, c0, d.la_min);
    const int cgrp = blockIdx.y;
    if (ce - cb <= 16 * cgrp) return;  // no columns in this group (for every node alike)
    const int cbase = cb + 16 * cgrp;
    const int mp = d.m - c0;
    const auto g = tree_geom<T, NB>(mp);
    int node = blockIdx.x;
    if (node >= g.L(0)) return;
    const int nint = internal_index(g, g.levels, 0);
    const int par = (c0 / NB) & 1;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, gq = lane >> 4, ln = lane & 15;
    const int ld = d.ld;
    T* W = d.W;
    int level = 0;
    const int lo = c0 + leaf_lo(node, mp, g.L(0));
    int mt = c0 + leaf_lo(node + 1, mp, g.L(0)) - lo;
    for (;;) {
        const int rbe = (mt + 15) >> 4;
        // explicit reflectors of the node, one row per thread, 32 columns at a time
        {
            const int s = tid;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                T v[32];
                if (level == 0) {
                    const RawBuf<T> bv(W + (size_t)c0 * ld, (unsigned)(nbk * ld * sizeof(T)));
                    const unsigned vo = s < mt ? (unsigned)((lo + s) * sizeof(T)) : kOob;
#pragma unroll
                    for (int c = 0; c < 32; ++c) {
                        const int col = 32 * h + c;
                        const T x = bv.load(vo + (unsigned)(col * ld * sizeof(T)));
                        v[c] = s > col ? x : ((s == col && s < mt && col < nbk) ? T(1) : T(0));
                    }
                } else {
                    const T* Vi =
                        (par ? d.Vint[1] : d.Vint[0]) + (size_t)internal_index(g, level, node) * C::MT_MAX * NB;
                    const RawBuf<T> bv(Vi, (unsigned)(nbk * C::MT_MAX * sizeof(T)));
                    const unsigned vo = s < mt ? (unsigned)(s * sizeof(T)) : kOob;
#pragma unroll
                    for (int c = 0; c < 32; ++c)
                        v[c] = bv.load(vo + (unsigned)((32 * h + c) * C::MT_MAX * sizeof(T)));
                }
#pragma unroll
                for (int c = 0; c < 32; ++c) s_V[s * VS + 32 * h + c] = v[c];
            }
        }
        // this wave's rows of C^T (layout of k_update); the buffer covers the
        // group's valid columns only
        const RawBuf<T> bc(W + (size_t)cbase * ld, (unsigned)(max(0, min(16, ce - cbase)) * ld * sizeof(T)));
        unsigned co[RBW];
        v4 cr[RBW];
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
            const int rb = wave * RBW + i;
            const int sr = rb * 16 + ln;
            const int wr = (rb >= rbe || sr >= mt) ? -1
                           : level == 0 ? lo + sr
                           : ((sr & (NB - 1)) < nbk ? s_rb[sr / NB] + (sr & (NB - 1)) : -1);
            co[i] = wr >= 0 ? (unsigned)((M::row(gq, 0) * ld + wr) * sizeof(T)) : kOob;
#pragma unroll
            for (int q = 0; q < 4; ++q) cr[i][q] = bc.load(co[i] + (unsigned)(M::row(0, q) * ld * sizeof(T)));
        }
        __syncthreads();  // s_V complete
        // this wave's share of W = V^T C
        T* X = s_X + wave * 16 * XS;
        v4 w[NKB];
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) w[kb] = v4{0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < RBW; ++i) {
            const int rb = wave * RBW + i;
            if (rb < rbe) {
                T ob[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) X[ln * XS + M::row(gq, v)] = cr[i][v];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) ob[kk] = X[(4 * kk + gq) * XS + ln];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const T* vr = s_V + (rb * 16 + 4 * kk + gq) * VS;
#pragma unroll
                    for (int kb = 0; kb < NKB; ++kb) w[kb] = M::mma(vr[16 * kb + ln], ob[kk], w[kb]);
                }
            }
        }
        // sum of the four shares, (P0 + P2) + (P1 + P3), in every wave
        if (wave >= 2) {
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                for (int v = 0; v < 4; ++v) s_E[(wave - 2) * SH + lane * 4 * NKB + 4 * kb + v] = w[kb][v];
        }
        __syncthreads();
        if (wave < 2) {
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                for (int v = 0; v < 4; ++v) w[kb][v] += s_E[wave * SH + lane * 4 * NKB + 4 * kb + v];
        }
        __syncthreads();
        if (wave == 1) {
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                for (int v = 0; v < 4; ++v) s_E[lane * 4 * NKB + 4 * kb + v] = w[kb][v];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    w[kb][v] += s_E[lane * 4 * NKB + 4 * kb + v];
                    s_E[SH + lane * 4 * NKB + 4 * kb + v] = w[kb][v];
                }
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
            for (int v = 0; v < 4; ++v) w[kb][v] = s_E[SH + lane * 4 * NKB + 4 * kb + v];
        // Y block o = wave (rows [16 o, 16 o + 16) of Y = T^T W)
        const RawBuf<T> bt((par ? d.Tm[1] : d.Tm[0]) + (size_t)node_index(g, level, node, d.tm_leaves) * NB * NB,
                           (unsigned)(NB * NB * sizeof(T)));
        v4 y = v4{0, 0, 0, 0};
        const int wu = __builtin_amdgcn_readfirstlane(wave);  // wave-uniform
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
            if (kb <= wu) {
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = kb * 16 + M::row(gq, j);
                    y = M::mma(bt.load((unsigned)(((16 * wave + ln) * NB + k) * sizeof(T))), w[kb][j], y);
                }
            }
        __syncthreads();  // every wave has read W
#pragma unroll
        for (int v = 0; v < 4; ++v) s_E[wave * 256 + lane * 4 + v] = y[v];
        __syncthreads();
        T yv[NKB][4];
#pragma unroll
        for (int o = 0; o < NKB; ++o)
#pragma unroll
            for (int v = 0; v < 4; ++v) yv[o][v] = s_E[o * 256 + lane * 4 + v];
        // C^T -= Y^T V^T on this wave's rows
#pragma unroll
        for (int pb = 0; pb < NKB; ++pb) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T a = -yv[pb][j];
                const int kcol = pb * 16 + M::row(gq, j);
                T vb[RBW];
#pragma unroll
                for (int i = 0; i < RBW; ++i) {
                    const int rb = wave * RBW + i;
                    vb[i] = rb < rbe ? s_V[(rb * 16 + ln) * VS + kcol] : T(0);
                }
#pragma unroll
                for (int i = 0; i < RBW; ++i)
                    if (wave * RBW + i < rbe) cr[i] = M::mma(a, vb[i], cr[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < RBW; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) bc.store(cr[i][q], co[i] + (unsigned)(M::row(0, q) * ld * sizeof(T)));
        // climb: the last child to arrive updates the parent's rows
        if (level + 1 >= g.levels) return;
        __threadfence();
        __syncthreads();
        const int parent = node / C::F;
        const int iidx = internal_index(g, level + 1, parent);
        const int nch = min(C::F, g.L(level) - parent * C::F);
        if (tid == 0) {
            unsigned* cnt = d.counters + kPanelCounters + cgrp * nint + iidx;
            const unsigned old = atomicAdd(cnt, 1u);
            s_last = (old == (unsigned)(nch - 1));
            if (s_last) *cnt = 0u;
        }
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        node = parent;
        ++level;
        mt = nch * NB;
        if (tid < nch) s_rb[tid] = c0 + leaf_lo((node * C::F + tid) * g.pw(level - 1), mp, g.L(0));
        __syncthreads();
    }
}

template <typename T, int NBW>
static void launch_update(dim3 grid, hipStream_t s, const QrDesc<T>* d, int c0, int lev) {
    if constexpr (NBW == 64) {
        hipLaunchKernelGGL(k_update64<T>, grid, dim3(256), 0, s, d, c0, lev);
    } else {
        constexpr int RB = QrCfg<T, 32>::MT_MAX / 16;
        hipLaunchKernelGGL((k_update<T, RB, false>), grid, dim3(256), 0, s, d, c0, lev);
    }
}
template <typename T, int NBW>
static void launch_la(dim3 grid, hipStream_t s, const QrDesc<T>* d, int c0) {
    if constexpr (NBW == 64) hipLaunchKernelGGL(k_la64<T>, grid, dim3(256), 0, s, d, c0);
    else hipLaunchKernelGGL(k_la<T>, grid, dim3(256), 0, s, d, c0);
}

// Batched augmented QR, panel by panel: panel factorization P(k), then the
// update of the trailing columns, split per problem (row_split_cols) between
// the row-split kernel (LA(k)) and the wide kernel's tree levels (REST(k)).
// Without `la` every step runs on s.  With `la` (look-ahead, depth 1), when
// every problem's next panel is in LA(k), panel k+1 is factored while REST(k)
// runs on the second stream:
//   crit: P(k), [wait REST(k-1)], LA(k), P(k+1) ...
//   rest: [wait LA(k)], REST(k)
// so P(k+1) runs beside REST(k) and LA(k) runs alone (it is short, and a
// small grid queued behind a large one is dispatched only after it).
// LA(k) must follow REST(k-1) (both touch panel k+1's columns); P(k+1)
// writes the other parity's T / reflector buffers while REST(k) reads
// panel k's.  crit starts after the work already on s, and s waits for both
// streams before returning.
// With tree_overlap, a 32-column panel of more than one tree level and no
// LA part runs as: the leaves of P(k) (k_panel, leaves_only), then one
// launch with the rest of P(k)'s tree beside REST(k)'s leaf level
// (k_update with CLIMB), then REST(k)'s upper levels.
template <typename T, int NBW>
static void qr_aug_batch_nb(const QrDesc<T>* d_descs, const QrDesc<T>* h, int count, hipStream_t s,
                            const QrStreams* la, bool tree_overlap) {
    using C = QrCfg<T, NBW>;
    int max_nf = 0;
    for (int i = 0; i < count; ++i)
        if (h[i].active) max_nf = max_nf > h[i].nf ? max_nf : h[i].nf;
    bool rest_pending = false;
    hipStream_t sc = s;  // critical-path stream
    if (la) {
        (void)hipEventRecord(la->evE, s);
        (void)hipStreamWaitEvent(la->crit, la->evE, 0);
        sc = la->crit;
    }
    Profiler* prof = g_prof;
    for (int c0 = 0; c0 < max_nf; c0 += C::NB) {
        int maxL[kMaxLevels] = {};
        int maxlev = 0, la_l0 = 0, la_groups = 0, rest_tiles = 0;
        bool overlap = true;  // every next panel's columns are in LA(k)
        // algorithmic work of this panel, per tree level: the update of level
        // l touches R_l rows (all panel rows at the leaves, nbk per child
        // above): 4 R nbk ntr + 2 nbk^2 ntr L_l flops, and reads + writes the
        // R x ntr trailing slice and reads the R x nbk reflectors once; the
        // two update kernels are charged by their share of the columns
        double pf = 0, pb = 0, lf = 0, lb = 0, uf[kMaxLevels] = {}, ub[kMaxLevels] = {};
        for (int i = 0; i < count; ++i) {
            if (!h[i].active || c0 >= h[i].nf) continue;
            const int mp = h[i].m - c0;
            const auto g = tree_geom<T, NBW>(mp);
            for (int l = 0; l < g.levels; ++l) maxL[l] = maxL[l] > g.L(l) ? maxL[l] : g.L(l);
            maxlev = maxlev > g.levels ? maxlev : g.levels;
            const int nbk = h[i].nf - c0 < C::NB ? h[i].nf - c0 : C::NB;
            const int trail = h[i].ncols - c0 - nbk;
            const int nla = row_split_cols(C::NB, h[i].nf, c0, h[i].la_min);
            if (nla > 0) {
                la_l0 = la_l0 > g.L(0) ? la_l0 : g.L(0);
                la_groups = la_groups > (nla + 15) / 16 ? la_groups : (nla + 15) / 16;
            }
            if (trail > nla) rest_tiles = rest_tiles > (trail - nla + 63) / 64 ? rest_tiles : (trail - nla + 63) / 64;
            const int nxt = h[i].nf - c0 - nbk < C::NB ? h[i].nf - c0 - nbk : C::NB;
            if (nxt > 0 && nla < nxt) overlap = false;
            if (prof) {
                pf += 2.0 * mp * nbk * nbk;  // Householder QR of the panel
                pb += 2.0 * mp * nbk * sizeof(T);
                const double share = trail > 0 ? (double)nla / trail : 0.0;
                for (int l = 0; l < g.levels; ++l) {
                    const double rows = l == 0 ? (double)mp : (double)g.L(l - 1) * nbk;
                    const double f = 4.0 * rows * nbk * trail + 2.0 * (double)nbk * nbk * trail * g.L(l);
                    const double b = (2.0 * rows * trail + rows * nbk) * sizeof(T);
                    lf += f * share;
                    lb += b * share;
                    uf[l] += f * (1.0 - share);
                    ub[l] += b * (1.0 - share);
                }
            }
        }
        if (maxL[0] == 0) continue;
        // the tree above the leaves factored beside the leaf-level update
        // (one launch) when no problem has a row-split part
        const bool fuse = NBW == 32 && tree_overlap && la_groups == 0 && maxlev > 1 && rest_tiles > 0;
        int pid = prof ? prof->begin(sc) : -1;
        hipLaunchKernelGGL((k_panel<T, NBW>), dim3(maxL[0], count), dim3(C::PT), 0, sc, d_descs, c0, fuse ? 1 : 0);
        if (prof) prof->end(pid, sc, PROF_PANEL, pf, pb);
        if (la_groups == 0 && rest_tiles == 0) continue;
        if (rest_pending) {  // REST(k-1) updated columns that LA(k) and REST(k) touch
            (void)hipStreamWaitEvent(sc, la->evR, 0);
            rest_pending = false;
        }
        if (fuse) {
            const int uid = prof ? prof->begin(sc) : -1;
            hipLaunchKernelGGL((k_update<T, QrCfg<T, 32>::MT_MAX / 16, true>), dim3(maxL[0], rest_tiles + 1, count),
                               dim3(256), 0, sc, d_descs, c0, 0);
            if (prof) prof->end(uid, sc, PROF_UPDATE, uf[0], ub[0]);
            for (int lev = 1; lev < maxlev; ++lev) {
                const int lid = prof ? prof->begin(sc) : -1;
                launch_update<T, NBW>(dim3(maxL[lev], rest_tiles, count), sc, d_descs, c0, lev);
                if (prof) prof->end(lid, sc, PROF_UPDATE, uf[lev], ub[lev]);
            }
            continue;
        }
        if (la_groups > 0) {
            const int lid = prof ? prof->begin(sc) : -1;
            launch_la<T, NBW>(dim3(la_l0, la_groups, count), sc, d_descs, c0);
            if (prof) prof->end(lid, sc, PROF_LA, lf, lb);
        }
        if (rest_tiles == 0) continue;
        hipStream_t st = sc;
        const bool side = la && la_groups > 0 && overlap;
        if (side) {
            // REST(k) is released after LA(k): a short LA launched while the
            // large REST grid is being dispatched would wait for all of it
            (void)hipEventRecord(la->evP, sc);
            (void)hipStreamWaitEvent(la->rest, la->evP, 0);
            st = la->rest;
        }
        for (int lev = 0; lev < maxlev; ++lev) {
            const int uid = prof ? prof->begin(st) : -1;
            launch_update<T, NBW>(dim3(maxL[lev], rest_tiles, count), st, d_descs, c0, lev);
            if (prof) prof->end(uid, st, PROF_UPDATE, uf[lev], ub[lev]);
        }
        if (side) {
            (void)hipEventRecord(la->evR, la->rest);
            rest_pending = true;
        }
    }
    if (la) {
        if (rest_pending) (void)hipStreamWaitEvent(sc, la->evR, 0);
        (void)hipEventRecord(la->evD, sc);
        (void)hipStreamWaitEvent(s, la->evD, 0);
    }
}
// Every problem of one call has the same panel width (the engine groups them).
template <typename T>
void qr_aug_batch(const QrDesc<T>* d_descs, const QrDesc<T>* h, int count, hipStream_t s, const QrStreams* la,
                  bool tree_overlap) {
    if (count <= 0) return;
    if (h[0].nb == 64) qr_aug_batch_nb<T, 64>(d_descs, h, count, s, la, tree_overlap);
    else qr_aug_batch_nb<T, 32>(d_descs, h, count, s, la, tree_overlap);
}
template void qr_aug_batch<double>(const QrDesc<double>*, const QrDesc<double>*, int, hipStream_t,
                                   const QrStreams*, bool);
template void qr_aug_batch<float>(const QrDesc<float>*, const QrDesc<float>*, int, hipStream_t,
                                  const QrStreams*, bool);

thread_local Profiler* g_prof = nullptr;

}  // namespace sdc
