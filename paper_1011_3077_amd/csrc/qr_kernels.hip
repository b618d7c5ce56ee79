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
#include "profiler.hpp"

namespace sdc {

// Householder QR of one tree node held in registers by a PT-thread
// workgroup (PT/32 = G row groups; with PT = 64 the workgroup is a single
// wavefront, so its barriers cost little).  Thread (grp = tid/32, c = tid%32) owns
// column c, rows r = G*i + grp (i < NR, NR a compile-time tile height).  Rows
// beyond the node and columns >= nbk are zero and stay zero, so every loop
// runs over all NR registers without guards.
//
// Column step j (the usual reflector H_j = I - tau v v^T, v_j = 1,
// beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta, v = x/(alpha - beta)):
// one reduction gives, for every column c, the dot product of column c with
// the part of column j below the diagonal; from it each thread gets the
// norm, the reflector scalars, w_c = v^T P[:, c] and (for c < j) the entries
// v_c^T v_j needed for the compact-WY factor T.  The broadcast column is read
// from LDS once into registers and serves both the reduction and the update;
// the broadcast buffers alternate between steps.
//
// On return the registers hold R (upper part, diagonal = beta) and V
// (strictly lower part); s_tau/s_beta hold tau and beta, s_T the
// upper-triangular T (stride NB+1) with H_0 ... H_{nbk-1} = I - V T V^T.
// Always inlined: a call would pass the register tile by reference and so
// force it into scratch memory.
template <typename T, int NR>
__device__ __forceinline__ void node_qr(T (&p)[NR], int nbk, T* s_col, T* s_row, T* s_red, T* s_Sm, T* s_T,
                                        T* s_tau, T* s_beta) {
    constexpr int NB = QrCfg<T>::NB, G = QrCfg<T>::PT / 32;
    // row j < NB of the node is register j / G of group j % G
    constexpr int NJ = NB / G;
    static_assert(NB % G == 0 && NJ <= NR, "the first NB rows must sit in registers [0, NB / G)");
    const int tid = threadIdx.x, grp = tid >> 5, c = tid & 31;
    for (int j = 0; j < nbk; ++j) {
        const int jr = j / G, jg = j % G;
        T* tcol = s_col + (j & 1) * G * NR;
        T* trow = s_row + (j & 1) * NB;
        T rj = 0;  // row j of this thread's column (meaningful in group jg)
#pragma unroll
        for (int i = 0; i < NJ; ++i) rj = i == jr ? p[i] : rj;
        if (c == j) {  // rows <= j (only in registers < NJ) are zeroed
#pragma unroll
            for (int i = 0; i < NJ; ++i) tcol[grp * NR + i] = (G * i + grp > j) ? p[i] : T(0);
#pragma unroll
            for (int i = NJ; i < NR; ++i) tcol[grp * NR + i] = p[i];
        }
        if (grp == jg) trow[c] = rj;
        __syncthreads();
        T x[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) x[i] = tcol[grp * NR + i];  // zero at rows <= j
        T z0 = 0, z1 = 0, z2 = 0, z3 = 0;
#pragma unroll
        for (int i = 0; i < NR; i += 4) {
            z0 += x[i] * p[i];
            if (i + 1 < NR) z1 += x[i + 1] * p[i + 1];
            if (i + 2 < NR) z2 += x[i + 2] * p[i + 2];
            if (i + 3 < NR) z3 += x[i + 3] * p[i + 3];
        }
        s_red[grp * NB + c] = (z0 + z1) + (z2 + z3);
        __syncthreads();
        T zc = 0, xn2 = 0;
#pragma unroll
        for (int q = 0; q < G; ++q) {
            zc += s_red[q * NB + c];
            xn2 += s_red[q * NB + j];
        }
        const T alpha = trow[j];
        T beta, tau, scale;
        if (xn2 == T(0)) {
            beta = alpha;
            tau = 0;
            scale = 0;
        } else {
            const T nrm = sqrt(alpha * alpha + xn2);
            beta = alpha >= T(0) ? -nrm : nrm;
            // one division: r = 1 / (beta (alpha - beta)) gives
            // scale = 1 / (alpha - beta) = beta r, tau = (beta - alpha) / beta = -(alpha - beta)^2 r
            const T d = alpha - beta;
            const T r = T(1) / (beta * d);
            scale = beta * r;
            tau = -(d * d) * r;
        }
        const T w = trow[c] + scale * zc;  // v_j^T P[:, c]  (= v_c^T v_j for c < j)
        // c > j: p -= tau w v = p - (tau w scale) x;  c < j: unchanged;
        // c == j: v = x scale below the diagonal (x = 0 at rows <= j, which
        // keep p; row j is set below).  Registers >= NJ hold rows >= NB > j,
        // where the two cases are p * 1 + x * (-coef) and p * 0 + x * scale.
        const T tw = c > j ? tau * w : T(0);
        const bool isj = c == j;
        const T coef = tw * scale;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            const T upd = p[i] - coef * x[i];
            p[i] = (isj && G * i + grp > j) ? x[i] * scale : upd;
        }
        const T m1 = isj ? T(0) : T(1), m2 = isj ? scale : -coef;
#pragma unroll
        for (int i = NJ; i < NR; ++i) p[i] = x[i] * m2 + p[i] * m1;
        if (grp == jg) {  // row j: beta on the diagonal, p - tau w v_j (v_j = 1) to the right
            const T nv = isj ? beta : rj - tw;
#pragma unroll
            for (int i = 0; i < NJ; ++i) p[i] = i == jr ? nv : p[i];
        }
        if (c < j && grp == 0) s_Sm[c * (NB + 1) + j] = w;
        if (tid == 0) {
            s_tau[j] = tau;
            s_beta[j] = beta;
        }
    }
    __syncthreads();
    // Compact-WY factor, forward columnwise recurrence
    //   T[i][j] = -tau_j sum_{l=i}^{j-1} T[i][l] (v_l^T v_j),  T[i][i] = tau_i:
    // thread r < NB keeps row r of T in registers; rows are independent.
    if (tid < NB) {
        const int r = tid;
        T t[NB];
#pragma unroll
        for (int l = 0; l < NB; ++l) t[l] = (l == r && l < nbk) ? s_tau[l] : T(0);
#pragma unroll
        for (int j = 1; j < NB; ++j) {
            if (j < nbk) {
                T a0 = 0, a1 = 0;
#pragma unroll
                for (int l = 0; l < j; ++l) {
                    const T term = l >= r ? t[l] * s_Sm[l * (NB + 1) + j] : T(0);
                    if (l & 1) a1 += term;
                    else a0 += term;
                }
                if (r < j) t[j] = -s_tau[j] * (a0 + a1);
            }
        }
#pragma unroll
        for (int l = 0; l < NB; ++l) s_T[r * (NB + 1) + l] = t[l];
    }
    __syncthreads();
}

// Factor the mt x nbk node staged column-major in s_tile (stride LDT) with an
// NR-row register tile: load, QR, write T (NB x NB, column-major) to Tg, and
// put R/V back into s_tile.  s_red/s_Sm/s_T alias the start of s_tile.
template <typename T, int NR>
__device__ __forceinline__ void factor_tile(T* s_tile, int mt, int nbk, T* s_col, T* s_row, T* s_tau, T* s_beta,
                                            T* Tg) {
    constexpr int NB = QrCfg<T>::NB, LDT = QrCfg<T>::MT_MAX + 1, G = QrCfg<T>::PT / 32, PT = QrCfg<T>::PT;
    const int tid = threadIdx.x, grp = tid >> 5, c = tid & 31;
    T* s_red = s_tile;
    T* s_Sm = s_tile + G * NB;
    T* s_T = s_Sm + NB * (NB + 1);
    T p[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const int r = G * i + grp;
        p[i] = r < mt ? s_tile[c * LDT + r] : T(0);
    }
    __syncthreads();
    node_qr<T, NR>(p, nbk, s_col, s_row, s_red, s_Sm, s_T, s_tau, s_beta);
    for (int e = tid; e < NB * NB; e += PT) {
        const int i = e % NB, j = e / NB;
        Tg[e] = (i <= j && j < nbk) ? s_T[i * (NB + 1) + j] : T(0);
    }
    __syncthreads();
    // rows >= mt hold zeros; the tile has LDT >= G NR rows, so store them all
#pragma unroll
    for (int i = 0; i < NR; ++i) s_tile[c * LDT + G * i + grp] = p[i];
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ void factor_node(T* s_tile, int mt, int nbk, T* s_col, T* s_row, T* s_tau, T* s_beta,
                                            T* Tg) {
    constexpr int NRL = QrCfg<T>::RPG, NRS = QrCfg<T>::RPG / 2, G = QrCfg<T>::PT / 32;
    if (mt <= G * NRS) factor_tile<T, NRS>(s_tile, mt, nbk, s_col, s_row, s_tau, s_beta, Tg);
    else factor_tile<T, NRL>(s_tile, mt, nbk, s_col, s_row, s_tau, s_beta, Tg);
}

template <typename T>
__global__ __launch_bounds__(QrCfg<T>::PT) void k_panel(const QrDesc<T>* __restrict__ descs, int c0) {
    using C = QrCfg<T>;
    constexpr int NB = C::NB, RPG = C::RPG, LDT = C::MT_MAX + 1, PT = C::PT, G = PT / 32;
    __shared__ T s_tile[LDT * NB];
    __shared__ T s_col[2 * G * RPG];
    __shared__ T s_row[2 * NB];
    __shared__ T s_tau[NB], s_beta[NB];
    __shared__ int s_last;

    const QrDesc<T> d = descs[blockIdx.y];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(NB, d.nf - c0);
    const int mp = d.m - c0;
    const auto g = tree_geom<T>(mp);
    int node = blockIdx.x;
    if (node >= g.L(0)) return;
    const int par = (c0 / NB) & 1;
    T* const Tm = (par ? d.Tm[1] : d.Tm[0]);
    const int tid = threadIdx.x;
    const size_t ld = (size_t)d.ld;
    T* W = d.W;

    // ---- leaf: rows [row0, row0 + mt) of the panel columns
    // Each thread moves whole rows (all NB columns), so its global accesses
    // are independent and in flight together; across threads every column
    // access is a contiguous run of rows.
    const int row0 = c0 + leaf_lo(node, mp, g.L(0));
    int mt = c0 + leaf_lo(node + 1, mp, g.L(0)) - row0;
    for (int r = tid; r < mt; r += PT) {
        T v[NB];
#pragma unroll
        for (int col = 0; col < NB; ++col) v[col] = col < nbk ? W[(size_t)(c0 + col) * ld + row0 + r] : T(0);
#pragma unroll
        for (int col = 0; col < NB; ++col) s_tile[col * LDT + r] = v[col];
    }
    __syncthreads();
    factor_node<T>(s_tile, mt, nbk, s_col, s_row, s_tau, s_beta, Tm + (size_t)node_index(g, 0, node, d.tm_leaves) * NB * NB);
    for (int r = tid; r < mt; r += PT) {
#pragma unroll
        for (int col = 0; col < NB; ++col)
            if (col < nbk) W[(size_t)(c0 + col) * ld + row0 + r] = s_tile[col * LDT + r];
    }

    // ---- climb the tree: the last child to arrive factors the parent
    for (int level = 1; level < g.levels; ++level) {
        __threadfence();
        __syncthreads();
        const int parent = node / C::F;
        const int iidx = internal_index(g, level, parent);
        const int nch = min(C::F, g.L(level - 1) - parent * C::F);
        if (tid == 0) {
            const unsigned old = atomicAdd(&d.counters[iidx], 1u);
            s_last = (old == (unsigned)(nch - 1));
            if (s_last) d.counters[iidx] = 0u;
        }
        __syncthreads();
        if (!s_last) return;
        __threadfence();
        node = parent;
        mt = nch * NB;
        // stacked upper-triangular R factors of the children (row s of the
        // stack is row s % NB of child s / NB)
        for (int s = tid; s < mt; s += PT) {
            const int t = s / NB, r = s % NB;
            const int rb = c0 + leaf_lo((node * C::F + t) * g.pw(level - 1), mp, g.L(0));
            T v[NB];
#pragma unroll
            for (int col = 0; col < NB; ++col)
                v[col] = (col < nbk && r <= col) ? W[(size_t)(c0 + col) * ld + rb + r] : T(0);
#pragma unroll
            for (int col = 0; col < NB; ++col) s_tile[col * LDT + s] = v[col];
        }
        __syncthreads();
        factor_node<T>(s_tile, mt, nbk, s_col, s_row, s_tau, s_beta,
                       Tm + (size_t)node_index(g, level, node, d.tm_leaves) * NB * NB);
        // explicit reflectors of this node, and its R into the top rows
        T* Vi = (par ? d.Vint[1] : d.Vint[0]) + (size_t)iidx * C::MT_MAX * NB;
        const int rbase = c0 + leaf_lo(node * g.pw(level), mp, g.L(0));
        for (int s = tid; s < C::MT_MAX; s += PT) {
#pragma unroll
            for (int col = 0; col < NB; ++col) {
                T v = 0;
                if (s < mt && col < nbk) v = s > col ? s_tile[col * LDT + s] : (s == col ? T(1) : T(0));
                Vi[(size_t)col * C::MT_MAX + s] = v;
            }
        }
        for (int e = tid; e < nbk * nbk; e += PT) {
            const int col = e / nbk, s = e % nbk;
            if (s <= col) W[(size_t)(c0 + col) * ld + rbase + s] = s_tile[col * LDT + s];
        }
    }
    if (tid < nbk) d.diag[c0 + tid] = s_beta[tid];
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
template <typename T, int RB>
__global__ __launch_bounds__(256, 2) void k_update(const QrDesc<T>* __restrict__ descs, int c0, int level,
                                                   int mode) {
    using C = QrCfg<T>;
    using M = Mfma<T>;
    typedef typename M::v4 v4;
    constexpr int NB = C::NB, VS = NB + 1, XS = 17;  // odd strides: conflict-free LDS access
    __shared__ T s_V[RB * 16 * VS];
    __shared__ T s_X[4 * 16 * XS];
    __shared__ int s_rb[32];

    const QrDesc<T> d = descs[blockIdx.z];
    if (!d.active || c0 >= d.nf) return;
    const int nbk = min(NB, d.nf - c0);
    // column range: all trailing columns (mode 0), the next panel's columns
    // (mode 1, the look-ahead part) or the columns after them (mode 2)
    int cb = c0 + nbk, ce = d.ncols;
    if (mode != 0) {
        const int nxt = max(0, min(NB, d.nf - cb));
        if (mode == 1) ce = cb + nxt;
        else cb += nxt;
    }
    const int col0 = cb + blockIdx.y * 64;
    if (col0 >= ce) return;
    const int par = (c0 / NB) & 1;
    const int mp = d.m - c0;
    const auto g = tree_geom<T>(mp);
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
    }
    const int rows_pad = ((mt + 15) >> 4) << 4;
    // reflectors: each thread moves whole rows (independent loads in flight)
    if (level == 0) {
        for (int s = tid; s < rows_pad; s += 256) {
            T v[NB];
#pragma unroll
            for (int col = 0; col < NB; ++col)
                v[col] = (s < mt && col < nbk) ? (s > col ? W[(size_t)(c0 + col) * ld + lo + s] : (s == col ? T(1) : T(0)))
                                               : T(0);
#pragma unroll
            for (int col = 0; col < NB; ++col) s_V[s * VS + col] = v[col];
        }
    } else {
        const T* Vi = (par ? d.Vint[1] : d.Vint[0]) + (size_t)internal_index(g, level, node) * C::MT_MAX * NB;
        for (int s = tid; s < rows_pad; s += 256) {
            T v[NB];
#pragma unroll
            for (int col = 0; col < NB; ++col) v[col] = (s < mt && col < nbk) ? Vi[(size_t)col * C::MT_MAX + s] : T(0);
#pragma unroll
            for (int col = 0; col < NB; ++col) s_V[s * VS + col] = v[col];
        }
    }
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63, gq = lane >> 4, ln = lane & 15;
    const int cbase = col0 + wave * 16;
    const int rbe = rows_pad >> 4;
    // T factor of this node, as the A operand of Y = T^T W:
    // lane (gq, ln) needs T[k][ln] for k = kb * 16 + row(gq, j)
    const T* Tg = (par ? d.Tm[1] : d.Tm[0]) + (size_t)node_index(g, level, node, d.tm_leaves) * NB * NB;
    T ta[2][2][4];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = kb * 16 + M::row(gq, j);
            ta[0][kb][j] = Tg[(size_t)ln * NB + k];
            ta[1][kb][j] = Tg[(size_t)(16 + ln) * NB + k];
        }

    // C^T slice: row block rb, lane (gq, ln), register v <-> node row 16 rb + ln,
    // column cbase + row(gq, v); wr = the row in W (-1: padding)
    v4 cr[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        cr[rb] = v4{0, 0, 0, 0};
        if (rb < rbe) {
            const int sr = rb * 16 + ln;
            const int wr = sr >= mt ? -1
                           : level == 0 ? lo + sr
                           : ((sr & (NB - 1)) < nbk ? s_rb[sr / NB] + (sr & (NB - 1)) : -1);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = cbase + M::row(gq, v);
                if (wr >= 0 && c < ce) cr[rb][v] = W[(size_t)c * ld + wr];
            }
        }
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
    // C^T -= Y^T V^T: k-steps outer, row blocks inner (RB independent
    // accumulators); each k-step's V^T operands are read from LDS together
    // before its MFMAs
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T a = -(pb ? y1[j] : y0[j]);
            const int kcol = pb * 16 + M::row(gq, j);
            T vb[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) vb[rb] = rb < rbe ? s_V[(rb * 16 + ln) * VS + kcol] : T(0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
                if (rb < rbe) cr[rb] = M::mma(a, vb[rb], cr[rb]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        if (rb < rbe) {
            const int sr = rb * 16 + ln;
            const int wr = sr >= mt ? -1
                           : level == 0 ? lo + sr
                           : ((sr & (NB - 1)) < nbk ? s_rb[sr / NB] + (sr & (NB - 1)) : -1);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = cbase + M::row(gq, v);
                if (wr >= 0 && c < ce) W[(size_t)c * ld + wr] = cr[rb][v];
            }
        }
    }
}

template <typename T>
static void launch_update(int rows, dim3 grid, hipStream_t s, const QrDesc<T>* d, int c0, int lev, int mode);
template <>
void launch_update<double>(int rows, dim3 grid, hipStream_t s, const QrDesc<double>* d, int c0, int lev,
                           int mode) {
    constexpr int RB = QrCfg<double>::MT_MAX / 16;
    (void)rows;
    hipLaunchKernelGGL((k_update<double, RB>), grid, dim3(256), 0, s, d, c0, lev, mode);
}
template <>
void launch_update<float>(int rows, dim3 grid, hipStream_t s, const QrDesc<float>* d, int c0, int lev,
                          int mode) {
    constexpr int RB = QrCfg<float>::MT_MAX / 16;
    (void)rows;
    hipLaunchKernelGGL((k_update<float, RB>), grid, dim3(256), 0, s, d, c0, lev, mode);
}

// Batched augmented QR, panel by panel.  Without `la` every step runs on s:
// panel factorization, then the tree levels of the trailing update.  With
// `la` (look-ahead, depth 1) panel k+1 is factored while the update of the
// columns after it runs concurrently:
//   crit: P(k), [wait rest(k-1)], LA(k) = update of panel k+1's columns, P(k+1) ...
//   rest: [wait P(k)], REST(k) = update of every column after panel k+1
// LA(k) must follow REST(k-1) (both touch panel k+1's columns); P(k+1)
// writes the other parity's T / reflector buffers while REST(k) reads
// panel k's.  crit starts after the work already on s, and s waits for both
// streams before returning.
template <typename T>
void qr_aug_batch(const QrDesc<T>* d_descs, const QrDesc<T>* h, int count, hipStream_t s, const QrStreams* la) {
    using C = QrCfg<T>;
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
    for (int c0 = 0; c0 < max_nf; c0 += C::NB) {
        int maxL[kMaxLevels] = {};
        int maxlev = 0, maxleaf = 0, maxtrail = 0;
        bool next = false;
        for (int i = 0; i < count; ++i) {
            if (!h[i].active || c0 >= h[i].nf) continue;
            const int mp = h[i].m - c0;
            const auto g = tree_geom<T>(mp);
            for (int l = 0; l < g.levels; ++l) maxL[l] = maxL[l] > g.L(l) ? maxL[l] : g.L(l);
            maxlev = maxlev > g.levels ? maxlev : g.levels;
            const int blocks16 = (mp + 15) / 16;
            const int leaf = g.L(0) == 1 ? mp : min(mp, (blocks16 + g.L(0) - 1) / g.L(0) * 16);
            maxleaf = maxleaf > leaf ? maxleaf : leaf;
            const int nbk = h[i].nf - c0 < C::NB ? h[i].nf - c0 : C::NB;
            const int trail = h[i].ncols - c0 - nbk;
            maxtrail = maxtrail > trail ? maxtrail : trail;
            next |= c0 + nbk < h[i].nf;
        }
        if (maxL[0] == 0) continue;
        // algorithmic work of this panel, per tree level: the update of level
        // l touches R_l rows (all panel rows at the leaves, nbk per child
        // above): 4 R nbk ntr + 2 nbk^2 ntr L_l flops, and reads + writes the
        // R x ntr trailing slice and reads the R x nbk reflectors once
        double pf = 0, pb = 0, uf[kMaxLevels] = {}, ub[kMaxLevels] = {};
        Profiler* prof = g_prof;
        if (prof) {
            for (int i = 0; i < count; ++i) {
                if (!h[i].active || c0 >= h[i].nf) continue;
                const int mp = h[i].m - c0;
                const auto g = tree_geom<T>(mp);
                const double nbk = h[i].nf - c0 < C::NB ? h[i].nf - c0 : C::NB;
                const double ntr = h[i].ncols - c0 - nbk;
                pf += 2.0 * mp * nbk * nbk;               // Householder QR of the panel
                pb += 2.0 * mp * nbk * sizeof(T);
                for (int l = 0; l < g.levels; ++l) {
                    const double rows = l == 0 ? (double)mp : (double)g.L(l - 1) * nbk;
                    uf[l] += 4.0 * rows * nbk * ntr + 2.0 * nbk * nbk * ntr * g.L(l);
                    ub[l] += (2.0 * rows * ntr + rows * nbk) * sizeof(T);
                }
            }
        }
        int pid = prof ? prof->begin(sc) : -1;
        hipLaunchKernelGGL(k_panel<T>, dim3(maxL[0], count), dim3(C::PT), 0, sc, d_descs, c0);
        if (prof) prof->end(pid, sc, PROF_PANEL, pf, pb);
        if (maxtrail <= 0) continue;
        auto run_levels = [&](hipStream_t st, int mode, int tiles, double share) {
            for (int lev = 0; lev < maxlev; ++lev) {
                const int rows = lev == 0 ? maxleaf : C::MT_MAX;
                const dim3 grid(maxL[lev], tiles, count);
                const int uid = prof ? prof->begin(st) : -1;
                launch_update<T>(rows, grid, st, d_descs, c0, lev, mode);
                if (prof) prof->end(uid, st, PROF_UPDATE, uf[lev] * share, ub[lev] * share);
            }
        };
        if (!la || !next) {
            if (rest_pending) {  // the previous rest update touches these columns
                (void)hipStreamWaitEvent(sc, la->evR, 0);
                rest_pending = false;
            }
            run_levels(sc, 0, (maxtrail + 63) / 64, 1.0);
            continue;
        }
        (void)hipEventRecord(la->evP, sc);
        if (rest_pending) (void)hipStreamWaitEvent(sc, la->evR, 0);
        const double f_la = maxtrail > 0 ? (double)C::NB / maxtrail : 0.0;
        run_levels(sc, 1, 1, f_la);
        (void)hipStreamWaitEvent(la->rest, la->evP, 0);
        // the next panel may be narrower than NB, so the rest can start
        // anywhere in [c0 + nbk, c0 + nbk + NB]: size the grid for all trailing
        // columns (tiles past a problem's range exit at once)
        run_levels(la->rest, 2, (maxtrail + 63) / 64, 1.0 - f_la);
        (void)hipEventRecord(la->evR, la->rest);
        rest_pending = true;
    }
    if (la) {
        if (rest_pending) (void)hipStreamWaitEvent(sc, la->evR, 0);
        (void)hipEventRecord(la->evD, sc);
        (void)hipStreamWaitEvent(s, la->evD, 0);
    }
}
template void qr_aug_batch<double>(const QrDesc<double>*, const QrDesc<double>*, int, hipStream_t,
                                   const QrStreams*);
template void qr_aug_batch<float>(const QrDesc<float>*, const QrDesc<float>*, int, hipStream_t,
                                  const QrStreams*);

thread_local Profiler* g_prof = nullptr;

}  // namespace sdc
