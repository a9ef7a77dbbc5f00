// Device kernels of block cyclic reduction for Hermitian positive definite
// block-tridiagonal systems (arXiv 1807.00370), written for gfx950 (CDNA4,
// wave64).
//
// A reduction level works on a block-tridiagonal system of n blocks in which
// position p couples with p - d and p + d (d = 1 for the one-sided schedule
// with compacted levels; d = 2^level for Algorithm 1, which keeps every block
// in place).  Three kernels make up one level:
//
//   k_elim    one work-group per eliminated block p: L_p = chol(A_p), then by
//             forward substitution P_p = L_p \ B_p^H, Q_p = L_p \ B_{p-d} and
//             g_p = L_p \ y_p -- the Section 4 recipe (Gt = L \ G) applied to
//             the three operands G of Eq. (Formulas).
//   k_reduce  one work-group per kept block q with eliminated neighbours
//             l = q - d and r = q + d: the reduced system of Eq. (Formulas),
//               A'_q = A_q - P_l^H P_l - Q_r^H Q_r   (lower triangle, mirrored,
//                                                    real diagonal: Section 4)
//               B'_q = -P_r^H Q_r
//               y'_q = y_q - P_l^H g_l - Q_r^H g_r
//   k_back    one work-group per eliminated block: recovers its unknowns from
//             the first block row of the reordered system (Section 2),
//               x_p = L_p^{-H} (g_p - Q_p x_{p-d} - P_p x_{p+d}).
//
// Work items of many systems (a ragged batch) share one launch: a launch gets
// a table of segments (one per system), each covering a contiguous range of
// work items; a work-group finds its segment by binary search and loops over
// work items grid-stride, so one launch per level serves the whole batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crs {

template <class T>
struct alignas(2 * sizeof(T)) cx {
    T r, i;
};

// Element of a real array (the real symmetric dtypes) read where complex
// elements are expected: the imaginary part is a constant zero.
template <class T>
struct rl {
    T r;
    static constexpr T i = T(0);
};

// Element of a level input read in another precision or kind (the mixed
// form's FP32 levels read the caller's FP64 arrays at level 0 and round on
// load; the real dtypes read real arrays).
template <class T, class S>
__device__ __forceinline__ cx<T> cvt(const cx<S> v)
{
    return cx<T>{(T)v.r, (T)v.i};
}
template <class T, class S>
__device__ __forceinline__ cx<T> cvt(const rl<S> v)
{
    return cx<T>{(T)v.r, T(0)};
}

// c -= a * b
template <class T>
__device__ __forceinline__ void msub(cx<T>& c, const cx<T> a, const cx<T> b)
{
    c.r = fma(-a.r, b.r, c.r);
    c.r = fma(a.i, b.i, c.r);
    c.i = fma(-a.r, b.i, c.i);
    c.i = fma(-a.i, b.r, c.i);
}

// c -= conj(a) * b
template <class T>
__device__ __forceinline__ void msub_ca(cx<T>& c, const cx<T> a, const cx<T> b)
{
    c.r = fma(-a.r, b.r, c.r);
    c.r = fma(-a.i, b.i, c.r);
    c.i = fma(-a.r, b.i, c.i);
    c.i = fma(a.i, b.r, c.i);
}

// c -= a * conj(b)
template <class T>
__device__ __forceinline__ void msub_cb(cx<T>& c, const cx<T> a, const cx<T> b)
{
    c.r = fma(-a.r, b.r, c.r);
    c.r = fma(-a.i, b.i, c.r);
    c.i = fma(-a.i, b.r, c.i);
    c.i = fma(a.r, b.i, c.i);
}

// One system at one level.  Offsets count complex elements from the base
// pointers the launch receives (user arrays at level 0, the workspace after).
struct Seg {
    int64_t w0;               // first work item of this segment in the launch
    int32_t n, m, k, d;       // blocks, block size, rhs columns, neighbour distance
    int32_t e0, es, ne;       // eliminated positions p = e0 + t * es, t < ne
    int32_t k0, ks, nk;       // kept positions q = k0 + t * ks, t < nk
    int32_t level, sys;
    int32_t out_by_pos, pad_; // reduced outputs indexed by q (1) or by t (0)
    int64_t xo, xs;           // unknowns of position p: block xo + xs * p of x
    int64_t ob0, obs;         // original 1-based block row of position p
    int64_t oA, oB, oy;       // level inputs
    int64_t oL, oP, oQ, og;   // per eliminated block (index t)
    int64_t oAo, oBo, oyo;    // reduced system
    int64_t ox;               // unknowns of the system
    int64_t oD;               // inverse diagonal tiles (block sizes above 32)
    int64_t oU;               // mixed form, level 0: the system's FP64 solution
};

// Store of element e of the unknowns x_p of an eliminated block.  Normally
// into xp (the level's unknowns); in the mixed form's level 0 (upd != 0) the
// value is the correction d_p and goes into the FP64 solution u_p instead:
// u = d (upd = 1) or u += d (upd = 2).
template <class T>
__device__ __forceinline__ void put_x(cx<T>* xp, cx<double>* up, int upd, int64_t e, cx<T> v)
{
    if (!upd) {
        xp[e] = v;
    } else if (upd == 1) {
        up[e] = cvt<double>(v);
    } else {
        cx<double> o = up[e];
        o.r += (double)v.r;
        o.i += (double)v.i;
        up[e] = o;
    }
}

// The mixed form's level 0 also moves the correction of the kept neighbour
// q = p + d (solved at the deeper levels) into the FP64 solution: elements
// [e0, e1) with stride es of u_q (+)= d_q.  Every kept block of level 0 has
// exactly one eliminated left neighbour, so each is updated once.
// Four elements at a time: their loads are issued together (element e0
// stands in past the end), so a chunk costs one round trip rather than one
// per element waiting behind the previous store.
template <class T>
__device__ __forceinline__ void put_kept(const cx<T>* dq, cx<double>* uq, int upd, int64_t e0,
                                         int64_t e1, int64_t es)
{
    constexpr int U = 4;
    for (int64_t e = e0; e < e1; e += U * es) {
        cx<T> dv[U];
        cx<double> ov[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t ei = e + u * es < e1 ? e + u * es : e0;
            dv[u] = dq[ei];
            ov[u] = upd == 2 ? uq[ei] : cx<double>{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e + u * es < e1)
                uq[e + u * es] = cx<double>{ov[u].r + (double)dv[u].r, ov[u].i + (double)dv[u].i};
    }
}

constexpr unsigned long long kNoFail = ~0ull;

__device__ __forceinline__ unsigned long long fail_key(int level, int64_t block)
{
    return ((unsigned long long)level << 40) | (unsigned long long)block;
}

// Row of packed lower-triangular index e (e = r (r + 1) / 2 + c, c <= r).
__device__ __forceinline__ int tri_row(int e)
{
    int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while ((r + 1) * (r + 2) / 2 <= e)
        ++r;
    while (r * (r + 1) / 2 > e)
        --r;
    return r;
}

__device__ __forceinline__ int find_seg(const Seg* __restrict__ s, int nseg, int64_t w)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s[mid].w0 <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ----------------------------------------------------------------- k_elim

template <class T, int MT, int NT, int PW, class EI = cx<T>>
__global__ __launch_bounds__(NT) void k_elim(const Seg* __restrict__ segs, int nseg, int64_t total,
                                             const EI* __restrict__ inA,
                                             const EI* __restrict__ inB,
                                             const EI* __restrict__ iny, cx<T>* __restrict__ W,
                                             unsigned long long* __restrict__ flags, int with_mat,
                                             int with_rhs)
{
    constexpr int LD = MT + 1;
    constexpr int GLD = PW + 1;
    __shared__ cx<T> sL[MT * LD];
    __shared__ cx<T> sG[MT * GLD];
    __shared__ T sInv[MT];
    __shared__ int sFail;
    const int tid = threadIdx.x;

    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const Seg& s = segs[find_seg(segs, nseg, w)];
        const int64_t t = w - s.w0;
        const int p = s.e0 + (int)t * s.es;
        const int m = s.m, k = s.k, d = s.d;
        const bool hasPrev = p - d >= 0, hasNext = p + d < s.n;
        if ((flags[s.sys] >> 40) < (unsigned long long)s.level)
            continue; // broke down at an earlier level: nothing left to do
        cx<T>* Lg = W + s.oL + t * (int64_t)m * m;
        __syncthreads();
        if (with_mat) {
            const EI* Ap = inA + s.oA + (int64_t)p * m * m;
            for (int e = tid; e < m * m; e += NT)
                sL[(e / m) * LD + e % m] = cvt<T>(Ap[e]);
            if (tid == 0)
                sFail = 0;
            __syncthreads();
            // right-looking Cholesky on the lower triangle
            for (int c = 0; c < m; ++c) {
                const T dg = sL[c * LD + c].r;
                const T sq = sqrt(dg);
                const T inv = T(1) / sq;
                for (int r = c + 1 + tid; r < m; r += NT) {
                    cx<T> v = sL[r * LD + c];
                    v.r *= inv;
                    v.i *= inv;
                    sL[r * LD + c] = v;
                }
                __syncthreads();
                if (tid == 0) {
                    sL[c * LD + c] = cx<T>{sq, inv}; // inverse pivot kept in the imaginary slot
                    sInv[c] = inv;
                    if (!(dg > T(0)))
                        sFail = 1;
                }
                const int nt = m - c - 1;
                for (int e = tid; e < nt * nt; e += NT) {
                    const int r = c + 1 + e / nt, q = c + 1 + e % nt;
                    if (q <= r) {
                        cx<T> v = sL[r * LD + q];
                        msub_cb(v, sL[r * LD + c], sL[q * LD + c]);
                        sL[r * LD + q] = v;
                    }
                }
                __syncthreads();
            }
            if (tid == 0 && sFail)
                atomicMin(&flags[s.sys], fail_key(s.level, s.ob0 + s.obs * p));
            for (int e = tid; e < m * (m + 1) / 2; e += NT) {
                const int r = tri_row(e), c = e - r * (r + 1) / 2;
                Lg[e] = sL[r * LD + c];
            }
        } else {
            for (int e = tid; e < m * (m + 1) / 2; e += NT) {
                const int r = tri_row(e), c = e - r * (r + 1) / 2;
                sL[r * LD + c] = Lg[e];
            }
            __syncthreads();
            for (int c = tid; c < m; c += NT)
                sInv[c] = sL[c * LD + c].i;
        }
        // forward substitution on the operands of Eq. (Formulas)
        for (int src = 0; src < 3; ++src) {
            int ncol, ldg;
            const EI* G;
            cx<T>* out;
            bool herm = false;
            if (src == 0) {
                if (!with_mat || !hasNext)
                    continue;
                ncol = m;
                ldg = m;
                G = inB + s.oB + (int64_t)p * m * m;
                herm = true;
                out = W + s.oP + t * (int64_t)m * m;
            } else if (src == 1) {
                if (!with_mat || !hasPrev)
                    continue;
                ncol = m;
                ldg = m;
                G = inB + s.oB + (int64_t)(p - d) * m * m;
                out = W + s.oQ + t * (int64_t)m * m;
            } else {
                if (!with_rhs)
                    continue;
                ncol = k;
                ldg = k;
                G = iny + s.oy + (int64_t)p * m * k;
                out = W + s.og + t * (int64_t)m * k;
            }
            for (int c0 = 0; c0 < ncol; c0 += PW) {
                const int cw = min(PW, ncol - c0);
                __syncthreads();
                if (herm) {
                    for (int e = tid; e < m * cw; e += NT) {
                        const int c = e / m, r = e % m;
                        cx<T> v = cvt<T>(G[(int64_t)(c0 + c) * m + r]);
                        v.i = -v.i;
                        sG[r * GLD + c] = v;
                    }
                } else {
                    for (int e = tid; e < m * cw; e += NT) {
                        const int r = e / cw, c = e % cw;
                        sG[r * GLD + c] = cvt<T>(G[(int64_t)r * ldg + c0 + c]);
                    }
                }
                __syncthreads();
                for (int r = 0; r < m; ++r) {
                    const T iv = sInv[r];
                    for (int c = tid; c < cw; c += NT) {
                        cx<T> v = sG[r * GLD + c];
                        v.r *= iv;
                        v.i *= iv;
                        sG[r * GLD + c] = v;
                    }
                    __syncthreads();
                    const int nr = m - r - 1;
                    for (int e = tid; e < nr * cw; e += NT) {
                        const int rr = r + 1 + e / cw, c = e % cw;
                        cx<T> v = sG[rr * GLD + c];
                        msub(v, sL[rr * LD + r], sG[r * GLD + c]);
                        sG[rr * GLD + c] = v;
                    }
                    __syncthreads();
                }
                for (int e = tid; e < m * cw; e += NT) {
                    const int r = e / cw, c = e % cw;
                    out[(int64_t)r * ldg + c0 + c] = sG[r * GLD + c];
                }
            }
        }
    }
}

// --------------------------------------------------------------- k_reduce

// acc[i][j] -= sum_t conj(X[t][a_i]) Y[t][b_j] for a_i = ty + 16 i < n1,
// b_j = tx + 16 j < n2, t < kd; X and Y are row-major with leading
// dimensions ldx, ldy.  Staged through shared memory KC rows at a time.
template <class T, int R, int NT, int KC>
__device__ __forceinline__ void gram_sub(cx<T> (&acc)[R][R], const cx<T>* __restrict__ X, int ldx,
                                         int n1, const cx<T>* __restrict__ Y, int ldy, int n2,
                                         int kd, cx<T>* sX, cx<T>* sY)
{
    constexpr int WD = 16 * R + 1;
    const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
    for (int k0 = 0; k0 < kd; k0 += KC) {
        const int kc = min(KC, kd - k0);
        __syncthreads();
        for (int e = tid; e < kc * n1; e += NT) {
            const int t = e / n1, a = e % n1;
            sX[t * WD + a] = X[(int64_t)(k0 + t) * ldx + a];
        }
        for (int e = tid; e < kc * n2; e += NT) {
            const int t = e / n2, b = e % n2;
            sY[t * WD + b] = Y[(int64_t)(k0 + t) * ldy + b];
        }
        __syncthreads();
        if (ty < 16) {
            for (int t = 0; t < kc; ++t) {
                cx<T> xa[R], yb[R];
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    xa[i] = sX[t * WD + ty + 16 * i];
                    yb[i] = sY[t * WD + tx + 16 * i];
                }
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        msub_ca(acc[i][j], xa[i], yb[j]);
            }
        }
    }
}

template <class T, int MT, int NT, class EI = cx<T>>
__global__ __launch_bounds__(NT) void k_reduce(const Seg* __restrict__ segs, int nseg, int64_t total,
                                               const EI* __restrict__ inA,
                                               const EI* __restrict__ iny,
                                               cx<T>* __restrict__ W,
                                               const unsigned long long* __restrict__ flags,
                                               int with_mat, int with_rhs)
{
    static_assert(NT == 256, "16 x 16 thread tile");
    constexpr int R = (MT + 15) / 16;
    constexpr int KC = 16;
    constexpr int WD = 16 * R + 1;
    __shared__ cx<T> sX[KC * WD];
    __shared__ cx<T> sY[KC * WD];
    const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;

    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const Seg& s = segs[find_seg(segs, nseg, w)];
        const int64_t t = w - s.w0;
        const int q = s.k0 + (int)t * s.ks;
        const int m = s.m, k = s.k, d = s.d, n = s.n;
        const int l = q - d, r = q + d;
        const bool hasL = l >= 0, hasR = r < n;
        const int64_t tl = hasL ? (l - s.e0) / s.es : 0, tr = hasR ? (r - s.e0) / s.es : 0;
        const int64_t oi = s.out_by_pos ? q : t;
        const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
        if ((flags[s.sys] >> 40) <= (unsigned long long)s.level)
            continue; // the level's elimination broke down: stop this system
        if (with_mat) {
            cx<T> acc[R][R];
            const EI* Aq = inA + s.oA + q * mm;
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int a = ty + 16 * i, b = tx + 16 * j;
                    acc[i][j] = (a < m && b < m && b <= a) ? cvt<T>(Aq[a * m + b]) : cx<T>{T(0), T(0)};
                }
            if (hasL) {
                const cx<T>* P = W + s.oP + tl * mm;
                gram_sub<T, R, NT, KC>(acc, P, m, m, P, m, m, m, sX, sY);
            }
            if (hasR) {
                const cx<T>* Q = W + s.oQ + tr * mm;
                gram_sub<T, R, NT, KC>(acc, Q, m, m, Q, m, m, m, sX, sY);
            }
            cx<T>* Vo = W + s.oAo + oi * mm;
#pragma unroll
            for (int i = 0; i < R; ++i)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int a = ty + 16 * i, b = tx + 16 * j;
                    if (a < m && b < m && b <= a) {
                        cx<T> v = acc[i][j];
                        if (a == b)
                            v.i = T(0);
                        Vo[a * m + b] = v;
                    }
                }
            if (hasR && r + d < n) {
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        acc[i][j] = cx<T>{T(0), T(0)};
                gram_sub<T, R, NT, KC>(acc, W + s.oP + tr * mm, m, m, W + s.oQ + tr * mm, m, m, m,
                                       sX, sY);
                cx<T>* Fo = W + s.oBo + oi * mm;
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int a = ty + 16 * i, b = tx + 16 * j;
                        if (a < m && b < m)
                            Fo[a * m + b] = acc[i][j];
                    }
            }
        }
        if (with_rhs) {
            const EI* yq = iny + s.oy + q * mk;
            cx<T>* yo = W + s.oyo + oi * mk;
            for (int c0 = 0; c0 < k; c0 += 16 * R) {
                const int cw = min(16 * R, k - c0);
                cx<T> acc[R][R];
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int a = ty + 16 * i, b = tx + 16 * j;
                        acc[i][j] = (a < m && b < cw) ? cvt<T>(yq[a * k + c0 + b]) : cx<T>{T(0), T(0)};
                    }
                if (hasL)
                    gram_sub<T, R, NT, KC>(acc, W + s.oP + tl * mm, m, m, W + s.og + tl * mk + c0,
                                           k, cw, m, sX, sY);
                if (hasR)
                    gram_sub<T, R, NT, KC>(acc, W + s.oQ + tr * mm, m, m, W + s.og + tr * mk + c0,
                                           k, cw, m, sX, sY);
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int j = 0; j < R; ++j) {
                        const int a = ty + 16 * i, b = tx + 16 * j;
                        if (a < m && b < cw)
                            yo[a * k + c0 + b] = acc[i][j];
                    }
            }
        }
    }
}

// ----------------------------------------------------------------- k_back

template <class T, int MT, int NT, int PW>
__global__ __launch_bounds__(NT) void k_back(const Seg* __restrict__ segs, int nseg, int64_t total,
                                             const cx<T>* __restrict__ W, cx<T>* __restrict__ X,
                                             const unsigned long long* __restrict__ flags,
                                             cx<double>* __restrict__ U, int upd)
{
    constexpr int LD = MT + 1;
    constexpr int GLD = PW + 1;
    __shared__ cx<T> sL[MT * LD];
    __shared__ cx<T> sW[MT * GLD];
    __shared__ T sInv[MT];
    const int tid = threadIdx.x;

    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const Seg& s = segs[find_seg(segs, nseg, w)];
        const int64_t t = w - s.w0;
        const int p = s.e0 + (int)t * s.es;
        const int m = s.m, k = s.k, d = s.d;
        const bool hasPrev = p - d >= 0, hasNext = p + d < s.n;
        const bool failed = flags[s.sys] != kNoFail;
        const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
        cx<T>* xp = X + s.ox + (s.xo + s.xs * p) * mk;
        cx<double>* up = upd ? U + s.oU + p * mk : nullptr;
        if (failed) {
            const T nan = T(NAN);
            for (int e = tid; e < m * k; e += NT) {
                put_x<T>(xp, up, upd ? 1 : 0, e, cx<T>{nan, nan});
                if (upd && hasNext)
                    put_x<T>(xp, up + d * mk, 1, e, cx<T>{nan, nan});
            }
            continue;
        }
        const cx<T>* xm = X + s.ox + (s.xo + s.xs * (p - d)) * mk;
        const cx<T>* xn = X + s.ox + (s.xo + s.xs * (p + d)) * mk;
        if (upd && hasNext)
            put_kept<T>(xn, up + d * mk, upd, tid, m * k, NT);
        const cx<T>* L = W + s.oL + t * mm;
        const cx<T>* P = W + s.oP + t * mm;
        const cx<T>* Q = W + s.oQ + t * mm;
        const cx<T>* g = W + s.og + t * mk;
        __syncthreads();
        for (int e = tid; e < m * (m + 1) / 2; e += NT) {
            const int r = tri_row(e), c = e - r * (r + 1) / 2;
            sL[r * LD + c] = L[e];
        }
        __syncthreads();
        for (int c = tid; c < m; c += NT)
            sInv[c] = sL[c * LD + c].i;
        for (int c0 = 0; c0 < k; c0 += PW) {
            const int cw = min(PW, k - c0);
            __syncthreads();
            for (int e = tid; e < m * cw; e += NT) {
                const int r = e / cw, c = e % cw;
                cx<T> v = g[r * k + c0 + c];
                if (hasPrev)
                    for (int u = 0; u < m; ++u)
                        msub(v, Q[r * m + u], xm[u * k + c0 + c]);
                if (hasNext)
                    for (int u = 0; u < m; ++u)
                        msub(v, P[r * m + u], xn[u * k + c0 + c]);
                sW[r * GLD + c] = v;
            }
            __syncthreads();
            // L^H x = w, backward substitution
            for (int r = m - 1; r >= 0; --r) {
                const T iv = sInv[r];
                for (int c = tid; c < cw; c += NT) {
                    cx<T> v = sW[r * GLD + c];
                    v.r *= iv;
                    v.i *= iv;
                    sW[r * GLD + c] = v;
                }
                __syncthreads();
                for (int e = tid; e < r * cw; e += NT) {
                    const int rr = e / cw, c = e % cw;
                    cx<T> v = sW[rr * GLD + c];
                    msub_ca(v, sL[r * LD + rr], sW[r * GLD + c]);
                    sW[rr * GLD + c] = v;
                }
                __syncthreads();
            }
            for (int e = tid; e < m * cw; e += NT) {
                const int r = e / cw, c = e % cw;
                put_x<T>(xp, up, upd, r * k + c0 + c, sW[r * GLD + c]);
            }
        }
    }
}

// ------------------------------------------------------------------- adjoint

// Per block row j of a system: gA_j = -lam_j x_j^H and, for j < N,
// gB_j = -(lam_{j+1} x_j^H + x_{j+1} lam_j^H).  Segments here describe whole
// systems (n = N blocks, one work item per block row; offsets oA/oB for the
// gradients, oy for lam and ox for x).
template <class T, int MT, int NT>
__global__ __launch_bounds__(NT) void k_grad(const Seg* __restrict__ segs, int nseg, int64_t total,
                                             const cx<T>* __restrict__ X,
                                             const cx<T>* __restrict__ Lam, cx<T>* __restrict__ gA,
                                             cx<T>* __restrict__ gB)
{
    constexpr int R = (MT + 15) / 16;
    constexpr int KC = 16;
    constexpr int WD = 16 * R + 1;
    __shared__ cx<T> sl0[KC * WD], sx0[KC * WD], sl1[KC * WD], sx1[KC * WD];
    const int tid = threadIdx.x, ty = tid / 16, tx = tid % 16;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        const Seg& s = segs[find_seg(segs, nseg, w)];
        const int j = (int)(w - s.w0);
        const int m = s.m, k = s.k, n = s.n;
        const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
        const bool hasB = j + 1 < n;
        const cx<T>* l0 = Lam + s.oy + j * mk;
        const cx<T>* x0 = X + s.ox + j * mk;
        const cx<T>* l1 = l0 + mk;
        const cx<T>* x1 = x0 + mk;
        cx<T> a0[R][R], a1[R][R];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int jj = 0; jj < R; ++jj) {
                a0[i][jj] = cx<T>{T(0), T(0)};
                a1[i][jj] = cx<T>{T(0), T(0)};
            }
        for (int c0 = 0; c0 < k; c0 += KC) {
            const int kc = min(KC, k - c0);
            __syncthreads();
            // stage columns c0..c0+kc of the m x k blocks, transposed: s[c][a]
            for (int e = tid; e < m * kc; e += NT) {
                const int a = e / kc, c = e % kc;
                sl0[c * WD + a] = l0[a * k + c0 + c];
                sx0[c * WD + a] = x0[a * k + c0 + c];
                if (hasB) {
                    sl1[c * WD + a] = l1[a * k + c0 + c];
                    sx1[c * WD + a] = x1[a * k + c0 + c];
                }
            }
            __syncthreads();
            for (int c = 0; c < kc; ++c) {
#pragma unroll
                for (int i = 0; i < R; ++i)
#pragma unroll
                    for (int jj = 0; jj < R; ++jj) {
                        const int a = ty + 16 * i, b = tx + 16 * jj;
                        if (a < m && b < m) {
                            msub_cb(a0[i][jj], sl0[c * WD + a], sx0[c * WD + b]);
                            if (hasB) {
                                msub_cb(a1[i][jj], sl1[c * WD + a], sx0[c * WD + b]);
                                msub_cb(a1[i][jj], sx1[c * WD + a], sl0[c * WD + b]);
                            }
                        }
                    }
            }
        }
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int jj = 0; jj < R; ++jj) {
                const int a = ty + 16 * i, b = tx + 16 * jj;
                if (a < m && b < m) {
                    gA[s.oA + j * mm + a * m + b] = a0[i][jj];
                    if (hasB)
                        gB[s.oB + j * mm + a * m + b] = a1[i][jj];
                }
            }
    }
}

// ------------------------------------------------------------------- status

__global__ void k_flags_init(unsigned long long* flags, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        flags[i] = kNoFail;
}

} // namespace crs
