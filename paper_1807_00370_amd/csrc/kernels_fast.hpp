// One-wave kernels of a reduction level for block sizes up to 32 (elimination,
// back substitution) and up to 64 (reduced-system products).  Same
// arithmetic and outputs as the work-group kernels in kernels.hpp; the
// difference is the mapping onto a single wave64:
//
//   k_elim_w    Cholesky of A_p on a packed lower triangle in LDS, then the
//               forward substitutions L \ [B_p^H | B_{p-d} | y_p] with one
//               lane per right-hand-side column, the column held in
//               registers and L read by broadcast from LDS -- no work-group
//               barriers inside the substitution.
//   k_reduce_m  the products P^H P, Q^H Q, P^H Q, P^H g, Q^H g of Eq.
//               (Formulas) on MFMA (16x16x4, real-pair 4-multiply complex
//               form), operands loaded from HBM straight into the MFMA lane
//               layout; diagonal blocks are written as their lower triangle
//               only (the Hermitian reading every consumer uses).
//   k_back_m    w = g - Q x_{p-d} - P x_{p+d} on MFMA, then L^H x = w with one
//               lane per column.
#pragma once

#include "kernels.hpp"

namespace crs {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <class T>
struct MF;
template <>
struct MF<double> {
    using v4 = d4v;
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output row of accumulator register v in a lane with kr = lane / 16
    static __device__ __forceinline__ int row(int kr, int v) { return kr + 4 * v; }
};
template <>
struct MF<float> {
    using v4 = f4v;
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int kr, int v) { return 4 * kr + v; }
};

// Waves per SIMD to ask the register allocator for when a column of MT
// complex values lives in registers (MT * sizeof(T) / 2 VGPRs) next to the
// operands of the substitution.
template <class T, int MT>
constexpr int col_waves()
{
    return (512 / (MT * (int)sizeof(T) / 2 + 96)) > 8 ? 8 : (512 / (MT * (int)sizeof(T) / 2 + 96));
}

template <class T>
__device__ __forceinline__ cx<T> czero()
{
    return cx<T>{T(0), T(0)};
}

// MFMA 16x16x4 lane layout (wave64, checked on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register v of lane l
// holds D[row][l % 16] with row = 4 (l / 16) + v for the f32 instruction and
// row = l / 16 + 4 v for the f64 instruction (MF<T>::row).

// Operands are loaded four k-steps at a time, one group ahead of the MFMAs
// that consume the previous group; the scheduling barrier keeps the compiler
// from hoisting every load of the tile to the top (register pressure).
constexpr int kGroup = 4;

// (cr, ci) += X^H Y on the 16 x 16 tile with rows cx0.. (columns of X) and
// columns cy0.. (columns of Y); X, Y row-major, contraction over their first
// kd rows.  Out-of-range rows and columns read as zero.
template <class T, int KS>
__device__ __forceinline__ void tile_hn(typename MF<T>::v4& cr, typename MF<T>::v4& ci,
                                        const cx<T>* __restrict__ X, int ldx, int ncx, int cx0,
                                        const cx<T>* __restrict__ Y, int ldy, int ncy, int cy0,
                                        int kd)
{
    constexpr int G = KS < kGroup ? KS : kGroup, NG = KS / G;
    const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int ax = cx0 + cc, by = cy0 + cc;
    const bool okx = ax < ncx, oky = by < ncy;
    const cx<T>* xb = X + (kr * ldx + ax);
    const cx<T>* yq = Y + (kr * ldy + by);
    const int sx = 4 * ldx, sy = 4 * ldy;
    cx<T> xa[2][G], yb[2][G];
    auto load = [&](int g, int b) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int ks = g * G + u, t = 4 * ks + kr;
            xa[b][u] = (t < kd && okx) ? xb[ks * sx] : czero<T>();
            yb[b][u] = (t < kd && oky) ? yq[ks * sy] : czero<T>();
        }
    };
    load(0, 0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG)
            load(g + 1, (g + 1) & 1);
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const cx<T> a = xa[g & 1][u], b = yb[g & 1][u];
            cr = MF<T>::mma(a.r, b.r, cr);
            cr = MF<T>::mma(a.i, b.i, cr);
            ci = MF<T>::mma(a.r, b.i, ci);
            ci = MF<T>::mma(-a.i, b.r, ci);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// (cr, ci) += X Y on the tile with rows rx0.. (rows of X) and columns cy0..
// (columns of Y); contraction over kd columns of X / rows of Y.
template <class T, int KS>
__device__ __forceinline__ void tile_nn(typename MF<T>::v4& cr, typename MF<T>::v4& ci,
                                        const cx<T>* __restrict__ X, int ldx, int nrx, int rx0,
                                        const cx<T>* __restrict__ Y, int ldy, int ncy, int cy0,
                                        int kd)
{
    constexpr int G = KS < kGroup ? KS : kGroup, NG = KS / G;
    const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int ar = rx0 + cc, by = cy0 + cc;
    const bool okx = ar < nrx, oky = by < ncy;
    const cx<T>* xb = X + (ar * ldx + kr);
    const cx<T>* yq = Y + (kr * ldy + by);
    const int sy = 4 * ldy;
    cx<T> xa[2][G], yb[2][G];
    auto load = [&](int g, int b) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int ks = g * G + u, t = 4 * ks + kr;
            xa[b][u] = (t < kd && okx) ? xb[4 * ks] : czero<T>();
            yb[b][u] = (t < kd && oky) ? yq[ks * sy] : czero<T>();
        }
    };
    load(0, 0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG)
            load(g + 1, (g + 1) & 1);
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const cx<T> a = xa[g & 1][u], b = yb[g & 1][u];
            cr = MF<T>::mma(a.r, b.r, cr);
            cr = MF<T>::mma(-a.i, b.i, cr);
            ci = MF<T>::mma(a.r, b.i, ci);
            ci = MF<T>::mma(a.i, b.r, ci);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ----------------------------------------------------------------- k_elim_w

template <class T, int MT>
__global__ __launch_bounds__(64, (col_waves<T, MT>())) void k_elim_w(const Seg* __restrict__ segs, int nseg,
                                               int64_t total, const cx<T>* __restrict__ inA,
                                               const cx<T>* __restrict__ inB,
                                               const cx<T>* __restrict__ iny,
                                               cx<T>* __restrict__ W,
                                               unsigned long long* __restrict__ flags,
                                               int with_mat, int with_rhs)
{
    static_assert(MT <= 32, "register-resident columns");
    constexpr int NP = MT * (MT + 1) / 2;
    constexpr int CH = MT < 8 ? MT : 8; // columns of B_p staged per chunk
    constexpr int CHN = MT / CH;
    __shared__ cx<T> sL[NP];
    __shared__ T sInv[MT];
    __shared__ cx<T> sT[MT * (CH + 1)];
    __shared__ int sFail;
    const int lane = threadIdx.x;

    {
        const int64_t w = blockIdx.x;
        if (w >= total)
            return;
        const Seg& s = segs[find_seg(segs, nseg, w)];
        const int64_t t = w - s.w0;
        const int p = s.e0 + (int)t * s.es;
        const int m = s.m, k = s.k, d = s.d;
        const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
        const int np = m * (m + 1) / 2;
        const bool hasPrev = p - d >= 0, hasNext = p + d < s.n;
        if ((flags[s.sys] >> 40) < (unsigned long long)s.level)
            return;
        cx<T>* Lg = W + s.oL + t * mm;
        __syncthreads();
        if (with_mat) {
            const cx<T>* Ap = inA + s.oA + (int64_t)p * mm;
            for (int e = lane; e < np; e += 64) {
                const int r = tri_row(e), c = e - r * (r + 1) / 2;
                sL[e] = Ap[r * m + c];
            }
            if (lane == 0)
                sFail = 0;
            __syncthreads();
            // right-looking Cholesky, packed lower triangle
            for (int c = 0; c < m; ++c) {
                const int dc = c * (c + 1) / 2 + c;
                const T dg = sL[dc].r;
                const T sq = sqrt(dg);
                const T inv = T(1) / sq;
                for (int r = c + 1 + lane; r < m; r += 64) {
                    cx<T> v = sL[r * (r + 1) / 2 + c];
                    v.r *= inv;
                    v.i *= inv;
                    sL[r * (r + 1) / 2 + c] = v;
                }
                __syncthreads();
                if (lane == 0) {
                    sL[dc] = cx<T>{sq, T(0)};
                    sInv[c] = inv;
                    if (!(dg > T(0)))
                        sFail = 1;
                }
                const int nt = m - c - 1;
                for (int e = lane; e < nt * (nt + 1) / 2; e += 64) {
                    const int rr = tri_row(e), qq = e - rr * (rr + 1) / 2;
                    const int r = c + 1 + rr, q = c + 1 + qq;
                    cx<T> v = sL[r * (r + 1) / 2 + q];
                    msub_cb(v, sL[r * (r + 1) / 2 + c], sL[q * (q + 1) / 2 + c]);
                    sL[r * (r + 1) / 2 + q] = v;
                }
                __syncthreads();
            }
            if (lane == 0 && sFail)
                atomicMin(&flags[s.sys], fail_key(s.level, s.ob0 + s.obs * p));
            for (int e = lane; e < np; e += 64)
                Lg[e] = sL[e];
        } else {
            for (int e = lane; e < np; e += 64)
                sL[e] = Lg[e];
            __syncthreads();
            for (int c = lane; c < m; c += 64)
                sInv[c] = T(1) / sL[c * (c + 1) / 2 + c].r;
        }
        __syncthreads();

        // forward substitutions, one lane per column of [B_p^H | B_{p-d} | y_p]
        const int nP = (with_mat && hasNext) ? m : 0;
        const int nQ = (with_mat && hasPrev) ? m : 0;
        const int nY = with_rhs ? k : 0;
        const int ncol = nP + nQ + nY;
        const cx<T>* Bp = inB + s.oB + (int64_t)p * mm;
        const cx<T>* Bq = inB + s.oB + (int64_t)(p - d) * mm;
        const cx<T>* yp = iny + s.oy + (int64_t)p * mk;
        for (int vc0 = 0; vc0 < ncol; vc0 += 64) {
            const int vc = vc0 + lane;
            const bool act = vc < ncol;
            const int src = vc < nP ? 0 : (vc < nP + nQ ? 1 : 2);
            const int col = src == 0 ? vc : (src == 1 ? vc - nP : vc - nP - nQ);
            cx<T> x[MT];
#pragma unroll
            for (int r = 0; r < MT; ++r)
                x[r] = czero<T>();
            if (vc0 == 0 && nP > 0) {
                // column col of B_p^H is the conjugate of row col of B_p: stage
                // CH columns of B_p at a time (coalesced rows), then each lane
                // picks its row
#pragma unroll
                for (int ch = 0; ch < CHN; ++ch) {
                    __syncthreads();
                    for (int e = lane; e < m * CH; e += 64) {
                        const int row = e / CH, j = e % CH, c2 = ch * CH + j;
                        sT[row * (CH + 1) + j] = c2 < m ? Bp[row * m + c2] : czero<T>();
                    }
                    __syncthreads();
                    if (src == 0) {
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const cx<T> v = sT[col * (CH + 1) + j];
                            x[ch * CH + j] = cx<T>{v.r, -v.i};
                        }
                    }
                }
            }
            if (act && src == 1) {
#pragma unroll
                for (int r = 0; r < MT; ++r)
                    if (r < m)
                        x[r] = Bq[r * m + col];
            } else if (act && src == 2) {
#pragma unroll
                for (int r = 0; r < MT; ++r)
                    if (r < m)
                        x[r] = yp[r * k + col];
            }
#pragma unroll
            for (int r = 0; r < MT; ++r) {
                if (r < m) {
                    cx<T> v = x[r];
#pragma unroll
                    for (int u = 0; u < r; ++u)
                        msub(v, sL[r * (r + 1) / 2 + u], x[u]);
                    const T iv = sInv[r];
                    v.r *= iv;
                    v.i *= iv;
                    x[r] = v;
                }
            }
            if (act) {
                cx<T>* out = src == 0 ? W + s.oP + t * mm
                                      : (src == 1 ? W + s.oQ + t * mm : W + s.og + t * mk);
                const int ld = src == 2 ? k : m;
#pragma unroll
                for (int r = 0; r < MT; ++r)
                    if (r < m)
                        out[r * ld + col] = x[r];
            }
        }
    }
}

// --------------------------------------------------------------- k_reduce_m

template <class T, int MT>
__global__ __launch_bounds__(64, (MT >= 64 ? 2 : 4)) void k_reduce_m(const Seg* __restrict__ segs, int nseg,
                                                 int64_t total, const cx<T>* __restrict__ inA,
                                                 const cx<T>* __restrict__ iny,
                                                 cx<T>* __restrict__ W,
                                                 const unsigned long long* __restrict__ flags,
                                                 int with_mat, int with_rhs)
{
    using v4 = typename MF<T>::v4;
    constexpr int NT16 = MT / 16, KS = MT / 4;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;

    {
        const int64_t w = blockIdx.x;
        if (w >= total)
            return;
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
            return;
        const cx<T>* Pl = W + s.oP + tl * mm;
        const cx<T>* Qr = W + s.oQ + tr * mm;
        const cx<T>* Pr = W + s.oP + tr * mm;
        if (with_mat) {
            const cx<T>* Aq = inA + s.oA + q * mm;
            cx<T>* Vo = W + s.oAo + oi * mm;
#pragma unroll 1
            for (int ti = 0; ti < NT16; ++ti) {
                if (16 * ti >= m)
                    break;
#pragma unroll 1
                for (int tj = 0; tj <= ti; ++tj) {
                    v4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
                    if (hasL)
                        tile_hn<T, KS>(cr, ci, Pl, m, m, 16 * ti, Pl, m, m, 16 * tj, m);
                    if (hasR)
                        tile_hn<T, KS>(cr, ci, Qr, m, m, 16 * ti, Qr, m, m, 16 * tj, m);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = 16 * ti + MF<T>::row(kr, v), j = 16 * tj + cc;
                        if (i < m && j <= i) {
                            const cx<T> a = Aq[i * m + j];
                            cx<T> o{a.r - cr[v], a.i - ci[v]};
                            if (i == j)
                                o.i = T(0);
                            Vo[i * m + j] = o;
                        }
                    }
                }
            }
            if (hasR && r + d < n) {
                cx<T>* Fo = W + s.oBo + oi * mm;
    #pragma unroll 1
            for (int ti = 0; ti < NT16; ++ti) {
                    if (16 * ti >= m)
                        break;
#pragma unroll 1
                    for (int tj = 0; tj < NT16; ++tj) {
                        if (16 * tj >= m)
                            break;
                        v4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
                        tile_hn<T, KS>(cr, ci, Pr, m, m, 16 * ti, Qr, m, m, 16 * tj, m);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = 16 * ti + MF<T>::row(kr, v), j = 16 * tj + cc;
                            if (i < m && j < m)
                                Fo[i * m + j] = cx<T>{-cr[v], -ci[v]};
                        }
                    }
                }
            }
        }
        if (with_rhs) {
            const cx<T>* gl = W + s.og + tl * mk;
            const cx<T>* gr = W + s.og + tr * mk;
            const cx<T>* yq = iny + s.oy + q * mk;
            cx<T>* vo = W + s.oyo + oi * mk;
#pragma unroll 1
            for (int ti = 0; ti < NT16; ++ti) {
                if (16 * ti >= m)
                    break;
#pragma unroll 1
                for (int c0 = 0; c0 < k; c0 += 16) {
                    v4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
                    if (hasL)
                        tile_hn<T, KS>(cr, ci, Pl, m, m, 16 * ti, gl, k, k, c0, m);
                    if (hasR)
                        tile_hn<T, KS>(cr, ci, Qr, m, m, 16 * ti, gr, k, k, c0, m);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = 16 * ti + MF<T>::row(kr, v), c = c0 + cc;
                        if (i < m && c < k) {
                            const cx<T> a = yq[i * k + c];
                            vo[i * k + c] = cx<T>{a.r - cr[v], a.i - ci[v]};
                        }
                    }
                }
            }
        }
    }
}

// ----------------------------------------------------------------- k_back_m

template <class T, int MT>
__global__ __launch_bounds__(64, (col_waves<T, MT>())) void k_back_m(const Seg* __restrict__ segs, int nseg,
                                               int64_t total, const cx<T>* __restrict__ W,
                                               cx<T>* __restrict__ X,
                                               const unsigned long long* __restrict__ flags)
{
    static_assert(MT % 16 == 0 && MT <= 32, "tile and register limits");
    using v4 = typename MF<T>::v4;
    constexpr int NP = MT * (MT + 1) / 2, KS = MT / 4, NT16 = MT / 16, WC = 16;
    __shared__ cx<T> sL[NP];
    __shared__ T sInv[MT];
    __shared__ cx<T> sW[MT * (WC + 1)];
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;

    {
        const int64_t w = blockIdx.x;
        if (w >= total)
            return;
        const Seg& s = segs[find_seg(segs, nseg, w)];
        const int64_t t = w - s.w0;
        const int p = s.e0 + (int)t * s.es;
        const int m = s.m, k = s.k, d = s.d;
        const bool hasPrev = p - d >= 0, hasNext = p + d < s.n;
        const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
        cx<T>* xp = X + s.ox + (s.xo + s.xs * p) * mk;
        if (flags[s.sys] != kNoFail) {
            const T nan = T(NAN);
            for (int e = lane; e < m * k; e += 64)
                xp[e] = cx<T>{nan, nan};
            return;
        }
        const cx<T>* xm = X + s.ox + (s.xo + s.xs * (p - d)) * mk;
        const cx<T>* xn = X + s.ox + (s.xo + s.xs * (p + d)) * mk;
        const cx<T>* L = W + s.oL + t * mm;
        const cx<T>* P = W + s.oP + t * mm;
        const cx<T>* Q = W + s.oQ + t * mm;
        const cx<T>* g = W + s.og + t * mk;
        __syncthreads();
        for (int e = lane; e < m * (m + 1) / 2; e += 64)
            sL[e] = L[e];
        __syncthreads();
        for (int c = lane; c < m; c += 64)
            sInv[c] = T(1) / sL[c * (c + 1) / 2 + c].r;
        for (int c0 = 0; c0 < k; c0 += WC) {
            const int cw = min(WC, k - c0);
            __syncthreads();
            for (int ti = 0; ti < NT16; ++ti) {
                if (16 * ti >= m)
                    break;
                v4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
                if (hasPrev)
                    tile_nn<T, KS>(cr, ci, Q, m, m, 16 * ti, xm + c0, k, cw, 0, m);
                if (hasNext)
                    tile_nn<T, KS>(cr, ci, P, m, m, 16 * ti, xn + c0, k, cw, 0, m);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * ti + MF<T>::row(kr, v);
                    if (i < m && cc < cw) {
                        const cx<T> a = g[i * k + c0 + cc];
                        sW[i * (WC + 1) + cc] = cx<T>{a.r - cr[v], a.i - ci[v]};
                    }
                }
            }
            __syncthreads();
            if (lane < cw) {
                cx<T> x[MT];
#pragma unroll
                for (int r = 0; r < MT; ++r)
                    x[r] = r < m ? sW[r * (WC + 1) + lane] : czero<T>();
#pragma unroll
                for (int r = MT - 1; r >= 0; --r) {
                    if (r < m) {
                        cx<T> v = x[r];
#pragma unroll
                        for (int u = r + 1; u < MT; ++u)
                            if (u < m)
                                msub_ca(v, sL[u * (u + 1) / 2 + r], x[u]);
                        const T iv = sInv[r];
                        v.r *= iv;
                        v.i *= iv;
                        x[r] = v;
                    }
                }
#pragma unroll
                for (int r = 0; r < MT; ++r)
                    if (r < m)
                        xp[r * k + c0 + lane] = x[r];
            }
        }
    }
}

} // namespace crs
