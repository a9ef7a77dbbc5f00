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
//   k_elim_mf   (8 < m <= 32) the Cholesky with each row's dot products
//               split over the wave's lane groups, then the substitutions
//               on MFMA with the inverses of the 16 x 16 diagonal tiles.
//   k_back_mf   w = g - Q x_{p-d} - P x_{p+d} on MFMA, then L^H x = w tile by
//               tile on MFMA with the inverse diagonal tiles.
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

// *p where ok, else zero.  The load is issued in every lane (from q, a valid
// address, where ok is false), so no branch surrounds it and the compiler's
// count of the wave's memory operations in flight stays exact: a wait for
// one group of a software pipeline's loads then does not also wait for the
// group issued after it.
template <class T>
__device__ __forceinline__ cx<T> ld_or0(const cx<T>* p, const cx<T>* q, bool ok)
{
    const cx<T> v = *(ok ? p : q);
    return ok ? v : czero<T>();
}

// 1 / sqrt(d) from the hardware reciprocal square root and one Newton step
// (relative error about the unit roundoff); NaN for d < 0, inf for d = 0.
__device__ __forceinline__ double rsqrt_nr(double d)
{
    const double r = __builtin_amdgcn_rsq(d);
    return r * fma(-0.5 * d * r, r, 1.5);
}
__device__ __forceinline__ float rsqrt_nr(float d)
{
    const float r = __builtin_amdgcn_rsqf(d);
    return r * fmaf(-0.5f * d * r, r, 1.5f);
}

// Value of x in lane l (uniform l) through the scalar registers.
__device__ __forceinline__ float lane_bcast(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_bcast(double x, int l)
{
    const long long v = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(v >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <class T>
__device__ __forceinline__ cx<T> lane_bcast(const cx<T> x, int l)
{
    return cx<T>{lane_bcast(x.r, l), lane_bcast(x.i, l)};
}

// Orders the LDS accesses of one wave: stores before the call are seen by
// loads after it from any lane of the same wave (a wave's LDS operations
// complete in order; the fences keep the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// x[l] + x[l ^ 32] in every lane l, through the gfx950 swap of the upper
// half of one register with the lower half of another (one VALU instruction
// per dword, no LDS round trip).  Swapping x with itself leaves one result
// holding the lower half's values in both halves and the other the upper
// half's, so their sum is the same, bit for bit, in every lane.
__device__ __forceinline__ float sum_xor32(float x)
{
    const unsigned v = __float_as_uint(x);
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double sum_xor32(double x)
{
    const unsigned long long v = (unsigned long long)__double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
// x[l] + x[l ^ 16], the same way with the swap of odd and even 16-lane rows.
__device__ __forceinline__ float sum_xor16(float x)
{
    const unsigned v = __float_as_uint(x);
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double sum_xor16(double x)
{
    const unsigned long long v = (unsigned long long)__double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
    return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
           __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// MFMA 16x16x4 lane layout (wave64, checked on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator register v of lane l
// holds D[row][l % 16] with row = 4 (l / 16) + v for the f32 instruction and
// row = l / 16 + 4 v for the f64 instruction (MF<T>::row).

// Operands are loaded four k-steps at a time, one group ahead of the MFMAs
// that consume the previous group; the scheduling barrier keeps the compiler
// from hoisting every load of the tile to the top (register pressure).
constexpr int kGroup = 4;

// Accumulators of the three-multiplication (3M) complex product: with
// a = op(A), b = op(B) split into real and imaginary parts,
//   t1 += Re a Re b,  t2 += Im a Im b,  t3 += (Re a + Im a)(Re b + Im b),
// and the product is Re = t1 - t2, Im = t3 - t1 - t2: three real MFMAs per
// complex contraction step instead of four.  The real part is the 4M one;
// the imaginary part carries an absolute error of a few units of roundoff
// times sum_t (|Re a| + |Im a|)(|Re b| + |Im b|) (normwise stable, not
// componentwise; Higham, Accuracy and Stability of Numerical Algorithms,
// Section 23.2.4).  For real data t2 = 0 and t3 = t1 bit for bit, so the
// imaginary part is exactly zero.
//
// RE (real data: every imaginary part is zero): only t1 is formed, one real
// MFMA per contraction step, Re = t1 and Im = 0 -- the same values the 3M
// form gives for real data (t2 = 0, t3 = t1), with a third of the MFMAs.
template <class T, int RM, int RN, bool RE = false>
struct Acc3 {
    using v4 = typename MF<T>::v4;
    v4 t1[RM][RN], t2[RE ? 1 : RM][RE ? 1 : RN], t3[RE ? 1 : RM][RE ? 1 : RN];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int i = 0; i < RM; ++i)
#pragma unroll
            for (int j = 0; j < RN; ++j) {
                t1[i][j] = v4{0, 0, 0, 0};
                if constexpr (!RE)
                    t2[i][j] = t3[i][j] = v4{0, 0, 0, 0};
            }
    }
    __device__ __forceinline__ T re(int i, int j, int v) const
    {
        if constexpr (RE)
            return t1[i][j][v];
        else
            return t1[i][j][v] - t2[i][j][v];
    }
    __device__ __forceinline__ T im(int i, int j, int v) const
    {
        if constexpr (RE)
            return T(0);
        else
            return t3[i][j][v] - t1[i][j][v] - t2[i][j][v];
    }
    // acc(i, j) += a b for one contraction step of real-pair operands
    __device__ __forceinline__ void step(int i, int j, T ar, T ai, T br, T bi)
    {
        t1[i][j] = MF<T>::mma(ar, br, t1[i][j]);
        if constexpr (!RE) {
            t2[i][j] = MF<T>::mma(ai, bi, t2[i][j]);
            t3[i][j] = MF<T>::mma(ar + ai, br + bi, t3[i][j]);
        }
    }
};

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
            xa[b][u] = ld_or0(xb + ks * sx, X, t < kd && okx);
            yb[b][u] = ld_or0(yq + ks * sy, Y, t < kd && oky);
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
            xa[b][u] = ld_or0(xb + 4 * ks, X, t < kd && okx);
            yb[b][u] = ld_or0(yq + ks * sy, Y, t < kd && oky);
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

// acc += X Y as tile_nn, in the 3M form.
template <class T, int KS>
__device__ __forceinline__ void tile_nn3(Acc3<T, 1, 1>& acc, const cx<T>* __restrict__ X, int ldx,
                                         int nrx, int rx0, const cx<T>* __restrict__ Y, int ldy,
                                         int ncy, int cy0, int kd)
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
            xa[b][u] = ld_or0(xb + 4 * ks, X, t < kd && okx);
            yb[b][u] = ld_or0(yq + ks * sy, Y, t < kd && oky);
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
            acc.t1[0][0] = MF<T>::mma(a.r, b.r, acc.t1[0][0]);
            acc.t2[0][0] = MF<T>::mma(a.i, b.i, acc.t2[0][0]);
            acc.t3[0][0] = MF<T>::mma(a.r + a.i, b.r + b.i, acc.t3[0][0]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ----------------------------------------------------------------- k_elim_w

template <class T, int MT, class EI = cx<T>>
__global__ __launch_bounds__(64, (col_waves<T, MT>())) void k_elim_w(const Seg* __restrict__ segs, int nseg,
                                               int64_t total, const EI* __restrict__ inA,
                                               const EI* __restrict__ inB,
                                               const EI* __restrict__ iny,
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
            const EI* Ap = inA + s.oA + (int64_t)p * mm;
            for (int e = lane; e < np; e += 64) {
                const int r = tri_row(e), c = e - r * (r + 1) / 2;
                sL[e] = cvt<T>(Ap[r * m + c]);
            }
            __syncthreads();
            // left-looking Cholesky: lane r < m keeps row r in registers; at
            // step c every row forms its dot product with row c of L (read by
            // broadcast from LDS), lane c's result gives the pivot, rows
            // below it get L[r][c], and column c is published to LDS
            cx<T> a[MT];
            const int rl = lane < m ? lane : 0;
#pragma unroll
            for (int u = 0; u < MT; ++u)
                a[u] = (u <= rl) ? sL[rl * (rl + 1) / 2 + u] : czero<T>();
            __syncthreads();
            bool fail = false;
#pragma unroll
            for (int c = 0; c < MT; ++c) {
                if (c < m) {
                    cx<T> s0 = czero<T>(), s1 = czero<T>();
#pragma unroll
                    for (int u = 0; u + 1 < c; u += 2) {
                        msub_cb(s0, a[u], sL[c * (c + 1) / 2 + u]);
                        msub_cb(s1, a[u + 1], sL[c * (c + 1) / 2 + u + 1]);
                    }
                    if (c & 1)
                        msub_cb(s0, a[c - 1], sL[c * (c + 1) / 2 + c - 1]);
                    // s = -(sum_u L[r][u] conj(L[c][u])); the pivot is lane c's
                    const cx<T> v{a[c].r + s0.r + s1.r, a[c].i + s0.i + s1.i};
                    const T dg = __shfl(v.r, c);
                    const T inv = rsqrt_nr(dg);
                    const T sq = dg * inv;
                    fail |= !(dg > T(0));
                    if (lane == c)
                        a[c] = cx<T>{sq, inv}; // inverse pivot kept in the imaginary slot
                    else
                        a[c] = cx<T>{v.r * inv, v.i * inv};
                    if (lane >= c && lane < m)
                        sL[lane * (lane + 1) / 2 + c] = a[c];
                    if (lane == 0)
                        sInv[c] = inv;
                    __syncthreads();
                }
                // keep the next step's loads from being hoisted (register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
            if (lane == 0)
                sFail = fail;
            if (lane == 0 && sFail)
                atomicMin(&flags[s.sys], fail_key(s.level, s.ob0 + s.obs * p));
            for (int e = lane; e < np; e += 64)
                Lg[e] = sL[e];
        } else {
            for (int e = lane; e < np; e += 64)
                sL[e] = Lg[e];
            __syncthreads();
            for (int c = lane; c < m; c += 64)
                sInv[c] = sL[c * (c + 1) / 2 + c].i;
        }
        __syncthreads();

        // forward substitutions, one lane per column of [B_p^H | B_{p-d} | y_p]
        const int nP = (with_mat && hasNext) ? m : 0;
        const int nQ = (with_mat && hasPrev) ? m : 0;
        const int nY = with_rhs ? k : 0;
        const int ncol = nP + nQ + nY;
        const EI* Bp = inB + s.oB + (int64_t)p * mm;
        const EI* Bq = inB + s.oB + (int64_t)(p - d) * mm;
        const EI* yp = iny + s.oy + (int64_t)p * mk;
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
                        sT[row * (CH + 1) + j] = c2 < m ? cvt<T>(Bp[row * m + c2]) : czero<T>();
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
                        x[r] = cvt<T>(Bq[r * m + col]);
            } else if (act && src == 2) {
#pragma unroll
                for (int r = 0; r < MT; ++r)
                    if (r < m)
                        x[r] = cvt<T>(yp[r * k + col]);
            }
            // forward substitution, L by broadcast from LDS; each row's sum
            // runs on four independent chains
#pragma unroll
            for (int r = 0; r < MT; ++r) {
                if (r < m) {
                    cx<T> v[4] = {x[r], czero<T>(), czero<T>(), czero<T>()};
#pragma unroll
                    for (int u = 0; u < r; ++u)
                        msub(v[u & 3], sL[r * (r + 1) / 2 + u], x[u]);
                    const T iv = sInv[r];
                    x[r] = cx<T>{((v[0].r + v[1].r) + (v[2].r + v[3].r)) * iv,
                                 ((v[0].i + v[1].i) + (v[2].i + v[3].i)) * iv};
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

// Replaces the packed lower triangle L (m <= 16 S, diagonal {L_cc, 1/L_cc})
// held in LDS by the inverses D_I = L_II^{-1} of its 16 x 16 diagonal tiles,
// sL[I * 256 + q * 16 + j] = D_I[q][j]: lane j < 16 S forms column j & 15 of
// D_{j / 16} by forward substitution (padded rows are identity rows).  Every
// lane of the work-group must call it.
template <class T, int S>
__device__ __forceinline__ void inverse_tiles_lds(cx<T>* sL, int m)
{
    const int lane = threadIdx.x & 63;
    const int I0 = (lane >> 4) < S ? (lane >> 4) : 0, jj = lane & 15;
    cx<T> z[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int gq = 16 * I0 + q;
        cx<T> v = q == jj ? cx<T>{T(1), T(0)} : czero<T>();
        if (gq < m) {
            const int base = gq * (gq + 1) / 2 + 16 * I0;
#pragma unroll
            for (int u = 0; u < q; ++u)
                msub(v, sL[base + u], z[u]);
            const T iq = sL[base + q].i;
            v = cx<T>{v.r * iq, v.i * iq};
        }
        z[q] = v;
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads(); // every read of L in LDS is done
    if (lane < 16 * S) {
#pragma unroll
        for (int q = 0; q < 16; ++q)
            sL[I0 * 256 + q * 16 + jj] = z[q];
    }
    __syncthreads();
}

// ---------------------------------------------------------------- k_elim_mf

// Elimination for block sizes 8 < m <= 32 with the forward substitutions on
// MFMA.  After the Cholesky (its dot products split over the lane groups) the
// inverses D_I = L_II^{-1} of the 16 x 16 diagonal tiles are formed, and each
// 16-column strip G of [B_p^H | B_{p-d} | y_p] is solved tile by tile,
// X_0 = D_0 G_0 and
// X_1 = D_1 (G_1 - L_10 X_0): register v of a lane's accumulator holds row
// MF::row(kr, v) of its column, which is the right operand of contraction
// step v when the left operand supplies column MF::row(kr, v), so the
// products chain through the accumulators.  Right-hand sides are read from
// memory straight into that layout, each next strip while the current one is
// solved.
//
// The register budget is held to three waves per SIMD (168 VGPRs for FP64,
// m = 32, no spills), which hides more of each block's latency than the
// 196 registers the compiler would take on its own.
//
// nsplit waves share a block: wave sp solves strips sp, sp + nsplit, ...
// Each of them factors the block itself (a few microseconds of latency,
// no cross-wave synchronisation); wave 0 alone stores L and raises the
// breakdown flag.  Levels with few blocks use nsplit > 1 to shorten the
// chain of strips that one wave walks through.
template <class T, int MT, class EI = cx<T>>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_elim_mf(const Seg* __restrict__ segs, int nseg,
                                                   int64_t total, int nsplit,
                                                   const EI* __restrict__ inA,
                                                   const EI* __restrict__ inB,
                                                   const EI* __restrict__ iny,
                                                   cx<T>* __restrict__ W,
                                                   unsigned long long* __restrict__ flags,
                                                   int with_mat, int with_rhs)
{
    static_assert(MT == 16 || MT == 32, "one or two 16-row tiles");
    using v4 = typename MF<T>::v4;
    constexpr int S = MT / 16;
    constexpr int NP = MT * (MT + 1) / 2;
    constexpr int NS = NP > S * 256 ? NP : S * 256;
    __shared__ cx<T> sL[NS]; // packed L, later the D tiles
    __shared__ int sFail;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
    const int64_t w = blockIdx.x / nsplit;
    const int sp = (int)(blockIdx.x - w * nsplit);
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
        return; // broke down at an earlier level: nothing left to do
    cx<T>* Lg = W + s.oL + t * mm;

    // strips: S of B_p^H (into P), S of B_{p-d} (into Q), ceil(k / 16) of y_p
    const int nP = (with_mat && hasNext) ? S : 0;
    const int nQ = (with_mat && hasPrev) ? S : 0;
    const int nst = nP + nQ + (with_rhs ? (k + 15) / 16 : 0);
    const EI* Bp = inB + s.oB + (int64_t)p * mm;
    const EI* Bq = inB + s.oB + (int64_t)(p - d) * mm;
    const EI* yp = iny + s.oy + (int64_t)p * mk;
    // element (r, c) of strip st's source is base[r * sr + c * sc], conjugated
    // for B_p^H
#define CRS_LOAD_STRIP(st, g)                                                                      \
    do {                                                                                           \
        const int src_ = (st) < nP ? 0 : ((st) < nP + nQ ? 1 : 2);                                 \
        const int c_ = 16 * (src_ == 0 ? (st) : (src_ == 1 ? (st) - nP : (st) - nP - nQ)) + cc;    \
        const EI* base_ = src_ == 0 ? Bp : (src_ == 1 ? Bq : yp);                              \
        const int sr_ = src_ == 0 ? 1 : (src_ == 1 ? m : k), sc_ = src_ == 0 ? m : 1;               \
        const bool okc_ = c_ < (src_ == 2 ? k : m);                                                \
        const T cj_ = src_ == 0 ? T(-1) : T(1);                                                    \
        const EI* col_ = base_ + (okc_ ? c_ : 0) * sc_;                                        \
        _Pragma("unroll") for (int I_ = 0; I_ < S; ++I_)                                           \
            _Pragma("unroll") for (int v_ = 0; v_ < 4; ++v_)                                       \
            {                                                                                      \
                const int r_ = 16 * I_ + MF<T>::row(kr, v_);                                       \
                const bool ok_ = okc_ && r_ < m;                                                   \
                const cx<T> x_ = cvt<T>(col_[(ok_ ? r_ : 0) * sr_]);                               \
                g[I_][v_] = ok_ ? cx<T>{x_.r, cj_ * x_.i} : czero<T>();                            \
            }                                                                                      \
    } while (0)
    cx<T> gn[S][4];

    // a lane's elements e = lane + 64 q of the packed lower triangle, all
    // loads issued before the first is used (one round trip, not NE); lanes
    // past the end load and store the last element (the same value), so no
    // branch holds a load back
    constexpr int NE = (NP + 63) / 64;
    if (with_mat) {
        const EI* Ap = inA + s.oA + (int64_t)p * mm;
        EI av[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = min(lane + 64 * q, np - 1), r = tri_row(e);
            av[q] = Ap[r * m + e - r * (r + 1) / 2];
        }
#pragma unroll
        for (int q = 0; q < NE; ++q)
            sL[min(lane + 64 * q, np - 1)] = cvt<T>(av[q]);
        __syncthreads();
        // left-looking Cholesky with each dot product split over the
        // G = 64 / MT lane groups: lane g MT + r keeps the entries u = G j + g
        // of row r (b[j]) and sums the terms u = g (mod G); the groups'
        // partial sums meet by lane swaps.  Each finished entry L[r][c] goes
        // to LDS in place of A's (row r is read only by its own lanes), from
        // where every later column c' reads row c' by broadcast.
        constexpr int G = 64 / MT, NB = MT / G;
        const int r = lane % MT, grp = lane / MT;
        const int rl = r < m ? r : 0;
        cx<T> b[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int u = G * j + grp;
            b[j] = (u <= rl) ? sL[rl * (rl + 1) / 2 + u] : czero<T>();
        }
        bool fail = false;
#pragma unroll
        for (int c = 0; c < MT; ++c) {
            if (c < m) {
                // row c of L (entries u < c final): every read issued before
                // the first product, so the LDS latency is paid once a column
                const cx<T>* rc = sL + c * (c + 1) / 2;
                cx<T> lc[NB];
#pragma unroll
                for (int j = 0; j < c / G; ++j)
                    lc[j] = rc[G * j + grp];
                if (c % G) // groups g >= c mod G read entry 0 and add zero
                    lc[c / G] = rc[grp < c % G ? G * (c / G) + grp : 0];
                __builtin_amdgcn_sched_barrier(0);
                cx<T> s0 = czero<T>(), s1 = czero<T>();
#pragma unroll
                for (int j = 0; j < c / G; ++j) {
                    if (j & 1)
                        msub_cb(s1, b[j], lc[j]);
                    else
                        msub_cb(s0, b[j], lc[j]);
                }
                if (c % G) { // the last terms: groups g < c mod G only
                    const int j = c / G;
                    msub_cb(s0, grp < c % G ? b[j] : czero<T>(), lc[j]);
                }
                cx<T> sm{s0.r + s1.r, s0.i + s1.i};
                if (G == 4) {
                    sm.r = sum_xor16(sm.r);
                    sm.i = sum_xor16(sm.i);
                }
                sm.r = sum_xor32(sm.r);
                sm.i = sum_xor32(sm.i);
                // group c mod G holds entry c of every row
                const int gc = c % G, jc = c / G;
                const cx<T> v{b[jc].r + sm.r, b[jc].i + sm.i};
                const T dg = lane_bcast(v.r, gc * MT + c);
                const T inv = rsqrt_nr(dg);
                const T sq = dg * inv;
                fail |= !(dg > T(0));
                // inverse pivot kept in the imaginary slot of the diagonal
                const cx<T> l = r == c ? cx<T>{sq, inv} : cx<T>{v.r * inv, v.i * inv};
                if (grp == gc) {
                    b[jc] = l;
                    if (r >= c && r < m)
                        sL[r * (r + 1) / 2 + c] = l;
                }
                wave_lds_sync();
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
        if (lane == 0)
            sFail = fail;
        if (sp == 0) {
            if (lane == 0 && sFail)
                atomicMin(&flags[s.sys], fail_key(s.level, s.ob0 + s.obs * p));
            for (int e = lane; e < np; e += 64)
                Lg[e] = sL[e];
        }
    } else {
        cx<T> lv[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q)
            lv[q] = Lg[min(lane + 64 * q, np - 1)];
#pragma unroll
        for (int q = 0; q < NE; ++q)
            sL[min(lane + 64 * q, np - 1)] = lv[q];
    }
    __syncthreads();

    // left operands: L_10, then the D tiles
    cx<T> aL[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 16 + cc, u = MF<T>::row(kr, v);
        aL[v] = (S == 2 && i < m) ? sL[i * (i + 1) / 2 + u] : czero<T>();
    }
    inverse_tiles_lds<T, S>(sL, m);
    cx<T> aD[S][4];
#pragma unroll
    for (int I = 0; I < S; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            aD[I][v] = sL[I * 256 + cc * 16 + MF<T>::row(kr, v)];

    if (sp < nst)
        CRS_LOAD_STRIP(sp, gn);
#pragma unroll 1
    for (int st = sp; st < nst; st += nsplit) {
        cx<T> g[S][4];
#pragma unroll
        for (int I = 0; I < S; ++I)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                g[I][v] = gn[I][v];
        // the next strip (the current one again after the last): issued in
        // every pass, so the wait for this strip's loads does not wait for it
        CRS_LOAD_STRIP(st + nsplit < nst ? st + nsplit : st, gn);
        // X_0 = D_0 G_0 (3M products, combined before they chain on)
        v4 x0r, x0i;
        {
            Acc3<T, 1, 1> p;
            p.zero();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cx<T> a = aD[0][v], b = g[0][v];
                p.t1[0][0] = MF<T>::mma(a.r, b.r, p.t1[0][0]);
                p.t2[0][0] = MF<T>::mma(a.i, b.i, p.t2[0][0]);
                p.t3[0][0] = MF<T>::mma(a.r + a.i, b.r + b.i, p.t3[0][0]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                x0r[v] = p.re(0, 0, v);
                x0i[v] = p.im(0, 0, v);
            }
        }
        v4 x1r = {0, 0, 0, 0}, x1i = {0, 0, 0, 0};
        if (S == 2) {
            // T = L_10 X_0, then X_1 = D_1 (G_1 - T)
            Acc3<T, 1, 1> p;
            p.zero();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cx<T> a = aL[v];
                p.t1[0][0] = MF<T>::mma(a.r, x0r[v], p.t1[0][0]);
                p.t2[0][0] = MF<T>::mma(a.i, x0i[v], p.t2[0][0]);
                p.t3[0][0] = MF<T>::mma(a.r + a.i, x0r[v] + x0i[v], p.t3[0][0]);
            }
            Acc3<T, 1, 1> q;
            q.zero();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cx<T> a = aD[S - 1][v];
                const T br = g[S - 1][v].r - p.re(0, 0, v), bi = g[S - 1][v].i - p.im(0, 0, v);
                q.t1[0][0] = MF<T>::mma(a.r, br, q.t1[0][0]);
                q.t2[0][0] = MF<T>::mma(a.i, bi, q.t2[0][0]);
                q.t3[0][0] = MF<T>::mma(a.r + a.i, br + bi, q.t3[0][0]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                x1r[v] = q.re(0, 0, v);
                x1i[v] = q.im(0, 0, v);
            }
        }
        const int src = st < nP ? 0 : (st < nP + nQ ? 1 : 2);
        const int c = 16 * (src == 0 ? st : (src == 1 ? st - nP : st - nP - nQ)) + cc;
        const int ld = src == 2 ? k : m;
        cx<T>* out = src == 0 ? W + s.oP + t * mm : (src == 1 ? W + s.oQ + t * mm : W + s.og + t * mk);
        if (c < ld) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r0 = MF<T>::row(kr, v);
                if (r0 < m)
                    out[r0 * ld + c] = cx<T>{x0r[v], x0i[v]};
                if (S == 2 && 16 + r0 < m)
                    out[(16 + r0) * ld + c] = cx<T>{x1r[v], x1i[v]};
            }
        }
    }
}

#undef CRS_LOAD_STRIP

// --------------------------------------------------------------- k_reduce_m

// MFMA operand tile: 16 columns [c0, c0 + 16) of a row-major matrix with
// kd rows, loaded once in the lane layout shared by the A and B operands
// (lane l holds rows 4 s + l / 16, column c0 + l % 16, s < KS).
template <class T, int KS>
struct OpTile {
    cx<T> v[KS];
    __device__ __forceinline__ void load(const cx<T>* __restrict__ X, int ld, int ncol, int c0,
                                         int kd)
    {
        const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
        const bool ok = c0 + cc < ncol;
        const cx<T>* b = X + (kr * ld + c0 + cc);
#pragma unroll
        for (int s = 0; s < KS; ++s)
            v[s] = (ok && 4 * s + kr < kd) ? b[4 * s * ld] : czero<T>();
    }
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int s = 0; s < KS; ++s)
            v[s] = czero<T>();
    }
};

// (cr, ci) += A^H B for operand tiles A (rows of the result) and B (columns).
template <class T, int KS>
__device__ __forceinline__ void mma_hn(typename MF<T>::v4& cr, typename MF<T>::v4& ci,
                                       const OpTile<T, KS>& A, const OpTile<T, KS>& B)
{
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        cr = MF<T>::mma(A.v[s].r, B.v[s].r, cr);
        cr = MF<T>::mma(A.v[s].i, B.v[s].i, cr);
        ci = MF<T>::mma(A.v[s].r, B.v[s].i, ci);
        ci = MF<T>::mma(-A.v[s].i, B.v[s].r, ci);
    }
}

// acc += A^H B for operand tiles A and B in the 3M form.
template <class T, int KS>
__device__ __forceinline__ void mma_hn3(Acc3<T, 1, 1>& acc, const OpTile<T, KS>& A,
                                        const OpTile<T, KS>& B)
{
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const T ar = A.v[s].r, ai = -A.v[s].i, br = B.v[s].r, bi = B.v[s].i;
        acc.t1[0][0] = MF<T>::mma(ar, br, acc.t1[0][0]);
        acc.t2[0][0] = MF<T>::mma(ai, bi, acc.t2[0][0]);
        acc.t3[0][0] = MF<T>::mma(ar + ai, br + bi, acc.t3[0][0]);
    }
}

// Reduced system for a kept block q with eliminated neighbours l, r:
//   A'_q = A_q - P_l^H P_l - Q_r^H Q_r,  B'_q = -P_r^H Q_r,
//   y'_q = y_q - P_l^H g_l - Q_r^H g_r.
// Each 16-column operand tile is loaded from memory once and reused by every
// output tile that needs it (NT16 = MT / 16 tiles per m x m operand).
template <class T, int MT, class EI = cx<T>>
__global__ __launch_bounds__(64, 2) void k_reduce_m(const Seg* __restrict__ segs, int nseg,
                                                    int64_t total, const EI* __restrict__ inA,
                                                    const EI* __restrict__ iny,
                                                    cx<T>* __restrict__ W,
                                                    const unsigned long long* __restrict__ flags,
                                                    int with_mat, int with_rhs)
{
    static_assert(MT == 16 || MT == 32, "one or two operand tiles");
    using v4 = typename MF<T>::v4;
    using Tile = OpTile<T, MT / 4>;
    constexpr int NT16 = MT / 16, NV = NT16 * (NT16 + 1) / 2;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
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
    const cx<T>* gl = W + s.og + tl * mk;
    const cx<T>* gr = W + s.og + tr * mk;
    const v4 z4 = {0, 0, 0, 0};

    // right-hand side columns beyond the first 16 are handled in later chunks
    const int kc0 = with_rhs ? (k < 16 ? k : 16) : 0;
    Tile X[NT16], G;
    Acc3<T, 1, 1> av[NV], ay[NT16];
#pragma unroll
    for (int i = 0; i < NV; ++i)
        av[i].zero();
#pragma unroll
    for (int i = 0; i < NT16; ++i)
        ay[i].zero();

    // phase 1: P_l^H P_l and P_l^H g_l;  phase 2: Q_r^H Q_r and Q_r^H g_r
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
        const bool on = ph == 0 ? hasL : hasR;
        if (!on)
            continue;
        const cx<T>* Xm = ph == 0 ? Pl : Qr;
        const cx<T>* Gm = ph == 0 ? gl : gr;
#pragma unroll
        for (int i = 0; i < NT16; ++i)
            X[i].load(Xm, m, m, 16 * i, m);
        if (kc0)
            G.load(Gm, k, kc0, 0, m);
        if (with_mat) {
#pragma unroll
            for (int i = 0, v = 0; i < NT16; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j, ++v)
                    mma_hn3<T, MT / 4>(av[v], X[i], X[j]);
        }
        if (kc0) {
#pragma unroll
            for (int i = 0; i < NT16; ++i)
                mma_hn3<T, MT / 4>(ay[i], X[i], G);
        }
    }
    // the epilogues load the four A_q or y_q elements of a tile together, in
    // every lane (element 0 stands in), before their stores: one round trip
    // per tile instead of one per element waiting behind the previous store
    if (with_mat) {
        const EI* Aq = inA + s.oA + q * mm;
        cx<T>* Vo = W + s.oAo + oi * mm;
#pragma unroll
        for (int i = 0, v = 0; i < NT16; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j, ++v) {
                cx<T> xa[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = 16 * i + MF<T>::row(kr, u), b = 16 * j + cc;
                    xa[u] = cvt<T>(Aq[(a < m && b <= a) ? a * m + b : 0]);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = 16 * i + MF<T>::row(kr, u), b = 16 * j + cc;
                    if (a < m && b <= a) {
                        cx<T> o{xa[u].r - av[v].re(0, 0, u), xa[u].i - av[v].im(0, 0, u)};
                        if (a == b)
                            o.i = T(0);
                        Vo[a * m + b] = o;
                    }
                }
            }
    }
    if (kc0) {
        const EI* yq = iny + s.oy + q * mk;
        cx<T>* yo = W + s.oyo + oi * mk;
#pragma unroll
        for (int i = 0; i < NT16; ++i) {
            cx<T> xy[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int a = 16 * i + MF<T>::row(kr, u), c = cc;
                xy[u] = cvt<T>(yq[(a < m && c < kc0) ? a * k + c : 0]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int a = 16 * i + MF<T>::row(kr, u), c = cc;
                if (a < m && c < kc0)
                    yo[a * k + c] = cx<T>{xy[u].r - ay[i].re(0, 0, u), xy[u].i - ay[i].im(0, 0, u)};
            }
        }
    }
    // phase 3: B'_q = -P_r^H Q_r (Q_r tiles are still in X when hasR)
    if (with_mat && hasR && r + d < n) {
        Tile Pt[NT16];
#pragma unroll
        for (int i = 0; i < NT16; ++i)
            Pt[i].load(Pr, m, m, 16 * i, m);
        cx<T>* Fo = W + s.oBo + oi * mm;
#pragma unroll
        for (int i = 0; i < NT16; ++i)
#pragma unroll
            for (int j = 0; j < NT16; ++j) {
                Acc3<T, 1, 1> af;
                af.zero();
                mma_hn3<T, MT / 4>(af, Pt[i], X[j]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = 16 * i + MF<T>::row(kr, u), b = 16 * j + cc;
                    if (a < m && b < m)
                        Fo[a * m + b] = cx<T>{-af.re(0, 0, u), -af.im(0, 0, u)};
                }
            }
    }
    // remaining right-hand-side chunks (k > 16)
    if (with_rhs && k > 16) {
        const EI* yq = iny + s.oy + q * mk;
        cx<T>* yo = W + s.oyo + oi * mk;
        for (int c0 = 16; c0 < k; c0 += 16) {
#pragma unroll
            for (int i = 0; i < NT16; ++i) {
                Acc3<T, 1, 1> ac;
                ac.zero();
                if (hasL) {
                    Tile A1, G1;
                    A1.load(Pl, m, m, 16 * i, m);
                    G1.load(gl, k, k, c0, m);
                    mma_hn3<T, MT / 4>(ac, A1, G1);
                }
                if (hasR) {
                    Tile A1, G1;
                    A1.load(Qr, m, m, 16 * i, m);
                    G1.load(gr, k, k, c0, m);
                    mma_hn3<T, MT / 4>(ac, A1, G1);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = 16 * i + MF<T>::row(kr, u), c = c0 + cc;
                    if (a < m && c < k) {
                        const cx<T> x = cvt<T>(yq[a * k + c]);
                        yo[a * k + c] = cx<T>{x.r - ac.re(0, 0, u), x.i - ac.im(0, 0, u)};
                    }
                }
            }
        }
    }
}

// --------------------------------------------------------------- k_reduce_t

template <class T, int MT, class EI = cx<T>>
__global__ __launch_bounds__(64, (MT >= 64 ? 2 : 4)) void k_reduce_t(const Seg* __restrict__ segs, int nseg,
                                                 int64_t total, const EI* __restrict__ inA,
                                                 const EI* __restrict__ iny,
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
            const EI* Aq = inA + s.oA + q * mm;
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
                            const cx<T> a = cvt<T>(Aq[i * m + j]);
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
            const EI* yq = iny + s.oy + q * mk;
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
                            const cx<T> a = cvt<T>(yq[i * k + c]);
                            vo[i * k + c] = cx<T>{a.r - cr[v], a.i - ci[v]};
                        }
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------- k_back_mf

// Back substitution for block sizes 8 < m <= 32 on MFMA: per 16-column strip
// of x_p, w = g - Q x_{p-d} - P x_{p+d} stays in the accumulators and the
// block upper triangular L^H x = w is solved tile by tile,
// x_1 = D_1^H w_1, x_0 = D_0^H (w_0 - L_10^H x_1), with the products chained
// through the accumulators as in k_elim_mf (D_I = L_II^{-1} formed from L).
template <class T, int MT>
__global__ __launch_bounds__(64, 2) void k_back_mf(const Seg* __restrict__ segs, int nseg,
                                                   int64_t total, const cx<T>* __restrict__ W,
                                                   cx<T>* __restrict__ X,
                                                   const unsigned long long* __restrict__ flags,
                                                   cx<double>* __restrict__ U, int upd)
{
    static_assert(MT == 16 || MT == 32, "one or two 16-row tiles");
    using v4 = typename MF<T>::v4;
    constexpr int S = MT / 16, KS = MT / 4;
    constexpr int NP = MT * (MT + 1) / 2;
    constexpr int NS = NP > S * 256 ? NP : S * 256;
    __shared__ cx<T> sL[NS]; // packed L, later the D tiles
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
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
    cx<double>* up = upd ? U + s.oU + p * mk : nullptr;
    if (flags[s.sys] != kNoFail) {
        const T nan = T(NAN);
        for (int e = lane; e < m * k; e += 64) {
            put_x<T>(xp, up, upd ? 1 : 0, e, cx<T>{nan, nan});
            if (upd && hasNext)
                put_x<T>(xp, up + d * mk, 1, e, cx<T>{nan, nan});
        }
        return;
    }
    const cx<T>* xm = X + s.ox + (s.xo + s.xs * (p - d)) * mk;
    const cx<T>* xn = X + s.ox + (s.xo + s.xs * (p + d)) * mk;
    if (upd && hasNext)
        put_kept<T>(xn, up + d * mk, upd, lane, mk, 64);
    const cx<T>* L = W + s.oL + t * mm;
    const cx<T>* P = W + s.oP + t * mm;
    const cx<T>* Q = W + s.oQ + t * mm;
    const cx<T>* g = W + s.og + t * mk;
    {
        // packed L: a lane's NE elements loaded together (lanes past the end
        // load and store the last one), one round trip
        constexpr int NE = (NP + 63) / 64;
        const int np = m * (m + 1) / 2;
        cx<T> lv[NE];
#pragma unroll
        for (int q = 0; q < NE; ++q)
            lv[q] = L[min(lane + 64 * q, np - 1)];
#pragma unroll
        for (int q = 0; q < NE; ++q)
            sL[min(lane + 64 * q, np - 1)] = lv[q];
    }
    __syncthreads();
    // left operands: (L_10^H)[i][u] = conj(L[16 + u][i]), then (D_I^H)[i][u] =
    // conj(D_I[u][i])
    cx<T> aLh[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int u = 16 + MF<T>::row(kr, v);
        const cx<T> a = (S == 2 && u < m) ? sL[u * (u + 1) / 2 + cc] : czero<T>();
        aLh[v] = cx<T>{a.r, -a.i};
    }
    inverse_tiles_lds<T, S>(sL, m);
    cx<T> aDh[S][4];
#pragma unroll
    for (int I = 0; I < S; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const cx<T> a = sL[I * 256 + MF<T>::row(kr, v) * 16 + cc];
            aDh[I][v] = cx<T>{a.r, -a.i};
        }
#pragma unroll 1
    for (int c0 = 0; c0 < k; c0 += 16) {
        const int cw = min(16, k - c0);
        // w_I = g_I - Q_I x_{p-d} - P_I x_{p+d} in the accumulator layout
        T wr[S][4], wi[S][4];
#pragma unroll
        for (int I = 0; I < S; ++I) {
            Acc3<T, 1, 1> acc;
            acc.zero();
            if (hasPrev)
                tile_nn3<T, KS>(acc, Q, m, m, 16 * I, xm + c0, k, cw, 0, m);
            if (hasNext)
                tile_nn3<T, KS>(acc, P, m, m, 16 * I, xn + c0, k, cw, 0, m);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * I + MF<T>::row(kr, v);
                const cx<T> gv = (r < m && cc < cw) ? g[r * k + c0 + cc] : czero<T>();
                wr[I][v] = gv.r - acc.re(0, 0, v);
                wi[I][v] = gv.i - acc.im(0, 0, v);
            }
        }
        // bottom tile first: x_{S-1} = D_{S-1}^H w_{S-1}
        v4 x1r = {0, 0, 0, 0}, x1i = {0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const cx<T> a = aDh[S - 1][v];
            x1r = MF<T>::mma(a.r, wr[S - 1][v], x1r);
            x1r = MF<T>::mma(-a.i, wi[S - 1][v], x1r);
            x1i = MF<T>::mma(a.r, wi[S - 1][v], x1i);
            x1i = MF<T>::mma(a.i, wr[S - 1][v], x1i);
        }
        v4 x0r = x1r, x0i = x1i;
        if (S == 2) {
            // w_0 -= L_10^H x_1, x_0 = D_0^H w_0
            v4 tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cx<T> a = aLh[v];
                tr = MF<T>::mma(a.r, x1r[v], tr);
                tr = MF<T>::mma(-a.i, x1i[v], tr);
                ti = MF<T>::mma(a.r, x1i[v], ti);
                ti = MF<T>::mma(a.i, x1r[v], ti);
            }
            x0r = v4{0, 0, 0, 0};
            x0i = v4{0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cx<T> a = aDh[0][v];
                const T br = wr[0][v] - tr[v], bi = wi[0][v] - ti[v];
                x0r = MF<T>::mma(a.r, br, x0r);
                x0r = MF<T>::mma(-a.i, bi, x0r);
                x0i = MF<T>::mma(a.r, bi, x0i);
                x0i = MF<T>::mma(a.i, br, x0i);
            }
        }
        if (cc < cw) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r0 = MF<T>::row(kr, v);
                if (r0 < m)
                    put_x<T>(xp, up, upd, r0 * k + c0 + cc, cx<T>{x0r[v], x0i[v]});
                if (S == 2 && 16 + r0 < m)
                    put_x<T>(xp, up, upd, (16 + r0) * k + c0 + cc, cx<T>{x1r[v], x1i[v]});
            }
        }
    }
}

} // namespace crs
