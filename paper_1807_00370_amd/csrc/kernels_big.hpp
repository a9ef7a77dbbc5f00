// Kernels of a reduction level for block sizes 32 < m <= 256 (the block 2D
// Poisson workload has m = 256).  A block no longer fits in LDS, so every
// step is cut into 16 x 16 MFMA tiles whose operands stream from L2 (the
// streaming products in the three-multiplication complex form, Acc3):
//
//   k_potrf_big   one work-group (four or eight waves) per eliminated
//                 block: blocked left-looking
//                 Cholesky L_p = chol(A_p) by 16-column panels.  The panel
//                 update L[R][<I] L[I][<I]^H runs on MFMA, each 16 x 16
//                 diagonal tile is factored in registers (one row per lane)
//                 and its inverse D_I = L_II^{-1} is kept for the
//                 substitutions; the tiles below become S_R D_I^H.
//   k_trsm_big    one work-group per (eliminated block, group of 16-column
//                 strips of [B_p^H | B_{p-d} | y_p]), one wave per row tile:
//                 blocked forward substitution
//                 X_I = D_I (G_I - L[I][<I] X_{<I}), the Section 4 recipe
//                 L \ G for the three operands of Eq. (Formulas).
//   k_reduce_big  one wave per (kept block, 16 or 32 wide tile) of the reduced
//                 system A' = A_q - P_l^H P_l - Q_r^H Q_r (lower triangle),
//                 B' = -P_r^H Q_r, y' = y_q - P_l^H g_l - Q_r^H g_r; with
//                 16 x 16 tiles it also serves the levels of m <= 32 that
//                 hold few blocks.
//   k_reduce_lds  A' and B' for blocks above 64: one work-group of four
//                 waves per 64 x 64 tile, operand panels staged in LDS.
//   k_back_big    one work-group per (eliminated block, 16-column strip of
//                 x_p), one wave per row tile: blocked back substitution of
//                 L^H x_p = g_p - Q_p x_{p-d} - P_p x_{p+d}.
//   k_grad_big    one wave per (block row, 32 x 32 tile) of the adjoint's
//                 gradient blocks.
//
// Storage for these sizes: L_p as a full m x m row-major slot (lower
// triangle used; the diagonal holds {L_cc, 1 / L_cc} like every other
// factor) and the inverse diagonal tiles D_I (16 x 16 row-major, lower
// triangular) at Seg::oD.  A trailing partial tile is padded with the
// identity, so the padding never reaches a stored value.
#pragma once

#include "kernels_fast.hpp"

namespace crs {

// Work item of this work-group when the 1-D grid (a multiple of 8 groups) is
// dealt round-robin over the 8 XCDs: consecutive items then run on one XCD,
// whose L2 holds the operands they share.
__device__ __forceinline__ int64_t xcd_item()
{
    const int64_t b = blockIdx.x, q = gridDim.x >> 3;
    return (b & 7) * q + (b >> 3);
}

// Operand of a wave-level product: element (o, t) at p[o * so + t * st] for
// o < no (zero beyond), where o is the row of a left operand or the column
// of a right operand and t the contraction index.
template <class T>
struct WOp {
    const cx<T>* p;
    int so, st, no;
};

// (cr, ci)[a][b] += opA(A) opB(B) over kd contraction steps for the RM x RN
// tiles of 16 x 16: rows 16 a + i of the left operand, columns 16 b + j of the
// right one; CA / CB conjugate the operand.  Operands are loaded G k-steps at
// a time, one group ahead of the MFMAs that consume the previous group.
template <class T, int RM, int RN, bool CA, bool CB, int G>
__device__ __forceinline__ void wave_mm(typename MF<T>::v4 (&cr)[RM][RN],
                                        typename MF<T>::v4 (&ci)[RM][RN], const WOp<T> A,
                                        const WOp<T> B, int kd)
{
    const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int ng = (kd + 4 * G - 1) / (4 * G);
    if (ng <= 0)
        return;
    const cx<T>* pa[RM];
    const cx<T>* pb[RN];
    bool oa[RM], ob[RN];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
        const int o = 16 * i + cc;
        oa[i] = o < A.no;
        pa[i] = A.p + ((oa[i] ? o : 0) * A.so + kr * A.st);
    }
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int o = 16 * j + cc;
        ob[j] = o < B.no;
        pb[j] = B.p + ((ob[j] ? o : 0) * B.so + kr * B.st);
    }
    const int sa = 4 * A.st, sb = 4 * B.st;
    cx<T> xa0[RM][G], yb0[RN][G], xa1[RM][G], yb1[RN][G];
    auto load = [&](cx<T>(&xa)[RM][G], cx<T>(&yb)[RN][G], int g) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int ks = g * G + u;
            const bool ok = 4 * ks + kr < kd;
#pragma unroll
            for (int i = 0; i < RM; ++i)
                xa[i][u] = ld_or0(pa[i] + ks * sa, A.p, ok && oa[i]);
#pragma unroll
            for (int j = 0; j < RN; ++j)
                yb[j][u] = ld_or0(pb[j] + ks * sb, B.p, ok && ob[j]);
        }
    };
    auto comp = [&](const cx<T>(&xa)[RM][G], const cx<T>(&yb)[RN][G]) {
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j) {
                    const T ar = xa[i][u].r, ai = CA ? -xa[i][u].i : xa[i][u].i;
                    const T br = yb[j][u].r, bi = CB ? -yb[j][u].i : yb[j][u].i;
                    cr[i][j] = MF<T>::mma(ar, br, cr[i][j]);
                    cr[i][j] = MF<T>::mma(-ai, bi, cr[i][j]);
                    ci[i][j] = MF<T>::mma(ar, bi, ci[i][j]);
                    ci[i][j] = MF<T>::mma(ai, br, ci[i][j]);
                }
    };
    load(xa0, yb0, 0);
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng)
            load(xa1, yb1, g + 1);
        comp(xa0, yb0);
        __builtin_amdgcn_sched_barrier(0);
        if (g + 1 < ng) {
            if (g + 2 < ng)
                load(xa0, yb0, g + 2);
            comp(xa1, yb1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// acc += opA(A) opB(B) in the 3M form (one real MFMA per step for real
// data, RE), operands as in wave_mm.
template <class T, int RM, int RN, bool CA, bool CB, int G, bool RE = false>
__device__ __forceinline__ void wave_mm3(Acc3<T, RM, RN, RE>& acc, const WOp<T> A, const WOp<T> B,
                                         int kd)
{
    const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int ng = (kd + 4 * G - 1) / (4 * G);
    if (ng <= 0)
        return;
    const cx<T>* pa[RM];
    const cx<T>* pb[RN];
    bool oa[RM], ob[RN];
#pragma unroll
    for (int i = 0; i < RM; ++i) {
        const int o = 16 * i + cc;
        oa[i] = o < A.no;
        pa[i] = A.p + ((oa[i] ? o : 0) * A.so + kr * A.st);
    }
#pragma unroll
    for (int j = 0; j < RN; ++j) {
        const int o = 16 * j + cc;
        ob[j] = o < B.no;
        pb[j] = B.p + ((ob[j] ? o : 0) * B.so + kr * B.st);
    }
    const int sa = 4 * A.st, sb = 4 * B.st;
    cx<T> xa0[RM][G], yb0[RN][G], xa1[RM][G], yb1[RN][G];
    auto load = [&](cx<T>(&xa)[RM][G], cx<T>(&yb)[RN][G], int g) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int ks = g * G + u;
            const bool ok = 4 * ks + kr < kd;
#pragma unroll
            for (int i = 0; i < RM; ++i)
                xa[i][u] = ld_or0(pa[i] + ks * sa, A.p, ok && oa[i]);
#pragma unroll
            for (int j = 0; j < RN; ++j)
                yb[j][u] = ld_or0(pb[j] + ks * sb, B.p, ok && ob[j]);
        }
    };
    auto comp = [&](const cx<T>(&xa)[RM][G], const cx<T>(&yb)[RN][G]) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            T ar[RM], ai[RM], as[RM], br[RN], bi[RN], bs[RN];
#pragma unroll
            for (int i = 0; i < RM; ++i) {
                ar[i] = xa[i][u].r;
                ai[i] = CA ? -xa[i][u].i : xa[i][u].i;
                as[i] = ar[i] + ai[i];
            }
#pragma unroll
            for (int j = 0; j < RN; ++j) {
                br[j] = yb[j][u].r;
                bi[j] = CB ? -yb[j][u].i : yb[j][u].i;
                bs[j] = br[j] + bi[j];
            }
#pragma unroll
            for (int i = 0; i < RM; ++i)
#pragma unroll
                for (int j = 0; j < RN; ++j) {
                    acc.t1[i][j] = MF<T>::mma(ar[i], br[j], acc.t1[i][j]);
                    if constexpr (!RE) {
                        acc.t2[i][j] = MF<T>::mma(ai[i], bi[j], acc.t2[i][j]);
                        acc.t3[i][j] = MF<T>::mma(as[i], bs[j], acc.t3[i][j]);
                    }
                }
        }
    };
    load(xa0, yb0, 0);
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng)
            load(xa1, yb1, g + 1);
        comp(xa0, yb0);
        __builtin_amdgcn_sched_barrier(0);
        if (g + 1 < ng) {
            if (g + 2 < ng)
                load(xa0, yb0, g + 2);
            comp(xa1, yb1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// (cr, ci) += H Y for the 16 x 16 tile with rows row0.. of H and columns of
// the right operand Y, where H is the Hermitian matrix read from the lower
// triangle and the real diagonal of the m x m row-major block A:
// H[i][t] = A[i][t] (t < i), Re A[i][i] (t = i), conj(A[t][i]) (t > i);
// contraction over all m columns, loaded as in wave_mm.
template <class T, int G>
__device__ __forceinline__ void wave_mm_herm(typename MF<T>::v4& cr, typename MF<T>::v4& ci,
                                             const cx<T>* __restrict__ A, int m, int row0,
                                             const WOp<T> B)
{
    const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int kd = m, ng = (kd + 4 * G - 1) / (4 * G);
    const int i = row0 + cc;
    const bool oa = i < m, ob = cc < B.no;
    const cx<T>* pb = B.p + ((ob ? cc : 0) * B.so + kr * B.st);
    const int sb = 4 * B.st;
    cx<T> xa0[G], yb0[G], xa1[G], yb1[G];
    auto load = [&](cx<T>(&xa)[G], cx<T>(&yb)[G], int g) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int ks = g * G + u, t = 4 * ks + kr;
            const bool ok = t < kd;
            cx<T> a = ld_or0(A + (t <= i ? i * m + t : t * m + i), A, ok && oa);
            a.i = t < i ? a.i : (t == i ? T(0) : -a.i);
            xa[u] = a;
            yb[u] = ld_or0(pb + ks * sb, B.p, ok && ob);
        }
    };
    auto comp = [&](const cx<T>(&xa)[G], const cx<T>(&yb)[G]) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            cr = MF<T>::mma(xa[u].r, yb[u].r, cr);
            cr = MF<T>::mma(-xa[u].i, yb[u].i, cr);
            ci = MF<T>::mma(xa[u].r, yb[u].i, ci);
            ci = MF<T>::mma(xa[u].i, yb[u].r, ci);
        }
    };
    load(xa0, yb0, 0);
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng)
            load(xa1, yb1, g + 1);
        comp(xa0, yb0);
        __builtin_amdgcn_sched_barrier(0);
        if (g + 1 < ng) {
            if (g + 2 < ng)
                load(xa0, yb0, g + 2);
            comp(xa1, yb1);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <class T, int RM, int RN>
__device__ __forceinline__ void zero_acc(typename MF<T>::v4 (&cr)[RM][RN],
                                         typename MF<T>::v4 (&ci)[RM][RN])
{
#pragma unroll
    for (int i = 0; i < RM; ++i)
#pragma unroll
        for (int j = 0; j < RN; ++j) {
            cr[i][j] = typename MF<T>::v4{0, 0, 0, 0};
            ci[i][j] = typename MF<T>::v4{0, 0, 0, 0};
        }
}

// The diagonal step of panel I of the tiled Cholesky, run by one wave: the
// tile S_II (lower triangle in sT, leading dimension 17) is factored by the
// left-looking lane-per-row Cholesky, lane r & 15 keeping row r in registers
// and the later columns reading the finished rows by broadcast (scalar
// registers for RB, else LDS over sT); then lane r forms column r of
// D_I = L_II^{-1} by forward substitution.  L_II goes to L (diagonal
// {L_cc, 1 / L_cc}), D_I to Dg and to sD (leading dimension 17).  Returns
// true on a pivot that is not > 0.
template <class T, bool RB>
__device__ __forceinline__ bool potrf_diag_tile(cx<T>* sT, cx<T>* sD, cx<T>* __restrict__ Lg,
                                                cx<T>* __restrict__ Dg, int m, int I)
{
    const int lane = threadIdx.x & 63, c0 = 16 * I;
    const int r = lane & 15, gi = c0 + r;
    const bool real = gi < m;
    cx<T> a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        if (real)
            a[u] = u <= r ? sT[r * 17 + u] : czero<T>();
        else
            a[u] = u == r ? cx<T>{T(1), T(0)} : czero<T>();
        if (u == r)
            a[u].i = T(0);
    }
    bool fail = false;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        cx<T> s0 = a[c], s1 = czero<T>();
#pragma unroll
        for (int u = 0; u + 1 < c; u += 2) {
            if constexpr (RB) {
                msub_cb(s0, a[u], lane_bcast(a[u], c));
                msub_cb(s1, a[u + 1], lane_bcast(a[u + 1], c));
            } else {
                msub_cb(s0, a[u], sT[c * 17 + u]);
                msub_cb(s1, a[u + 1], sT[c * 17 + u + 1]);
            }
        }
        if (c & 1)
            msub_cb(s0, a[c - 1], RB ? lane_bcast(a[c - 1], c) : sT[c * 17 + c - 1]);
        const cx<T> sv{s0.r + s1.r, s0.i + s1.i};
        const T dg = RB ? lane_bcast(sv.r, c) : __shfl(sv.r, c);
        const T inv = rsqrt_nr(dg);
        const T sq = dg * inv;
        fail |= (c0 + c < m) && !(dg > T(0));
        if (r == c)
            a[c] = cx<T>{sq, inv}; // inverse pivot kept in the imaginary slot
        else if (r > c)
            a[c] = cx<T>{sv.r * inv, sv.i * inv};
        if constexpr (!RB) {
            if (lane < 16)
                sT[r * 17 + c] = a[c];
            wave_lds_sync();
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    if (lane < 16 && real) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (u <= r)
                Lg[(int64_t)gi * m + c0 + u] = a[u];
    }
    cx<T> z[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        cx<T> v = q == r ? cx<T>{T(1), T(0)} : czero<T>();
#pragma unroll
        for (int u = 0; u < q; ++u)
            msub(v, RB ? lane_bcast(a[u], q) : sT[q * 17 + u], z[u]);
        const T iq = RB ? lane_bcast(a[q].i, q) : sT[q * 17 + q].i;
        z[q] = cx<T>{v.r * iq, v.i * iq};
    }
    if (lane < 16) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            Dg[I * 256 + q * 16 + r] = z[q];
            sD[q * 17 + r] = z[q];
        }
    }
    return fail;
}

// ------------------------------------------------------------- k_potrf_big

// RB: the diagonal tile's Cholesky and inverse read the rows of L through
// the scalar registers (lane c broadcasts row c) and the kernel is held to
// three waves per SIMD; otherwise the rows go through LDS and the compiler
// keeps two waves per SIMD.  The first is faster at m <= 64 (the diagonal
// tiles are a larger share of the work), the second at m = 256.
template <class T, bool RB, class EI = cx<T>, bool RE = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(RB ? 3 : 2, 8))) void k_potrf_big(const Seg* __restrict__ segs, int nseg,
                                                   int64_t total, const EI* __restrict__ inA,
                                                   cx<T>* __restrict__ W,
                                                   unsigned long long* __restrict__ flags)
{
    using v4 = typename MF<T>::v4;
    __shared__ cx<T> sT[16 * 17]; // diagonal tile S_I (row-major, leading dimension 17)
    __shared__ cx<T> sD[16 * 17]; // D_I for the tiles below the diagonal (leading dimension 17)
    __shared__ int sFail;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, kr = lane >> 4, cc = lane & 15;
    const int nw = blockDim.x >> 6;
    const int64_t w = blockIdx.x;
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int64_t t = w - s.w0;
    const int p = s.e0 + (int)t * s.es;
    const int m = s.m, S = (m + 15) >> 4;
    if ((flags[s.sys] >> 40) < (unsigned long long)s.level)
        return; // broke down at an earlier level
    const int64_t mm = (int64_t)m * m;
    const EI* Ap = inA + s.oA + (int64_t)p * mm;
    cx<T>* Lg = W + s.oL + t * mm;
    cx<T>* Dg = W + s.oD + t * (int64_t)S * 256;
    if (tid == 0)
        sFail = 0;
    for (int I = 0; I < S; ++I) {
        const int c0 = 16 * I;
        // panel column I: S_R = A[R][I] - L[R][<I] L[I][<I]^H for R >= I (the
        // Hermitian reading of A: lower triangle of the diagonal tile only)
        for (int R = I + wv; R < S; R += nw) {
            Acc3<T, 1, 1, RE> acc;
            acc.zero();
            wave_mm3<T, 1, 1, false, true, 4, RE>(acc, WOp<T>{Lg + (int64_t)16 * R * m, m, 1, m - 16 * R},
                                              WOp<T>{Lg + (int64_t)c0 * m, m, 1, m - c0}, c0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * R + MF<T>::row(kr, v), j = c0 + cc;
                if (i < m && j < m && (R > I || j <= i)) {
                    const cx<T> a = cvt<T>(Ap[(int64_t)i * m + j]);
                    const cx<T> o{a.r - acc.re(0, 0, v), a.i - acc.im(0, 0, v)};
                    if (R == I) // the diagonal tile goes to wave 0 through LDS
                        sT[(i - c0) * 17 + (j - c0)] = o;
                    else
                        Lg[(int64_t)i * m + j] = o;
                }
            }
        }
        __syncthreads();
        // diagonal tile (wave 0): lane r & 15 keeps row r in registers;
        // left-looking Cholesky whose later columns read the finished rows
        // of L by broadcast (scalar registers, or LDS over S_I, already in
        // registers); then lane r forms column r of D = L_II^{-1} by forward
        // substitution
        if (wv == 0) {
            const bool fail = potrf_diag_tile<T, RB>(sT, sD, Lg, Dg, m, I);
            if (lane == 0 && fail)
                sFail = 1;
        }
        __syncthreads();
        // tiles below the diagonal: L[R][I] = S_R D_I^H, in place.  Step q of
        // the contraction: lane (kr, cc) supplies S_R[cc][4 q + kr] and
        // conj(D_I[cc][4 q + kr]), the latter read from the LDS array itself
        // (a generic pointer would give flat loads, which wait behind the
        // wave's global stores of its previous tile)
        for (int R = I + 1 + wv; R < S; R += nw) {
            const int kd = min(16, m - c0);
            cx<T> sa[4], db[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * R + cc, tc = 4 * q + kr;
                sa[q] = (i < m && tc < kd) ? Lg[(int64_t)i * m + c0 + tc] : czero<T>();
                db[q] = tc < kd ? sD[cc * 17 + tc] : czero<T>();
            }
            Acc3<T, 1, 1, RE> acc;
            acc.zero();
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc.step(0, 0, sa[q].r, sa[q].i, db[q].r, -db[q].i);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * R + MF<T>::row(kr, v), j = c0 + cc;
                if (i < m && j < m)
                    Lg[(int64_t)i * m + j] = cx<T>{acc.re(0, 0, v), acc.im(0, 0, v)};
            }
        }
        __syncthreads();
    }
    if (tid == 0 && sFail)
        atomicMin(&flags[s.sys], fail_key(s.level, s.ob0 + s.obs * p));
}

// -------------------------------------------------------------- k_potrf_rl

// Right-looking form of the tiled Cholesky for launches of few blocks
// (m > 64, one work-group of eight waves per block), where one block's chain
// of panels sets the time.  Per 16-column panel I: the waves form the tiles
// below the diagonal, L_RI = S_RI D_I^H, into L and into LDS; then wave 0
// runs ahead on the next panel -- S_JJ -= L_JI L_JI^H for J = I + 1, straight
// into LDS, and the diagonal step of panel J (potrf_diag_tile: L_JJ, D_J) --
// while the other seven waves update the remaining trailing tiles
// S_RC -= L_RI L_CI^H (I < C <= R) in place in the L slot, eight tiles per
// batch of loads, both product operands from LDS.  The diagonal steps, a
// chain of one wave, thus overlap the trailing updates instead of idling
// the work-group.  Panel 0 reads the tiles of A (Hermitian reading: lower
// triangle, the diagonal's imaginary parts dropped when a diagonal tile is
// factored) and writes every lower tile of the slot once; later panels read
// and update the slot.  The trailing sums round once per panel: the same
// factorization as k_potrf_big up to rounding order.
template <class T, class EI = cx<T>, bool RE = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_potrf_rl(const Seg* __restrict__ segs, int nseg,
                                                  int64_t total, const EI* __restrict__ inA,
                                                  cx<T>* __restrict__ W,
                                                  unsigned long long* __restrict__ flags)
{
    constexpr int kMaxS = 16; // m <= 256
    constexpr int TB = 8;     // trailing tiles per batch of loads
    __shared__ cx<T> sT[16 * 17]; // diagonal tile S_I (row-major, leading dimension 17)
    __shared__ cx<T> sD[16 * 17]; // D_I (leading dimension 17)
    __shared__ cx<T> sP[(kMaxS - 1) * 256]; // L_RI of R > I: tile R - I - 1, 16 x 16 row-major
    __shared__ int sFail;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, kr = lane >> 4, cc = lane & 15;
    const int nw = blockDim.x >> 6;
    const int64_t w = blockIdx.x;
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int64_t t = w - s.w0;
    const int p = s.e0 + (int)t * s.es;
    const int m = s.m, S = (m + 15) >> 4;
    if ((flags[s.sys] >> 40) < (unsigned long long)s.level)
        return;
    const int64_t mm = (int64_t)m * m;
    const EI* Ap = inA + s.oA + (int64_t)p * mm;
    cx<T>* Lg = W + s.oL + t * mm;
    cx<T>* Dg = W + s.oD + t * (int64_t)S * 256;
    // element (i, j) of the lower triangle as panel I finds it, zero unless
    // ok; the load is issued in every lane (element (0, 0) stands in), so a
    // wave's count of memory operations in flight stays exact
    auto cur_el = [&](int I, int i, int j, bool ok) -> cx<T> {
        const int64_t e = ok ? (int64_t)i * m + j : 0;
        const cx<T> v = I == 0 ? cvt<T>(Ap[e]) : Lg[e];
        return ok ? v : czero<T>();
    };
    if (tid == 0)
        sFail = 0;
    bool fail = false;
    // panel 0's diagonal step (later ones run ahead, during the previous
    // panel's trailing updates)
    if (wv == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = kr * 4 + v;
            const cx<T> e = cur_el(0, i, cc, cc <= i && i < m);
            if (cc <= i && i < m)
                sT[i * 17 + cc] = e;
        }
        wave_lds_sync();
        fail |= potrf_diag_tile<T, false>(sT, sD, Lg, Dg, m, 0);
    }
    __syncthreads();
    for (int I = 0; I < S; ++I) {
        const int c0 = 16 * I, kd = min(16, m - c0);
        // tiles below the diagonal: L_RI = S_RI D_I^H, to L and to LDS.
        // Contraction step q: lane (kr, cc) supplies S_RI[cc][4 q + kr] and
        // conj(D_I[cc][4 q + kr])
        for (int R = I + 1 + wv; R < S; R += nw) {
            cx<T> sa[4], db[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * R + cc, tc = 4 * q + kr;
                sa[q] = cur_el(I, i, c0 + tc, i < m && tc < kd);
                db[q] = tc < kd ? sD[cc * 17 + tc] : czero<T>();
            }
            Acc3<T, 1, 1, RE> acc;
            acc.zero();
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc.step(0, 0, sa[q].r, sa[q].i, db[q].r, -db[q].i);
            cx<T>* tp = sP + (R - I - 1) * 256;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ii = MF<T>::row(kr, v), i = 16 * R + ii, j = c0 + cc;
                const cx<T> l{acc.re(0, 0, v), acc.im(0, 0, v)};
                const bool in = i < m && j < m;
                if (in)
                    Lg[(int64_t)i * m + j] = l;
                tp[ii * 16 + cc] = in ? l : czero<T>();
            }
        }
        __syncthreads();
        if (I + 1 < S) {
            const int nt = S - I - 1, ntile = nt * (nt + 1) / 2;
            if (wv == 0) {
                // look-ahead: S_JJ -= L_JI L_JI^H for J = I + 1 (sP tile 0),
                // straight into sT, then the diagonal step of panel J
                const int J = I + 1, cJ = 16 * J;
                Acc3<T, 1, 1, RE> acc;
                acc.zero();
                const int ta = cc * 16 + kr;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const cx<T> a = sP[ta + 4 * q];
                    acc.step(0, 0, a.r, a.i, a.r, -a.i);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = MF<T>::row(kr, v), gi = cJ + i, gj = cJ + cc;
                    const bool ok = cc <= i && gi < m;
                    const cx<T> o = cur_el(I, gi, gj, ok);
                    if (ok)
                        sT[i * 17 + cc] = cx<T>{o.r - acc.re(0, 0, v), o.i - acc.im(0, 0, v)};
                }
                wave_lds_sync();
                fail |= potrf_diag_tile<T, false>(sT, sD, Lg, Dg, m, J);
            } else {
                // the other trailing tiles S_RC -= L_RI L_CI^H, I < C <= R, row
                // by row (tile 0 is the look-ahead's), TB at a time: their
                // loads issued together before the stores, in every lane
                auto tile_rc = [&](int e, int& R, int& C) {
                    int r = (int)((sqrtf(8.0f * e + 1.0f) - 1.0f) * 0.5f);
                    while (r * (r + 1) / 2 > e)
                        --r;
                    while ((r + 1) * (r + 2) / 2 <= e)
                        ++r;
                    R = I + 1 + r;
                    C = I + 1 + (e - r * (r + 1) / 2);
                };
                const int nwt = nw - 1;
                for (int eb = wv; eb < ntile; eb += nwt * TB) {
                    cx<T> cur[TB][4];
#pragma unroll
                    for (int b = 0; b < TB; ++b) {
                        const int e = eb + nwt * b;
                        int R = I + 1, C = I + 1;
                        if (e < ntile)
                            tile_rc(e, R, C);
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = 16 * R + MF<T>::row(kr, v), j = 16 * C + cc;
                            cur[b][v] = cur_el(I, i, j, e < ntile && i < m && j <= i);
                        }
                    }
#pragma unroll
                    for (int b = 0; b < TB; ++b) {
                        const int e = eb + nwt * b;
                        if (e >= ntile)
                            break;
                        int R, C;
                        tile_rc(e, R, C);
                        Acc3<T, 1, 1, RE> acc;
                        acc.zero();
                        const int ta = (R - I - 1) * 256 + cc * 16 + kr, tb = (C - I - 1) * 256 + cc * 16 + kr;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const cx<T> a = sP[ta + 4 * q], bb = sP[tb + 4 * q];
                            acc.step(0, 0, a.r, a.i, bb.r, -bb.i);
                        }
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int i = 16 * R + MF<T>::row(kr, v), j = 16 * C + cc;
                            if (i < m && j <= i)
                                Lg[(int64_t)i * m + j] =
                                    cx<T>{cur[b][v].r - acc.re(0, 0, v), cur[b][v].i - acc.im(0, 0, v)};
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (wv == 0 && lane == 0 && fail)
        sFail = 1;
    __syncthreads();
    if (tid == 0 && sFail)
        atomicMin(&flags[s.sys], fail_key(s.level, s.ob0 + s.obs * p));
}

// -------------------------------------------------------------- k_trsm_big

// Strips per work-group of the tiled forward substitution: every L tile a
// wave loads serves this many 16-column strips.
template <class T>
constexpr int trsm_strips()
{
    return sizeof(T) == 8 ? 2 : 4;
}

// One work-group per (eliminated block, group of NC = trsm_strips<T>()
// 16-column strips of [B_p^H | B_{p-d} | y_p]), one wave per 16-row tile I
// (blockDim = 64 x the largest tile count of the launch).  Strip u of a block
// is a column strip of B_p^H for u < S, of B_{p-d} for u < 2 S (with_mat), of
// y_p after them (with_rhs).  Top-down over the tiles J: wave J forms
// X_J = D_J (G_J - acc_J), the accumulator being the right operand (see the
// note in k_elim_mf), stores it and publishes it in LDS; every wave I > J
// then accumulates acc_I += L_IJ X_J (its operand loaded one step ahead).
template <class T, class EI = cx<T>, bool RE = false>
__global__ __launch_bounds__(1024) void k_trsm_big(const Seg* __restrict__ segs, int nseg,
                                                   int64_t total, int ngrp, int with_mat,
                                                   int with_rhs, const EI* __restrict__ inB,
                                                   const EI* __restrict__ iny,
                                                   cx<T>* __restrict__ W,
                                                   const unsigned long long* __restrict__ flags)
{
    using v4 = typename MF<T>::v4;
    constexpr int NC = trsm_strips<T>();
    __shared__ cx<T> sx[NC][256]; // X_J of each strip, row-major 16 x 16
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int64_t li = xcd_item();
    const int64_t w = li / ngrp;
    const int grp = (int)(li - w * ngrp);
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int64_t t = w - s.w0;
    const int p = s.e0 + (int)t * s.es;
    const int m = s.m, k = s.k, d = s.d, S = (m + 15) >> 4;
    if ((flags[s.sys] >> 40) < (unsigned long long)s.level)
        return;
    const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
    const bool hasPrev = p - d >= 0, hasNext = p + d < s.n;
    const int nmat = with_mat ? 2 * S : 0;
    const int nstrip = nmat + (with_rhs ? (k + 15) / 16 : 0);
    // per strip slot b: element (r, c) of the right-hand side is
    // G[b][r * gr[b] + c * gc[b]] (conjugated for B_p^H), the solution goes
    // to out[b][r * ld[b] + c], columns c0[b] .. c0[b] + nc[b] - 1
    const EI* G[NC];
    cx<T>* out[NC];
    int gr[NC], gc[NC], ld[NC], c0[NC], nc[NC];
    bool cj[NC], on[NC];
    bool any = false;
#pragma unroll
    for (int b = 0; b < NC; ++b) {
        const int u = grp * NC + b;
        int src = 2, cu = u - nmat;
        if (u < nmat) {
            src = u < S ? 0 : 1;
            cu = u < S ? u : u - S;
        }
        on[b] = u < nstrip && (src == 0 ? hasNext : (src == 1 ? hasPrev : true));
        c0[b] = 16 * cu;
        const int ncol = src == 2 ? k : m;
        nc[b] = on[b] ? min(16, ncol - c0[b]) : 0;
        on[b] = on[b] && nc[b] > 0;
        cj[b] = src == 0;
        if (src == 0) {
            G[b] = inB + s.oB + (int64_t)p * mm;
            gr[b] = 1;
            gc[b] = m;
            out[b] = W + s.oP + t * mm;
            ld[b] = m;
        } else if (src == 1) {
            G[b] = inB + s.oB + (int64_t)(p - d) * mm;
            gr[b] = m;
            gc[b] = 1;
            out[b] = W + s.oQ + t * mm;
            ld[b] = m;
        } else {
            G[b] = iny + s.oy + (int64_t)p * mk;
            gr[b] = k;
            gc[b] = 1;
            out[b] = W + s.og + t * mk;
            ld[b] = k;
        }
        any |= on[b];
    }
    if (!any)
        return;
    const cx<T>* Lg = W + s.oL + t * mm;
    const cx<T>* Dg = W + s.oD + t * (int64_t)S * 256;
    const bool own = wv < S;
    const int r0 = 16 * wv;
    // D_I operand of this wave's tile and its right-hand sides (accumulator layout)
    cx<T> aD[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        aD[v] = own ? Dg[wv * 256 + cc * 16 + MF<T>::row(kr, v)] : czero<T>();
    v4 ar[NC], ai[NC];
#pragma unroll
    for (int b = 0; b < NC; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + MF<T>::row(kr, v);
            cx<T> x = czero<T>();
            if (own && on[b] && r < m && cc < nc[b])
                x = cvt<T>(G[b][r * gr[b] + (c0[b] + cc) * gc[b]]);
            ar[b][v] = x.r;
            ai[b][v] = cj[b] ? -x.i : x.i;
        }
    // operand of the update at step J: A(i, t) = L[r0 + i][16 J + t]
    auto load_l = [&](int J, cx<T>(&a)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = (own && wv > J && r0 + cc < m) ? Lg[(int64_t)(r0 + cc) * m + 16 * J + 4 * q + kr]
                                                  : czero<T>();
        }
    };
    cx<T> an[4];
    load_l(0, an);
    for (int J = 0; J < S; ++J) {
        cx<T> a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            a[q] = an[q];
        if (J + 1 < S)
            load_l(J + 1, an);
        if (wv == J) {
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                if (!on[b])
                    continue;
                // X_J = D_J acc (acc holds G_J - sum of the updates)
                v4 xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const cx<T> q = aD[v];
                    xr = MF<T>::mma(q.r, ar[b][v], xr);
                    if constexpr (!RE) {
                        xr = MF<T>::mma(-q.i, ai[b][v], xr);
                        xi = MF<T>::mma(q.r, ai[b][v], xi);
                        xi = MF<T>::mma(q.i, ar[b][v], xi);
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int rr = MF<T>::row(kr, v), r = r0 + rr;
                    sx[b][rr * 16 + cc] = cx<T>{xr[v], xi[v]};
                    if (r < m && cc < nc[b])
                        out[b][(int64_t)r * ld[b] + c0[b] + cc] = cx<T>{xr[v], xi[v]};
                }
            }
        }
        __syncthreads();
        if (own && wv > J) {
#pragma unroll
            for (int b = 0; b < NC; ++b) {
                if (!on[b])
                    continue;
                // acc_I -= L_IJ X_J: contraction step q pairs t = 4 q + kr
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const cx<T> x = sx[b][(4 * q + kr) * 16 + cc];
                    ar[b] = MF<T>::mma(-a[q].r, x.r, ar[b]);
                    if constexpr (!RE) {
                        ar[b] = MF<T>::mma(a[q].i, x.i, ar[b]);
                        ai[b] = MF<T>::mma(-a[q].r, x.i, ai[b]);
                        ai[b] = MF<T>::mma(-a[q].i, x.r, ai[b]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// One wave per (eliminated block, NW adjacent 16-column strips): the same
// substitution with each wave sweeping all row tiles of its strips (no
// barriers).  Work items of a block: with_mat gives ceil(S / NW) items of
// columns of B_p^H, then as many of B_{p-d}, with_rhs ceil(ceil(k / 16) / NW)
// items of y_p after them.  With NW = 2 every L tile a wave loads serves two
// strips, which halves the L traffic through L2 and the item count (blocks of
// 33..64; at m = 256 it measured no faster in complex and slower in real
// form).  Used for FP64 levels with many blocks, where the work-group form's
// idle waves would cost throughput, and with eight contraction steps per load
// group for FP64 levels of few blocks above 64.
template <class T, class EI = cx<T>, bool RE = false, int NW = 1, int GD = 0>
__global__ __launch_bounds__(64) void k_trsm_strip(const Seg* __restrict__ segs, int nseg,
                                                 int64_t total, int nstrip, int with_mat,
                                                 int with_rhs, const EI* __restrict__ inB,
                                                 const EI* __restrict__ iny,
                                                 cx<T>* __restrict__ W,
                                                 const unsigned long long* __restrict__ flags)
{
    using v4 = typename MF<T>::v4;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
    const int64_t li = xcd_item();
    const int64_t w = li / nstrip;
    int u = (int)(li - w * nstrip);
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int64_t t = w - s.w0;
    const int p = s.e0 + (int)t * s.es;
    const int m = s.m, k = s.k, d = s.d, S = (m + 15) >> 4;
    if ((flags[s.sys] >> 40) < (unsigned long long)s.level)
        return;
    const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
    const int SI = (S + NW - 1) / NW; // items of B_p^H (and of B_{p-d})
    int src = 2;
    if (with_mat) {
        if (u < 2 * SI)
            src = u < SI ? 0 : 1;
        else
            u -= 2 * SI;
    }
    int c0;
    if (src == 2) {
        c0 = 16 * NW * u;
        if (!with_rhs || c0 >= k)
            return;
    } else {
        c0 = 16 * NW * (src == 0 ? u : u - SI);
        if (src == 0 ? p + d >= s.n : p - d < 0)
            return;
    }
    const int nc = min(16 * NW, (src == 2 ? k : m) - c0);
    // element (r, c) of the right-hand side is G[r * gr + c * gc]
    const EI* G;
    int gr, gc;
    cx<T>* out;
    if (src == 0) {
        G = inB + s.oB + (int64_t)p * mm; // B_p^H: conjugated below
        gr = 1;
        gc = m;
        out = W + s.oP + t * mm;
    } else if (src == 1) {
        G = inB + s.oB + (int64_t)(p - d) * mm;
        gr = m;
        gc = 1;
        out = W + s.oQ + t * mm;
    } else {
        G = iny + s.oy + (int64_t)p * mk;
        gr = k;
        gc = 1;
        out = W + s.og + t * mk;
    }
    const int ldo = src == 2 ? k : m;
    const cx<T>* Lg = W + s.oL + t * mm;
    const cx<T>* Dg = W + s.oD + t * (int64_t)S * 256;
    // two complex strips keep two contraction steps per load group in flight
    // instead of four (the same operand registers); the real form has the
    // registers for four.  GD > 0 sets the depth (launches of few blocks,
    // where each wave's chain of loads, not the occupancy, sets the time).
    constexpr int GK = GD > 0 ? GD : ((NW == 1 || RE) ? 4 : 2);
    for (int I = 0; I < S; ++I) {
        const int r0 = 16 * I;
        Acc3<T, 1, NW, RE> acc;
        acc.zero();
        wave_mm3<T, 1, NW, false, false, GK, RE>(acc, WOp<T>{Lg + (int64_t)r0 * m, m, 1, m - r0},
                                                WOp<T>{out + c0, 1, ldo, nc}, r0);
        // w = G_I - acc stays in the accumulator layout: register v of lane
        // (kr, cc) holds row MF::row(kr, v) of column cc, which is the right
        // operand of contraction step v once the left operand D_I supplies
        // column MF::row(kr, v) of its row cc
        Acc3<T, 1, NW, RE> x;
        x.zero();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = MF<T>::row(kr, v), r = r0 + rr;
            const cx<T> a = Dg[I * 256 + cc * 16 + rr];
#pragma unroll
            for (int b = 0; b < NW; ++b) {
                const int c = 16 * b + cc;
                cx<T> g = (r < m && c < nc) ? cvt<T>(G[r * gr + (c0 + c) * gc]) : czero<T>();
                if (src == 0)
                    g.i = -g.i;
                const T br = g.r - acc.re(0, b, v), bi = g.i - acc.im(0, b, v);
                x.step(0, b, a.r, a.i, br, bi);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = r0 + MF<T>::row(kr, v);
#pragma unroll
            for (int b = 0; b < NW; ++b) {
                const int c = 16 * b + cc;
                if (r < m && c < nc)
                    out[(int64_t)r * ldo + c0 + c] = cx<T>{x.re(0, b, v), x.im(0, b, v)};
            }
        }
        __syncthreads(); // the rows just stored are the next tiles' operands
    }
}

// ------------------------------------------------------------ k_reduce_big

// One wave per output tile of TT = 16 TW rows and columns of a kept block
// (NT = ceil(m / TT)): with_mat gives the NT (NT + 1) / 2 lower tiles of A'
// and the NT^2 tiles of B', with_rhs the NT ceil(k / TT) tiles of y' after
// them.  TW = 2 serves the right-hand sides of blocks above 64 (k > 16);
// TW = 1 the blocks of 32 < m <= 64, the right-hand sides with k <= 16 of
// larger blocks, and the levels of m <= 32 with too few blocks to fill the
// GPU one wave per block.
template <class T, int TW, class EI = cx<T>, bool RE = false>
__global__ __launch_bounds__(64) void k_reduce_big(const Seg* __restrict__ segs, int nseg,
                                                   int64_t total, int ntile, int with_mat,
                                                   int with_rhs, const EI* __restrict__ inA,
                                                   const EI* __restrict__ iny,
                                                   cx<T>* __restrict__ W,
                                                   const unsigned long long* __restrict__ flags)
{
    using v4 = typename MF<T>::v4;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
    const int64_t li = xcd_item();
    const int64_t w = li / ntile;
    int u = (int)(li - w * ntile);
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
        return; // the level's elimination broke down: stop this system
    constexpr int TT = 16 * TW;
    const int NT = (m + TT - 1) / TT, nV = NT * (NT + 1) / 2, nF = NT * NT;
    int kind, ti, tj;
    if (with_mat && u < nV + nF) {
        if (u < nV) {
            kind = 0;
            ti = tri_row(u);
            tj = u - ti * (ti + 1) / 2;
        } else {
            kind = 1;
            u -= nV;
            ti = u / NT;
            tj = u % NT;
            if (!hasR || r + d >= n)
                return;
        }
    } else {
        if (with_mat)
            u -= nV + nF;
        const int Tk = (k + TT - 1) / TT;
        if (!with_rhs || u >= NT * Tk)
            return;
        kind = 2;
        ti = u / Tk;
        tj = u % Tk;
    }
    const cx<T>* Pl = W + s.oP + tl * mm;
    const cx<T>* Qr = W + s.oQ + tr * mm;
    const cx<T>* Pr = W + s.oP + tr * mm;
    const int i0 = TT * ti, j0 = TT * tj;
    // 16 x 16 tiles: the elements of A_q (kind 0) or y_q (kind 2) this lane
    // subtracts from, loaded first and in every lane (element 0 stands in):
    // the loads overlap the products and none waits behind a store of the
    // tile (32 x 32 tiles, short of registers, load each before its store)
    cx<T> xo[TW][TW][4];
    auto load_xo = [&] {
        if (kind == 1)
            return;
        const EI* src = kind == 0 ? inA + s.oA + q * mm : iny + s.oy + q * mk;
        const int ld = kind == 0 ? m : k;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
            for (int b = 0; b < TW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * a + MF<T>::row(kr, v), j = j0 + 16 * b + cc;
                    const bool ok = i < m && (kind == 0 ? j <= i : j < k);
                    xo[a][b][v] = cvt<T>(src[ok ? i * ld + j : 0]);
                }
    };
    if constexpr (TW == 1)
        load_xo();
    Acc3<T, TW, TW, RE> acc;
    acc.zero();
    if (kind == 0) {
        if (hasL)
            wave_mm3<T, TW, TW, true, false, 2 / TW, RE>(acc, WOp<T>{Pl + i0, 1, m, m - i0},
                                             WOp<T>{Pl + j0, 1, m, m - j0}, m);
        if (hasR)
            wave_mm3<T, TW, TW, true, false, 2 / TW, RE>(acc, WOp<T>{Qr + i0, 1, m, m - i0},
                                             WOp<T>{Qr + j0, 1, m, m - j0}, m);
        cx<T>* Vo = W + s.oAo + oi * mm;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
            for (int b = 0; b < TW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * a + MF<T>::row(kr, v), j = j0 + 16 * b + cc;
                    if (i < m && j <= i) {
                        const cx<T> x = TW == 1 ? xo[a][b][v] : cvt<T>(inA[s.oA + q * mm + i * m + j]);
                        cx<T> o{x.r - acc.re(a, b, v), x.i - acc.im(a, b, v)};
                        if (i == j)
                            o.i = T(0);
                        Vo[i * m + j] = o;
                    }
                }
    } else if (kind == 1) {
        wave_mm3<T, TW, TW, true, false, 2 / TW, RE>(acc, WOp<T>{Pr + i0, 1, m, m - i0},
                                         WOp<T>{Qr + j0, 1, m, m - j0}, m);
        cx<T>* Fo = W + s.oBo + oi * mm;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
            for (int b = 0; b < TW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * a + MF<T>::row(kr, v), j = j0 + 16 * b + cc;
                    if (i < m && j < m)
                        Fo[i * m + j] = cx<T>{-acc.re(a, b, v), -acc.im(a, b, v)};
                }
    } else {
        const cx<T>* gl = W + s.og + tl * mk;
        const cx<T>* gr = W + s.og + tr * mk;
        if (hasL)
            wave_mm3<T, TW, TW, true, false, 2 / TW, RE>(acc, WOp<T>{Pl + i0, 1, m, m - i0},
                                             WOp<T>{gl + j0, 1, k, k - j0}, m);
        if (hasR)
            wave_mm3<T, TW, TW, true, false, 2 / TW, RE>(acc, WOp<T>{Qr + i0, 1, m, m - i0},
                                             WOp<T>{gr + j0, 1, k, k - j0}, m);
        cx<T>* vo = W + s.oyo + oi * mk;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
            for (int b = 0; b < TW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * a + MF<T>::row(kr, v), c = j0 + 16 * b + cc;
                    if (i < m && c < k) {
                        const cx<T> x = TW == 1 ? xo[a][b][v] : cvt<T>(iny[s.oy + q * mk + i * k + c]);
                        vo[i * k + c] = cx<T>{x.r - acc.re(a, b, v), x.i - acc.im(a, b, v)};
                    }
                }
    }
}

// ------------------------------------------------------------ k_reduce_lds

// The matrix part of the reduced system (A' lower tiles, B') for blocks above
// 32 with the operand panels staged in LDS: one work-group of four waves per
// (kept block, 64 x 64 tile); wave (a, b) owns the 32 x 32 quarter at rows
// 32 a, columns 32 b of the tile.  For each 16-row panel of the contraction
// the work-group loads 16 x 64 of the left and of the right operand once
// (every element then feeds 32 output rows or columns instead of 16 in
// k_reduce_big) and the waves run their 3M products from LDS; the next panel
// is fetched into registers while the current one is consumed (two LDS
// buffers, one barrier per panel).  Items per kept block: the
// NT (NT + 1) / 2 lower tiles of A', then the NT^2 tiles of B' (NT =
// ceil(m / 64)).  The right-hand-side tiles y' run in k_reduce_big.
template <class T, class EI = cx<T>, bool RE = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_reduce_lds(const Seg* __restrict__ segs, int nseg,
                                                    int64_t total, int ntile,
                                                    const EI* __restrict__ inA,
                                                    cx<T>* __restrict__ W,
                                                    const unsigned long long* __restrict__ flags)
{
    constexpr int KP = 16, LD = 65;
    __shared__ cx<T> sA[2][KP * LD], sB[2][KP * LD];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, kr = lane >> 4, cc = lane & 15;
    const int wa = wv >> 1, wb = wv & 1;
    const int64_t li = xcd_item();
    const int64_t w = li / ntile;
    int u = (int)(li - w * ntile);
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int64_t t = w - s.w0;
    const int q = s.k0 + (int)t * s.ks;
    const int m = s.m, d = s.d, n = s.n;
    const int l = q - d, r = q + d;
    const bool hasL = l >= 0, hasR = r < n;
    const int64_t tl = hasL ? (l - s.e0) / s.es : 0, tr = hasR ? (r - s.e0) / s.es : 0;
    const int64_t oi = s.out_by_pos ? q : t;
    const int64_t mm = (int64_t)m * m;
    if ((flags[s.sys] >> 40) <= (unsigned long long)s.level)
        return; // the level's elimination broke down: stop this system
    const int NT = (m + 63) >> 6, nV = NT * (NT + 1) / 2, nF = NT * NT;
    int kind, ti, tj;
    if (u < nV) {
        kind = 0;
        ti = tri_row(u);
        tj = u - ti * (ti + 1) / 2;
    } else if (u < nV + nF) {
        kind = 1;
        u -= nV;
        ti = u / NT;
        tj = u % NT;
        if (!hasR || r + d >= n)
            return;
    } else {
        return;
    }
    const cx<T>* Pl = W + s.oP + tl * mm;
    const cx<T>* Qr = W + s.oQ + tr * mm;
    const cx<T>* Pr = W + s.oP + tr * mm;
    const int i0 = 64 * ti, j0 = 64 * tj;
    // products: A' tiles sum P_l^H P_l (hasL) and Q_r^H Q_r (hasR); B' tiles
    // are P_r^H Q_r
    const int npr = kind == 0 ? (hasL ? 1 : 0) + (hasR ? 1 : 0) : 1;
    const int nkp = (m + KP - 1) / KP, npan = npr * nkp;
    // quarters above the diagonal of a diagonal tile hold no output
    const bool live = !(kind == 0 && ti == tj && wb > wa);
    // thread tid moves elements e = tid + 256 e4 of a 16 x 64 panel: row
    // e / 64, column e % 64
    cx<T> ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
#define CRS_PANEL_LOAD(pn)                                                                         \
    do {                                                                                           \
        const int pr_ = (pn) / nkp, t0_ = ((pn) - pr_ * nkp) * KP;                                  \
        const cx<T>* X_ = kind == 1 ? Pr : ((hasL && pr_ == 0) ? Pl : Qr);                          \
        const cx<T>* Y_ = kind == 1 ? Qr : X_;                                                      \
        const int row_ = tid >> 6, col_ = tid & 63;                                                 \
        const bool oa_ = i0 + col_ < m, ob_ = j0 + col_ < m;                                        \
        const cx<T>* xa_ = X_ + (int64_t)(t0_ + row_) * m + i0 + col_;                              \
        const cx<T>* yb_ = Y_ + (int64_t)(t0_ + row_) * m + j0 + col_;                              \
        const int64_t st_ = 4 * (int64_t)m;                                                         \
        ra0 = (t0_ + row_ < m && oa_) ? xa_[0] : czero<T>();                                        \
        ra1 = (t0_ + row_ + 4 < m && oa_) ? xa_[st_] : czero<T>();                                  \
        ra2 = (t0_ + row_ + 8 < m && oa_) ? xa_[2 * st_] : czero<T>();                              \
        ra3 = (t0_ + row_ + 12 < m && oa_) ? xa_[3 * st_] : czero<T>();                             \
        rb0 = (t0_ + row_ < m && ob_) ? yb_[0] : czero<T>();                                        \
        rb1 = (t0_ + row_ + 4 < m && ob_) ? yb_[st_] : czero<T>();                                  \
        rb2 = (t0_ + row_ + 8 < m && ob_) ? yb_[2 * st_] : czero<T>();                              \
        rb3 = (t0_ + row_ + 12 < m && ob_) ? yb_[3 * st_] : czero<T>();                             \
    } while (0)
#define CRS_PANEL_STORE(b)                                                                         \
    do {                                                                                           \
        const int o_ = (tid >> 6) * LD + (tid & 63);                                                \
        sA[b][o_] = ra0;                                                                            \
        sA[b][o_ + 4 * LD] = ra1;                                                                   \
        sA[b][o_ + 8 * LD] = ra2;                                                                   \
        sA[b][o_ + 12 * LD] = ra3;                                                                  \
        sB[b][o_] = rb0;                                                                            \
        sB[b][o_ + 4 * LD] = rb1;                                                                   \
        sB[b][o_ + 8 * LD] = rb2;                                                                   \
        sB[b][o_ + 12 * LD] = rb3;                                                                  \
    } while (0)
    Acc3<T, 2, 2, RE> acc;
    acc.zero();
    if (npan > 0) {
        CRS_PANEL_LOAD(0);
        CRS_PANEL_STORE(0);
    }
    __syncthreads();
    for (int pn = 0; pn < npan; ++pn) {
        const int b = pn & 1;
        if (pn + 1 < npan)
            CRS_PANEL_LOAD(pn + 1);
        if (live) {
#pragma unroll
            for (int ks = 0; ks < KP / 4; ++ks) {
                const int row = 4 * ks + kr;
                T ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const cx<T> x = sA[b][row * LD + 32 * wa + 16 * i + cc];
                    ar[i] = x.r;
                    ai[i] = -x.i; // conj: the left operand is X^H
                    as[i] = ar[i] + ai[i];
                    const cx<T> y = sB[b][row * LD + 32 * wb + 16 * i + cc];
                    br[i] = y.r;
                    bi[i] = y.i;
                    bs[i] = br[i] + bi[i];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        acc.t1[i][j] = MF<T>::mma(ar[i], br[j], acc.t1[i][j]);
                        if constexpr (!RE) {
                            acc.t2[i][j] = MF<T>::mma(ai[i], bi[j], acc.t2[i][j]);
                            acc.t3[i][j] = MF<T>::mma(as[i], bs[j], acc.t3[i][j]);
                        }
                    }
            }
        }
        if (pn + 1 < npan)
            CRS_PANEL_STORE(b ^ 1);
        __syncthreads();
    }
#undef CRS_PANEL_LOAD
#undef CRS_PANEL_STORE
    const int ib = i0 + 32 * wa, jb = j0 + 32 * wb;
    if (kind == 0) {
        const EI* Aq = inA + s.oA + q * mm;
        cx<T>* Vo = W + s.oAo + oi * mm;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = ib + 16 * a + MF<T>::row(kr, v), j = jb + 16 * b + cc;
                    if (i < m && j <= i) {
                        const cx<T> x = cvt<T>(Aq[(int64_t)i * m + j]);
                        cx<T> o{x.r - acc.re(a, b, v), x.i - acc.im(a, b, v)};
                        if (i == j)
                            o.i = T(0);
                        Vo[(int64_t)i * m + j] = o;
                    }
                }
    } else {
        cx<T>* Fo = W + s.oBo + oi * mm;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = ib + 16 * a + MF<T>::row(kr, v), j = jb + 16 * b + cc;
                    if (i < m && j < m)
                        Fo[(int64_t)i * m + j] = cx<T>{-acc.re(a, b, v), -acc.im(a, b, v)};
                }
    }
}

// -------------------------------------------------------------- k_back_big

// One work-group per (eliminated block, 16-column strip of x_p), one wave per
// 16-row tile J of the block (blockDim = 64 x the largest tile count of the
// launch; waves beyond a block's S tiles only join the barriers):
//   phase A, all waves at once: w_J = g_J - Q_J x_{p-d} - P_J x_{p+d}, kept
//     in the MFMA accumulators;
//   phase B, bottom-up over the tiles I: wave I forms x_I = D_I^H w_I (the
//     accumulator is the right operand, see k_trsm_big), stores it and
//     publishes it in LDS; every wave J < I then applies
//     w_J -= L_IJ^H x_I (its operand loaded one step ahead).
// The block's serial chain is S short steps instead of S full tile sweeps.
template <class T, bool RE = false>
__global__ __launch_bounds__(1024) void k_back_big(const Seg* __restrict__ segs, int nseg,
                                                   int64_t total, int nstrip,
                                                   const cx<T>* __restrict__ W,
                                                   cx<T>* __restrict__ X,
                                                   const unsigned long long* __restrict__ flags,
                                                   cx<double>* __restrict__ U, int upd)
{
    using v4 = typename MF<T>::v4;
    __shared__ cx<T> sx[256]; // x_I, row-major 16 x 16
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int64_t li = xcd_item();
    const int64_t w = li / nstrip;
    const int u = (int)(li - w * nstrip);
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int64_t t = w - s.w0;
    const int p = s.e0 + (int)t * s.es;
    const int m = s.m, k = s.k, d = s.d, S = (m + 15) >> 4;
    const int c0 = 16 * u;
    if (c0 >= k)
        return;
    const int nc = min(16, k - c0);
    const bool hasPrev = p - d >= 0, hasNext = p + d < s.n;
    const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
    cx<T>* xp = X + s.ox + (s.xo + s.xs * p) * mk;
    cx<double>* up = upd ? U + s.oU + p * mk : nullptr;
    if (flags[s.sys] != kNoFail) {
        const T nan = T(NAN);
        for (int e = threadIdx.x; e < m * 16; e += blockDim.x)
            if ((e & 15) < nc) {
                const int64_t o = (e >> 4) * k + c0 + (e & 15);
                put_x<T>(xp, up, upd ? 1 : 0, o, cx<T>{nan, nan});
                if (upd && hasNext)
                    put_x<T>(xp, up + d * mk, 1, o, cx<T>{nan, nan});
            }
        return;
    }
    const cx<T>* xm = X + s.ox + (s.xo + s.xs * (p - d)) * mk;
    const cx<T>* xn = X + s.ox + (s.xo + s.xs * (p + d)) * mk;
    if (upd && hasNext) {
        // this strip's columns of the kept neighbour's correction (at most
        // four elements per thread: blockDim = 64 ceil(m / 16)), their loads
        // issued together before the stores
        cx<double>* uq = up + d * mk;
        cx<T> dv[4];
        cx<double> ov[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = threadIdx.x + u * blockDim.x;
            const bool ok = e < m * 16 && (e & 15) < nc;
            const int64_t o = ok ? (e >> 4) * k + c0 + (e & 15) : 0;
            dv[u] = xn[o];
            ov[u] = upd == 2 ? uq[o] : cx<double>{0.0, 0.0};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = threadIdx.x + u * blockDim.x;
            if (e < m * 16 && (e & 15) < nc)
                uq[(e >> 4) * k + c0 + (e & 15)] =
                    cx<double>{ov[u].r + (double)dv[u].r, ov[u].i + (double)dv[u].i};
        }
    }
    const cx<T>* L = W + s.oL + t * mm;
    const cx<T>* P = W + s.oP + t * mm;
    const cx<T>* Q = W + s.oQ + t * mm;
    const cx<T>* Dg = W + s.oD + t * (int64_t)S * 256;
    const cx<T>* g = W + s.og + t * mk;
    const bool own = wv < S;
    const int r0 = 16 * wv;
    // D_J^H operand of this wave's own tile: (D^H)[cc][rr] = conj(D[rr][cc])
    cx<T> aD[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
        aD[v] = own ? Dg[wv * 256 + MF<T>::row(kr, v) * 16 + cc] : czero<T>();
    // phase A
    Acc3<T, 1, 1, RE> acc;
    acc.zero();
    if (own && hasPrev)
        wave_mm3<T, 1, 1, false, false, 4, RE>(acc, WOp<T>{Q + (int64_t)r0 * m, m, 1, m - r0},
                                               WOp<T>{xm + c0, 1, k, nc}, m);
    if (own && hasNext)
        wave_mm3<T, 1, 1, false, false, 4, RE>(acc, WOp<T>{P + (int64_t)r0 * m, m, 1, m - r0},
                                               WOp<T>{xn + c0, 1, k, nc}, m);
    v4 wr, wi;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int r = r0 + MF<T>::row(kr, v);
        const cx<T> gv = (own && r < m && cc < nc) ? g[r * k + c0 + cc] : czero<T>();
        wr[v] = gv.r - acc.re(0, 0, v);
        wi[v] = gv.i - acc.im(0, 0, v);
    }
    // operand of the update at step I: A(i, t) = conj(L[16 I + t][r0 + i]),
    // lane (cc, kr) holds t = 4 s + kr for the contraction steps s
    auto load_l = [&](int I, cx<T>(&a)[4]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = 16 * I + 4 * q + kr;
            a[q] = (own && wv < I && row < m) ? L[(int64_t)row * m + r0 + cc] : czero<T>();
        }
    };
    cx<T> an[4];
    load_l(S - 1, an);
    // phase B
    for (int I = S - 1; I >= 0; --I) {
        cx<T> a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            a[q] = an[q];
        if (I > 0)
            load_l(I - 1, an);
        if (wv == I) {
            v4 xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cx<T> q = aD[v];
                xr = MF<T>::mma(q.r, wr[v], xr);
                if constexpr (!RE) {
                    xr = MF<T>::mma(q.i, wi[v], xr);
                    xi = MF<T>::mma(q.r, wi[v], xi);
                    xi = MF<T>::mma(-q.i, wr[v], xi);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = MF<T>::row(kr, v), r = r0 + rr;
                sx[rr * 16 + cc] = cx<T>{xr[v], xi[v]};
                if (r < m && cc < nc)
                    put_x<T>(xp, up, upd, (int64_t)r * k + c0 + cc, cx<T>{xr[v], xi[v]});
            }
        }
        __syncthreads();
        if (wv < I) {
            // w_J -= conj(L_IJ)^T x_I: contraction step q pairs t = 4 q + kr
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const cx<T> b = sx[(4 * q + kr) * 16 + cc];
                const T ar = a[q].r, ai = -a[q].i; // conj(L)
                wr = MF<T>::mma(-ar, b.r, wr);
                if constexpr (!RE) {
                    wr = MF<T>::mma(ai, b.i, wr);
                    wi = MF<T>::mma(-ar, b.i, wi);
                    wi = MF<T>::mma(-ai, b.r, wi);
                }
            }
        }
        __syncthreads();
    }
}

// -------------------------------------------------------------- k_grad_big

// gA_j = -lam_j x_j^H and gB_j = -(lam_{j+1} x_j^H + x_{j+1} lam_j^H), one
// wave per (block row j, 32 x 32 tile); whole-system segments as in k_grad.
template <class T>
__global__ __launch_bounds__(64) void k_grad_big(const Seg* __restrict__ segs, int nseg,
                                                 int64_t total, int ntile,
                                                 const cx<T>* __restrict__ X,
                                                 const cx<T>* __restrict__ Lam,
                                                 cx<T>* __restrict__ gA, cx<T>* __restrict__ gB)
{
    using v4 = typename MF<T>::v4;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
    const int64_t li = xcd_item();
    const int64_t w = li / ntile;
    const int u = (int)(li - w * ntile);
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int j = (int)(w - s.w0);
    const int m = s.m, k = s.k, n = s.n, T32 = (m + 31) >> 5;
    if (u >= T32 * T32)
        return;
    const int i0 = 32 * (u / T32), j0 = 32 * (u % T32);
    const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
    const cx<T>* l0 = Lam + s.oy + j * mk;
    const cx<T>* x0 = X + s.ox + j * mk;
    v4 cr[2][2], ci[2][2];
    zero_acc<T, 2, 2>(cr, ci);
    wave_mm<T, 2, 2, false, true, 2>(cr, ci, WOp<T>{l0 + (int64_t)i0 * k, k, 1, m - i0},
                                     WOp<T>{x0 + (int64_t)j0 * k, k, 1, m - j0}, k);
    cx<T>* ga = gA + s.oA + j * mm;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + 16 * a + MF<T>::row(kr, v), c = j0 + 16 * b + cc;
                if (i < m && c < m)
                    ga[i * m + c] = cx<T>{-cr[a][b][v], -ci[a][b][v]};
            }
    if (j + 1 >= n)
        return;
    zero_acc<T, 2, 2>(cr, ci);
    wave_mm<T, 2, 2, false, true, 2>(cr, ci, WOp<T>{l0 + mk + (int64_t)i0 * k, k, 1, m - i0},
                                     WOp<T>{x0 + (int64_t)j0 * k, k, 1, m - j0}, k);
    wave_mm<T, 2, 2, false, true, 2>(cr, ci, WOp<T>{x0 + mk + (int64_t)i0 * k, k, 1, m - i0},
                                     WOp<T>{l0 + (int64_t)j0 * k, k, 1, m - j0}, k);
    cx<T>* gb = gB + s.oB + j * mm;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + 16 * a + MF<T>::row(kr, v), c = j0 + 16 * b + cc;
                if (i < m && c < m)
                    gb[i * m + c] = cx<T>{-cr[a][b][v], -ci[a][b][v]};
            }
}

} // namespace crs
