// Kernels of the mixed-precision form: precision conversion jobs (the
// reduced system at the first FP64 level and the FP64 tail's unknowns), and
// the FP64 residual r = y - A x of Eq. (Axb) with deterministic per-system
// norms.  The update x += d is part of the level-0 back substitution.
#pragma once

#include "kernels_big.hpp"

namespace crs {

// A flat range of complex elements copied with a change of precision.
struct CvtJob {
    int64_t w0;      // first element of this job within the launch
    int64_t src;     // element offset in the source array
    int64_t dst;     // element offset in the destination array
    int64_t count;   // complex elements
};

// Each work-group converts ranges of kCvtPer * 256 consecutive elements: the
// job of a range's first element is found once (binary search by thread 0),
// later elements advance through the job table linearly.
constexpr int kCvtPer = 8;

template <class Ts, class Td>
__global__ __launch_bounds__(256) void k_convert(const CvtJob* __restrict__ jobs, int njobs,
                                                 int64_t total, const cx<Ts>* __restrict__ src,
                                                 cx<Td>* __restrict__ dst)
{
    __shared__ int sj;
    constexpr int64_t R = 256 * kCvtPer;
    for (int64_t base = (int64_t)blockIdx.x * R; base < total; base += (int64_t)gridDim.x * R) {
        if (threadIdx.x == 0) {
            int lo = 0, hi = njobs - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].w0 <= base)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            sj = lo;
        }
        __syncthreads();
        int j = sj;
#pragma unroll
        for (int q = 0; q < kCvtPer; ++q) {
            const int64_t e = base + q * 256 + threadIdx.x;
            if (e < total) {
                while (j + 1 < njobs && jobs[j + 1].w0 <= e)
                    ++j;
                const CvtJob& jb = jobs[j];
                const int64_t i = e - jb.w0;
                const cx<Ts> v = src[jb.src + i];
                dst[jb.dst + i] = cx<Td>{(Td)v.r, (Td)v.i};
            }
        }
        __syncthreads(); // sj is rewritten for the next range
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// Work items per block row of the residual: for k = 1 one per 16-row tile
// (VALU products), otherwise one per 16-column strip of the right-hand side,
// with every row tile of the block row in the same wave so that x_{j-1},
// x_j and x_{j+1} are read once per strip.
__host__ __device__ inline int resid_items(int m, int k)
{
    return k == 1 ? (m + 15) >> 4 : (k + 15) >> 4;
}

// (cr, ci)[a] += H Y for the RM tiles of 16 rows at row0 + 16 a of the
// Hermitian matrix H read from the lower triangle and the real diagonal of
// the m x m row-major block A (H[i][t] = A[i][t] for t < i, Re A[i][i],
// conj(A[t][i]) for t > i) and the right operand Y (as in wave_mm); the
// contraction runs over all m columns.
template <class T, int RM, int G>
__device__ __forceinline__ void wave_mm_herm_r(typename MF<T>::v4 (&cr)[RM][1],
                                               typename MF<T>::v4 (&ci)[RM][1],
                                               const cx<T>* __restrict__ A, int m, int row0,
                                               const WOp<T> B)
{
    const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int ng = (m + 4 * G - 1) / (4 * G);
    const bool ob = cc < B.no;
    const cx<T>* pb = B.p + ((ob ? cc : 0) * B.so + kr * B.st);
    const int sb = 4 * B.st;
    cx<T> xa0[RM][G], yb0[G], xa1[RM][G], yb1[G];
    auto load = [&](cx<T>(&xa)[RM][G], cx<T>(&yb)[G], int g) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int t = 4 * (g * G + u) + kr;
#pragma unroll
            for (int a = 0; a < RM; ++a) {
                const int i = row0 + 16 * a + cc;
                cx<T> v = ld_or0(A + (t <= i ? i * m + t : t * m + i), A, t < m && i < m);
                v.i = t < i ? v.i : (t == i ? T(0) : -v.i);
                xa[a][u] = v;
            }
            yb[u] = ld_or0(pb + (g * G + u) * sb, B.p, t < m && ob);
        }
    };
    auto comp = [&](const cx<T>(&xa)[RM][G], const cx<T>(&yb)[G]) {
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int a = 0; a < RM; ++a) {
                cr[a][0] = MF<T>::mma(xa[a][u].r, yb[u].r, cr[a][0]);
                cr[a][0] = MF<T>::mma(-xa[a][u].i, yb[u].i, cr[a][0]);
                ci[a][0] = MF<T>::mma(xa[a][u].r, yb[u].i, ci[a][0]);
                ci[a][0] = MF<T>::mma(xa[a][u].i, yb[u].r, ci[a][0]);
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

// The FP64 residual of Eq. (Axb) for the systems of a launch (segment n = N,
// oA/oB/ox/oy offsets into the caller's FP64 arrays, og the offset of r in
// R, ob0 the system's first partial-sum pair):
//   r_j = y_j - B_{j-1} x_{j-1} - A_j x_j - B_j^H x_{j+1},
// stored in R (FP64, laid out like y) unless R is null.  One wave per work
// item (resid_items per block row; it = j * items + item): for k = 1 the
// 16-row tile `item` on VALU products, otherwise the 16-column strip `item`
// with its RM row tiles at a time on MFMA.  part[2 (ob0 + it)] = the item's
// ||r||_F^2, part[2 (ob0 + it) + 1] = the same for y.
template <int RM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_residual(const Seg* __restrict__ segs, int nseg,
                                                 int64_t total, const cx<double>* __restrict__ A,
                                                 const cx<double>* __restrict__ B,
                                                 const cx<double>* __restrict__ X,
                                                 const cx<double>* __restrict__ Y,
                                                 cx<double>* __restrict__ R,
                                                 double* __restrict__ part)
{
    using T = double;
    using v4 = typename MF<T>::v4;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
    // consecutive block rows (which share B_j and x_j) run on one XCD
    const int64_t w = xcd_item();
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int m = s.m, k = s.k, n = s.n, ni = resid_items(m, k);
    const int64_t it = w - s.w0;
    const int j = (int)(it / ni), item = (int)(it - (int64_t)j * ni);
    const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
    const cx<T>* Aj = A + s.oA + j * mm;
    const cx<T>* Bm = B + s.oB + (int64_t)(j - 1) * mm;
    const cx<T>* Bj = B + s.oB + (int64_t)j * mm;
    const cx<T>* xj = X + s.ox + j * mk;
    const cx<T>* yj = Y + s.oy + j * mk;
    cx<T>* rj = R ? R + s.og + j * mk : nullptr;
    double sr = 0.0, sy = 0.0;
    if (k == 1) {
        // one right-hand side: VALU products (an MFMA tile would use one of
        // its 16 columns).  Lane (kr, cc) sums the contraction indices
        // t = kr, kr + 4, ... of row i = 16 item + cc (16 rows x 4
        // consecutive t per load), then the four kr lanes of a row combine.
        const int i = 16 * item + cc;
        const bool oi = i < m, hasM = j > 0, hasP = j + 1 < n;
        cx<T> acc = czero<T>();
#pragma unroll 4
        for (int tt = kr; tt < m; tt += 4) {
            cx<T> hv = ld_or0(Aj + (tt <= i ? i * m + tt : tt * m + i), Aj, oi);
            hv.i = tt < i ? hv.i : (tt == i ? T(0) : -hv.i);
            const cx<T> bm = ld_or0(Bm + i * m + tt, Aj, oi && hasM);
            cx<T> bp = ld_or0(Bj + tt * m + i, Aj, oi && hasP);
            bp.i = -bp.i; // (B_j^H)[i][t] = conj(B_j[t][i])
            const cx<T> x0 = xj[tt];
            const cx<T> xm = ld_or0(xj + tt - mk, xj, hasM);
            const cx<T> xp = ld_or0(xj + tt + mk, xj, hasP);
            acc.r += hv.r * x0.r - hv.i * x0.i + bm.r * xm.r - bm.i * xm.i + bp.r * xp.r -
                     bp.i * xp.i;
            acc.i += hv.r * x0.i + hv.i * x0.r + bm.r * xm.i + bm.i * xm.r + bp.r * xp.i +
                     bp.i * xp.r;
        }
        acc.r += __shfl_xor(acc.r, 16);
        acc.i += __shfl_xor(acc.i, 16);
        acc.r += __shfl_xor(acc.r, 32);
        acc.i += __shfl_xor(acc.i, 32);
        if (kr == 0 && oi) {
            const cx<T> y = yj[i];
            const cx<T> r{y.r - acc.r, y.i - acc.i};
            sr += r.r * r.r + r.i * r.i;
            sy += y.r * y.r + y.i * y.i;
            if (rj)
                rj[i] = r;
        }
    } else {
        const int c0 = 16 * item, cw = min(16, k - c0);
        constexpr int G = RM >= 2 ? 2 : 4;
        // B_j is read by rows j (as B_j^H) and j + 1 (as B_j), which run
        // side by side on one XCD: an even row takes its products in the
        // order B_{j-1}, A_j, B_j^H and an odd row in the reverse order, so
        // both readers of a B_j fetch it at the same phase of their lives and
        // the second read finds it in L2.
        const bool odd = j & 1;
        for (int r0 = 0; r0 < m; r0 += 16 * RM) {
            v4 cr[RM][1], ci[RM][1];
            zero_acc<T, RM, 1>(cr, ci);
            auto prev = [&] { // B_{j-1} x_{j-1}
                if (j > 0)
                    wave_mm<T, RM, 1, false, false, G>(cr, ci, WOp<T>{Bm + (int64_t)r0 * m, m, 1, m - r0},
                                                       WOp<T>{xj - mk + c0, 1, k, cw}, m);
            };
            auto next = [&] { // B_j^H x_{j+1}
                if (j + 1 < n)
                    wave_mm<T, RM, 1, true, false, G>(cr, ci, WOp<T>{Bj + r0, 1, m, m - r0},
                                                      WOp<T>{xj + mk + c0, 1, k, cw}, m);
            };
            if (odd)
                next();
            else
                prev();
            wave_mm_herm_r<T, RM, G>(cr, ci, Aj, m, r0, WOp<T>{xj + c0, 1, k, cw});
            if (odd)
                prev();
            else
                next();
            // y's elements loaded together, in every lane (element 0 stands
            // in), before the first store of r: one round trip, not one per
            // element behind the previous store
            cx<T> yv[RM][4];
#pragma unroll
            for (int a = 0; a < RM; ++a)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = r0 + 16 * a + MF<T>::row(kr, u), c = c0 + cc;
                    yv[a][u] = yj[(i < m && c < k) ? i * k + c : 0];
                }
#pragma unroll
            for (int a = 0; a < RM; ++a)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int i = r0 + 16 * a + MF<T>::row(kr, u), c = c0 + cc;
                    if (i < m && c < k) {
                        const cx<T> y = yv[a][u];
                        const cx<T> r{y.r - cr[a][0][u], y.i - ci[a][0][u]};
                        sr += r.r * r.r + r.i * r.i;
                        sy += y.r * y.r + y.i * y.i;
                        if (rj)
                            rj[i * k + c] = r;
                    }
                }
        }
    }
    sr = wave_sum(sr);
    sy = wave_sum(sy);
    if (lane == 0) {
        part[2 * (s.ob0 + it)] = sr;
        part[2 * (s.ob0 + it) + 1] = sy;
    }
}

// norms[2 s + q] = sum over the n resid_items(m, k) partial-sum pairs of
// system s of part[2 (ob0 + e) + q], in a fixed order (one work-group per
// system).
__global__ __launch_bounds__(256) void k_norms(const Seg* __restrict__ segs, int nseg,
                                               const double* __restrict__ part,
                                               double* __restrict__ norms)
{
    __shared__ double sh[2][256];
    const int sidx = blockIdx.x;
    if (sidx >= nseg)
        return;
    const Seg& s = segs[sidx];
    double a = 0.0, b = 0.0;
    const int64_t ne = (int64_t)s.n * resid_items(s.m, s.k);
    const double2* pp = (const double2*)part + s.ob0;
    // eight loads in flight per thread, summed in a fixed order
    constexpr int U = 8;
    int64_t e0 = threadIdx.x;
    for (; e0 + 256 * (U - 1) < ne; e0 += 256 * U) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = pp[e0 + 256 * u];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a += v[u].x;
            b += v[u].y;
        }
    }
    for (; e0 < ne; e0 += 256) {
        a += pp[e0].x;
        b += pp[e0].y;
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        norms[2 * s.sys] = sh[0][0];
        norms[2 * s.sys + 1] = sh[1][0];
    }
}

} // namespace crs
