// Kernels of the mixed-precision form: precision conversion jobs, the FP64
// residual r = y - A x of Eq. (Axb) with deterministic per-system norms, and
// the FP64 update x += d.
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

// One wave per (block row j, 16-row tile ti) of a system (segment n = N,
// oA/oB/ox/oy offsets into the caller's FP64 arrays, og the offset of r in
// R, ob0 the system's first partial-sum pair):
//   r_j = y_j - B_{j-1} x_{j-1} - A_j x_j - B_j^H x_{j+1}
// rows 16 ti .. 16 ti + 15, stored in R (unless R is null) as FP32 (r_f32)
// or FP64; with S = ceil(m / 16) tiles per row and it = j S + ti,
// part[2 (ob0 + it)] = ||rows of r_j||_F^2, part[2 (ob0 + it) + 1] = the
// same for y_j.  MFMA products, VALU products for k = 1.
__global__ __launch_bounds__(64) void k_residual(const Seg* __restrict__ segs, int nseg,
                                                 int64_t total, const cx<double>* __restrict__ A,
                                                 const cx<double>* __restrict__ B,
                                                 const cx<double>* __restrict__ X,
                                                 const cx<double>* __restrict__ Y,
                                                 void* __restrict__ R, int r_f32,
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
    const int m = s.m, k = s.k, n = s.n, S = (m + 15) >> 4;
    const int64_t it = w - s.w0;
    const int j = (int)(it / S), ti = (int)(it - (int64_t)j * S);
    const int r0 = 16 * ti;
    const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
    const cx<T>* Aj = A + s.oA + j * mm;
    const cx<T>* Bm = B + s.oB + (int64_t)(j - 1) * mm;
    const cx<T>* Bj = B + s.oB + (int64_t)j * mm;
    const cx<T>* xj = X + s.ox + j * mk;
    const cx<T>* yj = Y + s.oy + j * mk;
    double sr = 0.0, sy = 0.0;
    if (k == 1) {
        // one right-hand side: VALU products (an MFMA tile would use one of
        // its 16 columns).  Lane (kr, cc) sums the contraction indices
        // t = kr, kr + 4, ... of row i = r0 + cc with the loads of the MFMA
        // path (16 rows x 4 consecutive t per load), then the four kr lanes
        // of a row are combined.
        const int i = r0 + cc;
        const bool oi = i < m, hasM = j > 0, hasP = j + 1 < n;
        cx<T> acc = czero<T>();
#pragma unroll 4
        for (int tt = kr; tt < m; tt += 4) {
            cx<T> hv = czero<T>(), bm = czero<T>(), bp = czero<T>();
            if (oi) {
                hv = Aj[tt <= i ? i * m + tt : tt * m + i];
                hv.i = tt < i ? hv.i : (tt == i ? T(0) : -hv.i);
                if (hasM)
                    bm = Bm[i * m + tt];
                if (hasP) {
                    bp = Bj[tt * m + i];
                    bp.i = -bp.i; // (B_j^H)[i][t] = conj(B_j[t][i])
                }
            }
            const cx<T> x0 = xj[tt];
            const cx<T> xm = hasM ? xj[tt - mk] : czero<T>();
            const cx<T> xp = hasP ? xj[tt + mk] : czero<T>();
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
            if (R) {
                if (r_f32)
                    ((cx<float>*)R)[s.og + j * mk + i] = cx<float>{(float)r.r, (float)r.i};
                else
                    ((cx<double>*)R)[s.og + j * mk + i] = r;
            }
        }
    }
    for (int c0 = 0; c0 < k && k > 1; c0 += 16) {
        const int cw = min(16, k - c0);
        v4 cr[1][1], ci[1][1];
        zero_acc<T, 1, 1>(cr, ci);
        if (j > 0) // B_{j-1} x_{j-1}
            wave_mm<T, 1, 1, false, false, 4>(cr, ci, WOp<T>{Bm + r0 * m, m, 1, m - r0},
                                              WOp<T>{xj - mk + c0, 1, k, cw}, m);
        wave_mm_herm<T, 4>(cr[0][0], ci[0][0], Aj, m, r0, WOp<T>{xj + c0, 1, k, cw});
        if (j + 1 < n) // B_j^H x_{j+1}
            wave_mm<T, 1, 1, true, false, 4>(cr, ci, WOp<T>{Bj + r0, 1, m, m - r0},
                                             WOp<T>{xj + mk + c0, 1, k, cw}, m);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = r0 + MF<T>::row(kr, u), c = c0 + cc;
            if (i < m && c < k) {
                const cx<T> y = yj[i * k + c];
                const cx<T> r{y.r - cr[0][0][u], y.i - ci[0][0][u]};
                sr += r.r * r.r + r.i * r.i;
                sy += y.r * y.r + y.i * y.i;
                if (!R)
                    continue;
                if (r_f32)
                    ((cx<float>*)R)[s.og + j * mk + i * k + c] = cx<float>{(float)r.r, (float)r.i};
                else
                    ((cx<double>*)R)[s.og + j * mk + i * k + c] = r;
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

// norms[2 s + q] = sum over the n ceil(m / 16) partial-sum pairs of system s
// of part[2 (ob0 + e) + q], in a fixed order (one work-group per system).
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
    const int64_t ne = (int64_t)s.n * ((s.m + 15) >> 4);
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

// x = (assign ? 0 : x) + d over a flat range of complex elements.
__global__ __launch_bounds__(256) void k_update(cx<double>* __restrict__ x,
                                                const cx<float>* __restrict__ d, int64_t n,
                                                int assign)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * 256) {
        const cx<float> v = d[e];
        cx<double> o = assign ? cx<double>{0.0, 0.0} : x[e];
        o.r += (double)v.r;
        o.i += (double)v.i;
        x[e] = o;
    }
}

} // namespace crs
