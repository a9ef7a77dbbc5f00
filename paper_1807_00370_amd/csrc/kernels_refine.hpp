// Kernels of the mixed-precision form: precision conversion jobs, the FP64
// residual r = y - A x of Eq. (Axb) with deterministic per-system norms, and
// the FP64 update x += d.
#pragma once

#include "kernels_fast.hpp"

namespace crs {

// A flat range of complex elements copied with a change of precision.
struct CvtJob {
    int64_t w0;      // first element of this job within the launch
    int64_t src;     // element offset in the source array
    int64_t dst;     // element offset in the destination array
    int64_t count;   // complex elements
};

template <class Ts, class Td>
__global__ __launch_bounds__(256) void k_convert(const CvtJob* __restrict__ jobs, int njobs,
                                                 int64_t total, const cx<Ts>* __restrict__ src,
                                                 cx<Td>* __restrict__ dst)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * 256) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].w0 <= e)
                lo = mid;
            else
                hi = mid - 1;
        }
        const CvtJob& j = jobs[lo];
        const int64_t i = e - j.w0;
        const cx<Ts> v = src[j.src + i];
        dst[j.dst + i] = cx<Td>{(Td)v.r, (Td)v.i};
    }
}

// (cr, ci) += H X on a tile, where H is the Hermitian matrix read from the
// lower triangle and the real diagonal of the m x m block A (row-major):
// H[i][t] = A[i][t] (t < i), Re A[i][i] (t = i), conj(A[t][i]) (t > i).
template <int KS>
__device__ __forceinline__ void tile_herm(typename MF<double>::v4& cr, typename MF<double>::v4& ci,
                                          const cx<double>* __restrict__ A, int m, int rx0,
                                          const cx<double>* __restrict__ Y, int ldy, int ncy,
                                          int kd)
{
    using T = double;
    const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
    const int ar = rx0 + cc;
    const bool okx = ar < m, oky = cc < ncy;
    const cx<T>* yq = Y + (kr * ldy + cc);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        const int t = 4 * s + kr;
        cx<T> a = czero<T>();
        if (okx && t < kd) {
            const int idx = t <= ar ? ar * m + t : t * m + ar;
            a = A[idx];
            if (t > ar)
                a.i = -a.i;
            else if (t == ar)
                a.i = T(0);
        }
        const cx<T> b = (t < kd && oky) ? yq[s * 4 * ldy] : czero<T>();
        cr = MF<T>::mma(a.r, b.r, cr);
        cr = MF<T>::mma(-a.i, b.i, cr);
        ci = MF<T>::mma(a.r, b.i, ci);
        ci = MF<T>::mma(a.i, b.r, ci);
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o);
    return v;
}

// One wave per block row j of a system (segment n = N, oA/oB/ox/oy offsets
// into the caller's FP64 arrays, og the offset of r in R, ob0 the first row
// of the system in the norm partials):
//   r_j = y_j - B_{j-1} x_{j-1} - A_j x_j - B_j^H x_{j+1}
// stored in R (unless R is null) as FP32 (r_f32) or FP64;
// part[2 (ob0 + j)] = ||r_j||_F^2 and
// part[2 (ob0 + j) + 1] = ||y_j||_F^2.
template <int MT>
__global__ __launch_bounds__(64, 2) void k_residual(const Seg* __restrict__ segs, int nseg,
                                                    int64_t total, const cx<double>* __restrict__ A,
                                                    const cx<double>* __restrict__ B,
                                                    const cx<double>* __restrict__ X,
                                                    const cx<double>* __restrict__ Y,
                                                    void* __restrict__ R, int r_f32,
                                                    double* __restrict__ part)
{
    using T = double;
    using v4 = typename MF<T>::v4;
    constexpr int MTT = MT < 16 ? 16 : MT, KS = MTT / 4, NT16 = MTT / 16;
    const int lane = threadIdx.x, kr = lane >> 4, cc = lane & 15;
    const int64_t w = blockIdx.x;
    if (w >= total)
        return;
    const Seg& s = segs[find_seg(segs, nseg, w)];
    const int j = (int)(w - s.w0);
    const int m = s.m, k = s.k, n = s.n;
    const int64_t mm = (int64_t)m * m, mk = (int64_t)m * k;
    const cx<T>* Aj = A + s.oA + j * mm;
    const cx<T>* Bm = B + s.oB + (int64_t)(j - 1) * mm;
    const cx<T>* Bj = B + s.oB + (int64_t)j * mm;
    const cx<T>* xj = X + s.ox + j * mk;
    const cx<T>* yj = Y + s.oy + j * mk;
    const v4 z4 = {0, 0, 0, 0};
    double sr = 0.0, sy = 0.0;
    for (int ti = 0; ti < NT16; ++ti) {
        if (16 * ti >= m)
            break;
        for (int c0 = 0; c0 < k; c0 += 16) {
            const int cw = min(16, k - c0);
            v4 cr = z4, ci = z4;
            if (j > 0)
                tile_nn<T, KS>(cr, ci, Bm, m, m, 16 * ti, xj - mk + c0, k, cw, 0, m);
            tile_herm<KS>(cr, ci, Aj, m, 16 * ti, xj + c0, k, cw, m);
            if (j + 1 < n)
                tile_hn<T, KS>(cr, ci, Bj, m, m, 16 * ti, xj + mk + c0, k, cw, 0, m);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = 16 * ti + MF<T>::row(kr, u), c = c0 + cc;
                if (i < m && c < k) {
                    const cx<T> y = yj[i * k + c];
                    const cx<T> r{y.r - cr[u], y.i - ci[u]};
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
    }
    sr = wave_sum(sr);
    sy = wave_sum(sy);
    if (lane == 0) {
        part[2 * (s.ob0 + j)] = sr;
        part[2 * (s.ob0 + j) + 1] = sy;
    }
}

// norms[2 s + q] = sum over the block rows j < n of system s of
// part[2 (ob0 + j) + q], in a fixed order (one work-group per system).
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
    for (int j = threadIdx.x; j < s.n; j += 256) {
        a += part[2 * (s.ob0 + j)];
        b += part[2 * (s.ob0 + j) + 1];
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
