// Host driver and C ABI of the block cyclic reduction library (crsolve.h).
//
// A plan fixes, for every system of a batch, the sequence of reduction levels
// and the layout of everything the levels write into the caller's workspace.
// Each level is a handful of launches (k_elim, k_reduce; k_back on the way
// back), one per block-size class present at that level; every launch covers
// all systems of its class through a segment table that lives in the
// workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/crsolve.h"
#include "kernels.hpp"
#include "kernels_fast.hpp"

using crs::cx;
using crs::Seg;

namespace {

constexpr int kNT = 256;
constexpr int kNumCls = 5;
constexpr int kClsM[kNumCls] = {4, 8, 16, 32, 64};
constexpr size_t kAlign = 256;
constexpr int kMaxGrid = 1 << 16; // work-group kernels loop grid-stride above this grid

int cls_of(int m)
{
    for (int c = 0; c < kNumCls; ++c)
        if (m <= kClsM[c])
            return c;
    return -1;
}

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Launch {
    int level;
    int cls;
    int seg0, nseg; // slice of the segment table
    int64_t total;  // work items
    bool from_user; // level inputs are the caller's arrays
};

// Per-system level geometry (one-sided schedule): n_0 = N, n_{l+1} = n_l / 2
// (floor), until n_l = 0.  Odd 1-based positions are eliminated at every
// level, even ones kept; an odd count eliminates its last block too, so no
// padding is needed.
std::vector<int> cr_levels(int N)
{
    std::vector<int> n;
    for (int v = N; v > 0; v /= 2)
        n.push_back(v);
    return n;
}

// Algorithm 1 in place: after level l position i couples with i +- 2^(l+1);
// levels run until 2^l >= N, when every block is uncoupled (the last level
// only factors and solves).
int pcr_depth(int N)
{
    int D = 0;
    while ((1ll << D) < N)
        ++D;
    return D;
}

} // namespace

struct crsolve_plan {
    int batch = 0;
    std::vector<int> N, m, k, cls;
    crsolve_dtype dtype = CRSOLVE_C128;
    crsolve_precision prec = CRSOLVE_PREC_NATIVE;
    crsolve_schedule sched = CRSOLVE_SCHED_CR;
    double rtol = 1e-12;
    int max_refine = 30;
    int tail = 8;
    size_t esz = 16; // bytes of one complex element

    // packed user arrays, complex-element offsets per system
    std::vector<int64_t> offA, offB, offy;

    // workspace layout (bytes)
    size_t off_flags = 0, off_segs = 0, ws_bytes = 0;

    std::vector<Seg> segs;                      // host copy of the segment table
    std::vector<Launch> elim, reduce, back, grad;
    int nlevels = 0;

    // per-kernel timing (crsolve_timing_enable / crsolve_timing_read)
    mutable bool timing = false;
    mutable std::vector<hipEvent_t> evpool;
    mutable size_t evused = 0;
    mutable std::vector<int> reckid; // kernel id of record i: events 2i, 2i+1

    ~crsolve_plan()
    {
        for (hipEvent_t e : evpool)
            (void)hipEventDestroy(e);
    }
};

namespace {

enum KernelId { KID_ELIM, KID_REDUCE, KID_BACK, KID_GRAD, KID_FLAGS, KID_FINAL, KID_COUNT };
const char* const kKernelName[KID_COUNT] = {"k_elim", "k_reduce", "k_back", "k_grad",
                                            "k_flags_init", "k_finalize"};

hipEvent_t pool_event(const crsolve_plan* p)
{
    if (p->evused == p->evpool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        p->evpool.push_back(e);
    }
    return p->evpool[p->evused++];
}

// Brackets one launch with two events when the plan's timing is enabled.
struct Timed {
    const crsolve_plan* p;
    hipStream_t st;
    hipEvent_t b = nullptr;
    Timed(const crsolve_plan* pp, int kid, hipStream_t s) : p(pp), st(s)
    {
        if (!p->timing)
            return;
        hipEvent_t a = pool_event(p);
        b = pool_event(p);
        if (!a || !b) {
            b = nullptr;
            return;
        }
        p->reckid.push_back(kid);
        (void)hipEventRecord(a, st);
    }
    ~Timed()
    {
        if (b)
            (void)hipEventRecord(b, st);
    }
};

template <class T>
struct Disp {
    template <int MT>
    static void elim(const Launch& L, const Seg* segs, const void* inA, const void* inB,
                     const void* iny, void* W, unsigned long long* flags, int mat, int rhs,
                     hipStream_t st)
    {
        int grid = (int)std::min<int64_t>(L.total, kMaxGrid);
        if constexpr (MT <= 32) {
            hipLaunchKernelGGL((crs::k_elim_w<T, MT>), dim3((unsigned)L.total), dim3(64), 0, st, segs + L.seg0,
                               L.nseg, L.total, (const cx<T>*)inA, (const cx<T>*)inB,
                               (const cx<T>*)iny, (cx<T>*)W, flags, mat, rhs);
        } else {
            constexpr int PW = sizeof(T) == 8 ? 32 : 64;
            hipLaunchKernelGGL((crs::k_elim<T, MT, kNT, PW>), dim3(grid), dim3(kNT), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const cx<T>*)inA,
                               (const cx<T>*)inB, (const cx<T>*)iny, (cx<T>*)W, flags, mat, rhs);
        }
    }
    template <int MT>
    static void reduce(const Launch& L, const Seg* segs, const void* inA, const void* iny, void* W,
                       const unsigned long long* flags, int mat, int rhs, hipStream_t st)
    {
        int grid = (int)std::min<int64_t>(L.total, kMaxGrid);
        if constexpr (MT == 16 || MT == 32) {
            hipLaunchKernelGGL((crs::k_reduce_m<T, MT>), dim3((unsigned)L.total), dim3(64), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const cx<T>*)inA,
                               (const cx<T>*)iny, (cx<T>*)W, flags, mat, rhs);
        } else if constexpr (MT == 64) {
            hipLaunchKernelGGL((crs::k_reduce_t<T, MT>), dim3((unsigned)L.total), dim3(64), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const cx<T>*)inA,
                               (const cx<T>*)iny, (cx<T>*)W, flags, mat, rhs);
        } else {
            hipLaunchKernelGGL((crs::k_reduce<T, MT, kNT>), dim3(grid), dim3(kNT), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const cx<T>*)inA,
                               (const cx<T>*)iny, (cx<T>*)W, flags, mat, rhs);
        }
    }
    template <int MT>
    static void back(const Launch& L, const Seg* segs, const void* W, void* X,
                     const unsigned long long* flags, hipStream_t st)
    {
        int grid = (int)std::min<int64_t>(L.total, kMaxGrid);
        if constexpr (MT == 16 || MT == 32) {
            hipLaunchKernelGGL((crs::k_back_m<T, MT>), dim3((unsigned)L.total), dim3(64), 0, st, segs + L.seg0,
                               L.nseg, L.total, (const cx<T>*)W, (cx<T>*)X, flags);
        } else {
            constexpr int PW = 32;
            hipLaunchKernelGGL((crs::k_back<T, MT, kNT, PW>), dim3(grid), dim3(kNT), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const cx<T>*)W, (cx<T>*)X, flags);
        }
    }
    template <int MT>
    static void grad(const Launch& L, const Seg* segs, const void* X, const void* Lam, void* gA,
                     void* gB, hipStream_t st)
    {
        int grid = (int)std::min<int64_t>(L.total, kMaxGrid);
        hipLaunchKernelGGL((crs::k_grad<T, MT, kNT>), dim3(grid), dim3(kNT), 0, st,
                           segs + L.seg0, L.nseg, L.total, (const cx<T>*)X, (const cx<T>*)Lam,
                           (cx<T>*)gA, (cx<T>*)gB);
    }
};

#define CRS_BY_CLASS(cls, CALL)                                                                    \
    switch (cls) {                                                                                 \
    case 0: CALL(4); break;                                                                        \
    case 1: CALL(8); break;                                                                        \
    case 2: CALL(16); break;                                                                       \
    case 3: CALL(32); break;                                                                       \
    default: CALL(64); break;                                                                      \
    }

struct Ctx {
    const crsolve_plan* p;
    char* ws;
    const Seg* dsegs;
    unsigned long long* flags;
    hipStream_t st;
};

template <class T>
void run_elim(const Ctx& c, const Launch& L, const void* A, const void* B, const void* y, int mat,
              int rhs)
{
    const void* inA = L.from_user ? A : c.ws;
    const void* inB = L.from_user ? B : c.ws;
    const void* iny = L.from_user ? y : c.ws;
    Timed tm(c.p, KID_ELIM, c.st);
#define CALL(MT) Disp<T>::template elim<MT>(L, c.dsegs, inA, inB, iny, c.ws, c.flags, mat, rhs, c.st)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

template <class T>
void run_reduce(const Ctx& c, const Launch& L, const void* A, const void* y, int mat, int rhs)
{
    const void* inA = L.from_user ? A : c.ws;
    const void* iny = L.from_user ? y : c.ws;
    Timed tm(c.p, KID_REDUCE, c.st);
#define CALL(MT) Disp<T>::template reduce<MT>(L, c.dsegs, inA, iny, c.ws, c.flags, mat, rhs, c.st)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

template <class T>
void run_back(const Ctx& c, const Launch& L, void* x)
{
    Timed tm(c.p, KID_BACK, c.st);
#define CALL(MT) Disp<T>::template back<MT>(L, c.dsegs, c.ws, x, c.flags, c.st)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

template <class T>
void run_grad(const Ctx& c, const Launch& L, const void* x, const void* lam, void* gA, void* gB)
{
    Timed tm(c.p, KID_GRAD, c.st);
#define CALL(MT) Disp<T>::template grad<MT>(L, c.dsegs, x, lam, gA, gB, c.st)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

__global__ void k_finalize(const unsigned long long* flags, crsolve_info* info, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        unsigned long long f = flags[i];
        crsolve_info v;
        v.status = f != crs::kNoFail;
        v.level = v.status ? (int32_t)(f >> 40) : -1;
        v.block = v.status ? (int64_t)(f & ((1ull << 40) - 1)) : -1;
        v.refine_iters = 0;
        v.fp64_fallback = 0;
        v.rel_residual = 0.0;
        info[i] = v;
    }
}

// ------------------------------------------------------------------ plan build

// Appends launches for one phase: for each level, one launch per class with
// work, segments contiguous in the table.  `count(s, lvl)` gives the work
// items of system s at level lvl (0 = none); `make(s, lvl)` its segment.
template <class Count, class Make>
void add_launches(crsolve_plan* p, std::vector<Launch>& out, int nlev, Count count, Make make)
{
    for (int lvl = 0; lvl < nlev; ++lvl)
        for (int c = 0; c < kNumCls; ++c) {
            Launch L{lvl, c, (int)p->segs.size(), 0, 0, lvl == 0};
            for (int s = 0; s < p->batch; ++s) {
                if (p->cls[s] != c)
                    continue;
                int64_t cnt = count(s, lvl);
                if (cnt <= 0)
                    continue;
                Seg g = make(s, lvl);
                g.w0 = L.total;
                L.total += cnt;
                p->segs.push_back(g);
                ++L.nseg;
            }
            if (L.nseg)
                out.push_back(L);
            else
                p->segs.resize(L.seg0);
        }
}

int build_plan(crsolve_plan* p)
{
    const size_t es = p->esz;
    size_t off = 0;
    p->off_flags = off;
    off = align_up(off + sizeof(unsigned long long) * p->batch);

    // per-system per-level workspace offsets (complex elements)
    struct Lv {
        int n, ne, nk;
        int64_t oL, oP, oQ, og, oAo, oBo, oyo; // outputs of this level
        int64_t oA, oB, oy;                    // inputs of this level (ws), level >= 1
    };
    std::vector<std::vector<Lv>> lv(p->batch);
    auto take = [&](int64_t elems) {
        int64_t o = (int64_t)(off / es);
        off = align_up(off + (size_t)elems * es);
        return o;
    };
    int maxlev = 0;
    for (int s = 0; s < p->batch; ++s) {
        const int64_t mm = (int64_t)p->m[s] * p->m[s], mk = (int64_t)p->m[s] * p->k[s];
        if (p->sched == CRSOLVE_SCHED_CR) {
            std::vector<int> ns = cr_levels(p->N[s]);
            lv[s].resize(ns.size());
            for (size_t l = 0; l < ns.size(); ++l) {
                Lv& v = lv[s][l];
                v.n = ns[l];
                v.ne = (v.n + 1) / 2;
                v.nk = v.n / 2;
                v.oL = take(v.ne * mm);
                v.oP = take(v.ne * mm);
                v.oQ = take(v.ne * mm);
                v.oAo = take(v.nk * mm);
                v.oBo = take(std::max(v.nk - 1, 0) * mm);
            }
            // right-hand-side scratch (solve phase)
            for (size_t l = 0; l < ns.size(); ++l) {
                Lv& v = lv[s][l];
                v.og = take(v.ne * mk);
                v.oyo = take(v.nk * mk);
            }
            for (size_t l = 1; l < ns.size(); ++l) {
                lv[s][l].oA = lv[s][l - 1].oAo;
                lv[s][l].oB = lv[s][l - 1].oBo;
                lv[s][l].oy = lv[s][l - 1].oyo;
            }
            maxlev = std::max<int>(maxlev, (int)ns.size());
        } else {
            const int N = p->N[s], D = pcr_depth(N);
            lv[s].resize(D + 1);
            int64_t oL = take(N * mm), oP = take(N * mm), oQ = take(N * mm), og = take(N * mk);
            int64_t bA[2], bB[2], by[2];
            for (int b = 0; b < 2; ++b) {
                bA[b] = take(N * mm);
                bB[b] = take(N * mm);
                by[b] = take(N * mk);
            }
            for (int l = 0; l <= D; ++l) {
                Lv& v = lv[s][l];
                v.n = N;
                v.ne = N;
                v.nk = l < D ? N : 0;
                v.oL = oL; v.oP = oP; v.oQ = oQ; v.og = og;
                v.oAo = bA[(l + 1) & 1]; v.oBo = bB[(l + 1) & 1]; v.oyo = by[(l + 1) & 1];
                v.oA = bA[l & 1]; v.oB = bB[l & 1]; v.oy = by[l & 1];
            }
            maxlev = std::max(maxlev, D + 1);
        }
    }
    p->nlevels = maxlev;

    auto seg_of = [&](int s, int l) {
        const Lv& v = lv[s][l];
        Seg g;
        std::memset(&g, 0, sizeof(g));
        g.n = v.n;
        g.m = p->m[s];
        g.k = p->k[s];
        g.level = l;
        g.sys = s;
        g.oL = v.oL; g.oP = v.oP; g.oQ = v.oQ; g.og = v.og;
        g.oAo = v.oAo; g.oBo = v.oBo; g.oyo = v.oyo;
        g.oA = l == 0 ? p->offA[s] : v.oA;
        g.oB = l == 0 ? p->offB[s] : v.oB;
        g.oy = l == 0 ? p->offy[s] : v.oy;
        g.ox = p->offy[s];
        if (p->sched == CRSOLVE_SCHED_CR) {
            g.d = 1;
            g.e0 = 0; g.es = 2; g.ne = v.ne;
            g.k0 = 1; g.ks = 2; g.nk = v.nk;
            g.out_by_pos = 0;
            g.xo = (1ll << l) - 1;
            g.xs = 1ll << l;
            g.ob0 = 1ll << l;
            g.obs = 1ll << l;
        } else {
            g.d = (int)std::min<int64_t>(1ll << l, (int64_t)1 << 30);
            g.e0 = 0; g.es = 1; g.ne = v.ne;
            g.k0 = 0; g.ks = 1; g.nk = v.nk;
            g.out_by_pos = 1;
            g.xo = 0;
            g.xs = 1;
            g.ob0 = 1;
            g.obs = 1;
        }
        return g;
    };
    auto has = [&](int s, int l) { return l < (int)lv[s].size(); };

    p->segs.clear();
    p->elim.clear();
    p->reduce.clear();
    p->back.clear();
    p->grad.clear();
    add_launches(p, p->elim, maxlev,
                 [&](int s, int l) -> int64_t { return has(s, l) ? lv[s][l].ne : 0; }, seg_of);
    add_launches(p, p->reduce, maxlev,
                 [&](int s, int l) -> int64_t { return has(s, l) ? lv[s][l].nk : 0; }, seg_of);
    // Recovery of the unknowns: the one-sided schedule back-substitutes at
    // every level; Algorithm 1 only solves the uncoupled blocks of its last
    // level (reassembly is the identity on the in-place layout).
    add_launches(p, p->back, maxlev,
                 [&](int s, int l) -> int64_t {
                     if (!has(s, l))
                         return 0;
                     if (p->sched == CRSOLVE_SCHED_PCR && l + 1 != (int)lv[s].size())
                         return 0;
                     return lv[s][l].ne;
                 },
                 seg_of);
    // gradient launches: one work item per block row of each system
    add_launches(p, p->grad, 1, [&](int s, int) -> int64_t { return p->N[s]; },
                 [&](int s, int) {
                     Seg g;
                     std::memset(&g, 0, sizeof(g));
                     g.n = p->N[s];
                     g.m = p->m[s];
                     g.k = p->k[s];
                     g.sys = s;
                     g.oA = p->offA[s];
                     g.oB = p->offB[s];
                     g.oy = p->offy[s];
                     g.ox = p->offy[s];
                     return g;
                 });
    p->off_segs = off;
    off = align_up(off + sizeof(Seg) * p->segs.size());
    p->ws_bytes = off;
    return CRSOLVE_OK;
}

int check_ws(const crsolve_plan* p, const void* ws, size_t ws_bytes)
{
    if (!ws || ((uintptr_t)ws % kAlign))
        return CRSOLVE_EINVAL;
    if (ws_bytes < p->ws_bytes)
        return CRSOLVE_EWORKSPACE;
    return CRSOLVE_OK;
}

bool aligned(const void* ptr, size_t a) { return ptr && ((uintptr_t)ptr % a) == 0; }

bool any_B(const crsolve_plan* p)
{
    for (int s = 0; s < p->batch; ++s)
        if (p->N[s] > 1)
            return true;
    return false;
}

int upload(const crsolve_plan* p, char* ws, hipStream_t st)
{
    if (hipMemcpyAsync(ws + p->off_segs, p->segs.data(), sizeof(Seg) * p->segs.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return CRSOLVE_EHIP;
    return CRSOLVE_OK;
}

int last_err()
{
    return hipGetLastError() == hipSuccess ? CRSOLVE_OK : CRSOLVE_EHIP;
}

Ctx make_ctx(const crsolve_plan* p, void* ws, void* stream)
{
    Ctx c;
    c.p = p;
    c.ws = (char*)ws;
    c.dsegs = (const Seg*)(c.ws + p->off_segs);
    c.flags = (unsigned long long*)(c.ws + p->off_flags);
    c.st = (hipStream_t)stream;
    return c;
}

template <class T>
void levels_down(const Ctx& c, const void* A, const void* B, const void* y, int mat, int rhs)
{
    const crsolve_plan* p = c.p;
    size_t ie = 0, ir = 0;
    for (int l = 0; l < p->nlevels; ++l) {
        for (; ie < p->elim.size() && p->elim[ie].level == l; ++ie)
            run_elim<T>(c, p->elim[ie], A, B, y, mat, rhs);
        for (; ir < p->reduce.size() && p->reduce[ir].level == l; ++ir)
            run_reduce<T>(c, p->reduce[ir], A, y, mat, rhs);
    }
}

template <class T>
void levels_up(const Ctx& c, void* x)
{
    const crsolve_plan* p = c.p;
    for (size_t i = p->back.size(); i-- > 0;)
        run_back<T>(c, p->back[i], x);
}

void finalize(const Ctx& c, crsolve_info* info)
{
    if (!info)
        return;
    int n = c.p->batch;
    Timed tm(c.p, KID_FINAL, c.st);
    hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, c.st, c.flags, info, n);
}

void init_flags(const Ctx& c)
{
    int n = c.p->batch;
    Timed tm(c.p, KID_FLAGS, c.st);
    hipLaunchKernelGGL(crs::k_flags_init, dim3((n + 255) / 256), dim3(256), 0, c.st, c.flags, n);
}

} // namespace

// ======================================================================= C ABI

extern "C" {

int crsolve_plan_create(const crsolve_desc* d, crsolve_plan** out)
{
    if (!d || !out || d->batch < 1 || !d->N || !d->m || !d->k)
        return CRSOLVE_EINVAL;
    if (d->dtype != CRSOLVE_C128 && d->dtype != CRSOLVE_C64)
        return CRSOLVE_EINVAL;
    if (d->precision != CRSOLVE_PREC_NATIVE && d->precision != CRSOLVE_PREC_FP32_REFINE)
        return CRSOLVE_EINVAL;
    if (d->schedule != CRSOLVE_SCHED_CR && d->schedule != CRSOLVE_SCHED_PCR)
        return CRSOLVE_EINVAL;
    if (d->precision == CRSOLVE_PREC_FP32_REFINE)
        return CRSOLVE_EUNSUPPORTED;
    if (d->schedule == CRSOLVE_SCHED_PCR &&
        (d->dtype != CRSOLVE_C128 || d->precision != CRSOLVE_PREC_NATIVE))
        return CRSOLVE_EUNSUPPORTED;
    for (int s = 0; s < d->batch; ++s) {
        if (d->N[s] < 1 || d->m[s] < 1 || d->k[s] < 1)
            return CRSOLVE_EINVAL;
        if (d->m[s] > 64)
            return CRSOLVE_EUNSUPPORTED;
        if ((int64_t)d->N[s] >= (1ll << 31) / 2)
            return CRSOLVE_EUNSUPPORTED;
    }
    crsolve_plan* p = new (std::nothrow) crsolve_plan();
    if (!p)
        return CRSOLVE_EINVAL;
    p->batch = d->batch;
    p->N.assign(d->N, d->N + d->batch);
    p->m.assign(d->m, d->m + d->batch);
    p->k.assign(d->k, d->k + d->batch);
    p->dtype = d->dtype;
    p->prec = d->precision;
    p->sched = d->schedule;
    p->rtol = d->rtol;
    p->max_refine = d->max_refine;
    p->tail = d->fp64_tail_blocks;
    p->esz = d->dtype == CRSOLVE_C128 ? 16 : 8;
    p->cls.resize(p->batch);
    int64_t oa = 0, ob = 0, oy = 0;
    for (int s = 0; s < p->batch; ++s) {
        p->cls[s] = cls_of(p->m[s]);
        p->offA.push_back(oa);
        p->offB.push_back(ob);
        p->offy.push_back(oy);
        oa += (int64_t)p->N[s] * p->m[s] * p->m[s];
        ob += (int64_t)(p->N[s] - 1) * p->m[s] * p->m[s];
        oy += (int64_t)p->N[s] * p->m[s] * p->k[s];
    }
    int rc = build_plan(p);
    if (rc != CRSOLVE_OK) {
        delete p;
        return rc;
    }
    *out = p;
    return CRSOLVE_OK;
}

int crsolve_workspace_size(const crsolve_plan* p, size_t* bytes)
{
    if (!p || !bytes)
        return CRSOLVE_EINVAL;
    *bytes = p->ws_bytes;
    return CRSOLVE_OK;
}

int crsolve_timing_enable(crsolve_plan* p, int enable)
{
    if (!p)
        return CRSOLVE_EINVAL;
    p->timing = enable != 0;
    p->evused = 0;
    p->reckid.clear();
    return CRSOLVE_OK;
}

int crsolve_timing_read(crsolve_plan* p, crsolve_kernel_time* out, int cap, int* n)
{
    if (!p || !n || (cap > 0 && !out))
        return CRSOLVE_EINVAL;
    int cnt[KID_COUNT] = {0};
    double ms[KID_COUNT] = {0};
    if (!p->reckid.empty() &&
        hipEventSynchronize(p->evpool[2 * p->reckid.size() - 1]) != hipSuccess)
        return CRSOLVE_EHIP;
    for (size_t i = 0; i < p->reckid.size(); ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, p->evpool[2 * i], p->evpool[2 * i + 1]) != hipSuccess)
            return CRSOLVE_EHIP;
        cnt[p->reckid[i]] += 1;
        ms[p->reckid[i]] += t;
    }
    int j = 0;
    for (int kid = 0; kid < KID_COUNT; ++kid) {
        if (!cnt[kid])
            continue;
        if (j < cap) {
            std::memset(out[j].name, 0, sizeof(out[j].name));
            std::strncpy(out[j].name, kKernelName[kid], sizeof(out[j].name) - 1);
            out[j].launches = cnt[kid];
            out[j].total_ms = ms[kid];
        }
        ++j;
    }
    *n = j;
    return CRSOLVE_OK;
}

int crsolve_plan_destroy(crsolve_plan* p)
{
    delete p;
    return CRSOLVE_OK;
}

const char* crsolve_error_string(int code)
{
    switch (code) {
    case CRSOLVE_OK: return "ok";
    case CRSOLVE_EINVAL: return "invalid argument";
    case CRSOLVE_EHIP: return "HIP runtime error";
    case CRSOLVE_EWORKSPACE: return "workspace too small";
    case CRSOLVE_EUNSUPPORTED: return "unsupported combination";
    case CRSOLVE_ESTATE: return "call out of order";
    default: return "unknown error";
    }
}

int crsolve_factor(crsolve_plan* p, const void* A, const void* B, void* ws, size_t ws_bytes,
                   crsolve_info* info, void* stream)
{
    if (!p)
        return CRSOLVE_EINVAL;
    if (p->sched != CRSOLVE_SCHED_CR)
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!aligned(A, p->esz) || (any_B(p) && !aligned(B, p->esz)))
        return CRSOLVE_EINVAL;
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    init_flags(c);
    if (p->dtype == CRSOLVE_C128)
        levels_down<double>(c, A, B, nullptr, 1, 0);
    else
        levels_down<float>(c, A, B, nullptr, 1, 0);
    finalize(c, info);
    return last_err();
}

int crsolve_solve(const crsolve_plan* p, void* ws, size_t ws_bytes, const void* A, const void* B,
                  const void* y, void* x, crsolve_info* info, void* stream)
{
    (void)A;
    (void)B;
    (void)info;
    if (!p)
        return CRSOLVE_EINVAL;
    if (p->sched != CRSOLVE_SCHED_CR)
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!aligned(y, p->esz) || !aligned(x, p->esz))
        return CRSOLVE_EINVAL;
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    if (p->dtype == CRSOLVE_C128) {
        levels_down<double>(c, nullptr, nullptr, y, 0, 1);
        levels_up<double>(c, x);
    } else {
        levels_down<float>(c, nullptr, nullptr, y, 0, 1);
        levels_up<float>(c, x);
    }
    return last_err();
}

int crsolve_factor_solve(crsolve_plan* p, const void* A, const void* B, const void* y, void* ws,
                         size_t ws_bytes, void* x, crsolve_info* info, void* stream)
{
    if (!p)
        return CRSOLVE_EINVAL;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!aligned(A, p->esz) || (any_B(p) && !aligned(B, p->esz)) || !aligned(y, p->esz) ||
        !aligned(x, p->esz))
        return CRSOLVE_EINVAL;
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    init_flags(c);
    if (p->dtype == CRSOLVE_C128) {
        levels_down<double>(c, A, B, y, 1, 1);
        levels_up<double>(c, x);
    } else {
        levels_down<float>(c, A, B, y, 1, 1);
        levels_up<float>(c, x);
    }
    finalize(c, info);
    return last_err();
}

int crsolve_backward(const crsolve_plan* p, void* ws, size_t ws_bytes, const void* x,
                     const void* grad_x, void* grad_y, void* grad_A, void* grad_B, void* stream)
{
    if (!p)
        return CRSOLVE_EINVAL;
    if (p->sched != CRSOLVE_SCHED_CR || p->prec != CRSOLVE_PREC_NATIVE)
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!aligned(x, p->esz) || !aligned(grad_x, p->esz) || !aligned(grad_y, p->esz) ||
        !aligned(grad_A, p->esz) || (any_B(p) && !aligned(grad_B, p->esz)))
        return CRSOLVE_EINVAL;
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    // lam = A^{-1} grad_x with the stored factors, written straight into grad_y
    if (p->dtype == CRSOLVE_C128) {
        levels_down<double>(c, nullptr, nullptr, grad_x, 0, 1);
        levels_up<double>(c, grad_y);
        for (const Launch& L : p->grad)
            run_grad<double>(c, L, x, grad_y, grad_A, grad_B);
    } else {
        levels_down<float>(c, nullptr, nullptr, grad_x, 0, 1);
        levels_up<float>(c, grad_y);
        for (const Launch& L : p->grad)
            run_grad<float>(c, L, x, grad_y, grad_A, grad_B);
    }
    return last_err();
}

} // extern "C"
