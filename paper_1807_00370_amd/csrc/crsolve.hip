// Host driver and C ABI of the block cyclic reduction library (crsolve.h).
//
// A plan fixes, for every system of a batch, the sequence of reduction levels
// (one-sided: n_{l+1} = floor(n_l / 2) until no block is left; Algorithm 1:
// in place with doubling neighbour distance), the precision of each level and
// the layout of everything the levels write into the caller's workspace.
// Each level is a handful of launches (k_elim, k_reduce; k_back on the way
// back), one per (block-size class, precision) present at that level; every
// launch covers all its systems through a segment table in the workspace.
//
// The mixed-precision form adds conversion jobs (level-0 inputs to FP32, the
// reduced system back to FP64 at the first FP64 level, the FP64 tail's
// unknowns into the FP32 correction), the FP64 residual of Eq. (Axb) and a
// host-driven refinement loop.  A system whose FP32 factorization breaks down,
// or whose refinement stalls or misses the tolerance, is solved again by a
// one-system FP64 plan in a workspace region sized for the largest system.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <mutex>
#include <string>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "../../include/crsolve.h"
#include "kernels.hpp"
#include "kernels_fast.hpp"
#include "kernels_refine.hpp"
#include "kernels_big.hpp"

using crs::CvtJob;
using crs::cx;
using crs::Seg;

namespace {

constexpr int kNT = 256;
constexpr int kNumCls = 6;
constexpr int kClsM[kNumCls] = {4, 8, 16, 32, 64, 256};
constexpr int kBig = 5; // block sizes 64 < m <= 256
// Classes whose elimination, back substitution and gradient run on the tiled
// kernels of kernels_big.hpp (full m x m L slots plus inverse diagonal tiles);
// their reduced-system step takes the tiled kernel as variant 0.
bool tiled(int cls) { return cls >= 4; }
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
    int f64;         // kernels instantiated in double (1) or float (0)
    int seg0, nseg;  // slice of the segment table
    int64_t total;   // work items
    bool userAB;     // matrix inputs are the caller's arrays
    bool userY;      // right-hand-side input is the caller's array
    bool userX;      // unknowns are written to the caller's x
    bool in64;       // the level's inputs are FP64 (FP32 levels round on load)
    bool upd;        // mixed form, level 0: corrections go into the FP64 x
    bool inreal;     // the level's inputs are the caller's real arrays
};

struct CvtLaunch {
    int f64_src, f64_dst;
    bool user_src;   // source is a caller array (level-0 inputs)
    int which;       // 0: A, 1: B, 2: y (selects the caller array)
    int job0, njobs;
    int64_t total;
};

// One level of one system.
struct LevelSpec {
    int n = 0, ne = 0, nk = 0;
    int f64 = 1;
    int64_t oL = 0, oP = 0, oQ = 0, og = 0, oAo = 0, oBo = 0, oyo = 0; // ws, level type
    int64_t oD = 0;                                                   // big blocks only
    int64_t oA = 0, oB = 0, oy = 0;                                   // inputs, level type
    bool userAB = false, userY = false, userX = false;
    bool in64 = false, upd = false, inreal = false;
    int64_t ox = 0, xo = 0, xs = 1;
    int64_t oU = 0;
    // Algorithm 1 in place (the PCR schedule, or the tail of the one-sided
    // schedule): neighbour distance d, position p is original block
    // obs (p + 1) (1-based)
    bool pcr = false;
    int d = 1;
    int64_t obs = 1;
};

// Algorithm 1 in place: levels run until 2^l >= N, when every block is
// uncoupled (the last level only factors and solves).
int pcr_depth(int N)
{
    int D = 0;
    while ((1ll << D) < N)
        ++D;
    return D;
}

enum KernelId {
    KID_ELIM,
    KID_REDUCE,
    KID_BACK,
    KID_GRAD,
    KID_FLAGS,
    KID_FINAL,
    KID_CONVERT,
    KID_RESIDUAL,
    KID_NORMS,
    KID_POTRF,
    KID_TRSM,
    KID_REALOUT,
    KID_COUNT
};
const char* const kKernelName[KID_COUNT] = {"k_elim",       "k_reduce",   "k_back",
                                            "k_grad",       "k_flags_init", "k_finalize",
                                            "k_convert",    "k_residual", "k_norms",
                                            "k_potrf_big",  "k_trsm_big", "k_real_out"};

} // namespace

struct crsolve_plan {
    int batch = 0;
    std::vector<int> N, m, k, cls;
    crsolve_dtype dtype = CRSOLVE_C128;
    bool real = false;    // real symmetric dtypes (R64, R32)
    size_t off_xc = 0;    // real dtypes: the unknowns, complex like y, before Re -> x
    crsolve_precision prec = CRSOLVE_PREC_NATIVE;
    crsolve_schedule sched = CRSOLVE_SCHED_CR;
    double rtol = 1e-12;
    int max_refine = 30;
    int tail = 8;
    int hyb = 0; // one-sided schedule: Algorithm 1 below this many blocks

    // packed caller arrays: complex-element offsets per system
    std::vector<int64_t> offA, offB, offy;
    int64_t totA = 0, totB = 0, toty = 0, totN = 0;

    // workspace layout (bytes)
    size_t off_flags = 0, off_segs = 0, off_jobs = 0, ws_bytes = 0;
    size_t off_part = 0, off_norms = 0, off_info = 0, off_fb = 0;
    size_t off_d32 = 0;   // refinement correction (complex FP32, like y)
    size_t off_r64 = 0;   // refinement residual r = y - A x (complex FP64, like y)
    size_t off_fbits = 0; // refinement: int32 per system, 1 = solved by its FP64 plan

    std::vector<std::vector<LevelSpec>> lv; // per system
    std::vector<int> sw;                    // first FP64 level per system (refine)
    std::vector<Seg> segs;
    std::vector<CvtJob> jobs;
    std::vector<Launch> elim, reduce, back, grad, resid;
    int norm_seg0 = 0;
    std::vector<std::vector<CvtLaunch>> cvt_factor_sw, cvt_solve_sw, scatter_sw;
    int nlevels = 0;

    // refinement: one FP64 plan per system, run in the region at off_fb
    // (sized for the largest system) for the systems that fall back
    std::vector<std::unique_ptr<crsolve_plan>> fbs;

    // workspaces this plan has factored (host record; solve and backward on
    // any other workspace return CRSOLVE_ESTATE)
    mutable std::vector<const void*> factored;
    void mark_factored(const void* ws) const
    {
        if (std::find(factored.begin(), factored.end(), ws) == factored.end())
            factored.push_back(ws);
    }
    bool is_factored(const void* ws) const
    {
        return std::find(factored.begin(), factored.end(), ws) != factored.end();
    }

    // kernel variant per (role: elim, reduce, back; class; precision):
    // 0 = one-wave / MFMA kernels, 1 = work-group kernels (autotuner)
    int var[3][kNumCls][2] = {};
    // launch shapes of the levels with few blocks (autotuner): waves per
    // level for the split elimination, block count below which the reduced
    // system is formed one wave per 16 x 16 tile
    int64_t tail_waves = 2048, tail_blocks = 1024;

    // recorded HIP graphs (crsolve_set_graphs)
    struct GraphEntry {
        std::vector<const void*> key;
        hipGraphExec_t exec;
    };
    bool graphs_on = false;
    mutable std::vector<GraphEntry> graphs;
    mutable hipStream_t cap_stream = nullptr;

    // per-kernel timing (crsolve_timing_enable / crsolve_timing_read)
    mutable bool timing = false;
    mutable std::vector<hipEvent_t> evpool;
    mutable size_t evused = 0;
    mutable std::vector<int> reckid;
    crsolve_plan* timing_parent = nullptr;

    void drop_graphs() const
    {
        for (GraphEntry& g : graphs)
            (void)hipGraphExecDestroy(g.exec);
        graphs.clear();
    }

    ~crsolve_plan()
    {
        drop_graphs();
        if (cap_stream)
            (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : evpool)
            (void)hipEventDestroy(e);
    }
};

namespace {

const crsolve_plan* tplan(const crsolve_plan* p) { return p->timing_parent ? p->timing_parent : p; }

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
    Timed(const crsolve_plan* pp, int kid, hipStream_t s, int cls = 0, int f64 = 0)
        : p(tplan(pp)), st(s)
    {
        if (!p->timing)
            return;
        hipEvent_t a = pool_event(p);
        b = pool_event(p);
        if (!a || !b) {
            b = nullptr;
            return;
        }
        p->reckid.push_back(kid | (cls << 8) | (f64 << 12));
        (void)hipEventRecord(a, st);
    }
    ~Timed()
    {
        if (b)
            (void)hipEventRecord(b, st);
    }
};

unsigned grid_of(int64_t total) { return (unsigned)std::min<int64_t>(total, kMaxGrid); }

// Kernel dispatch per block-size class MT, element type T, level-input
// element EI (cx<double> for the FP32 levels that read FP64 inputs, rl<T> for
// the real dtypes' level 0) and real data (RE: the tiled kernels form one
// real MFMA per product step).
template <class T, class EI = cx<T>, bool RE = false>
struct Disp {
    template <int MT>
    static void elim(const Launch& L, const Seg* segs, const void* inA, const void* inB,
                     const void* iny, void* W, unsigned long long* flags, int mat, int rhs,
                     hipStream_t st, int variant, int nsplit)
    {
        if ((MT == 16 || MT == 32) && variant == 0) {
            hipLaunchKernelGGL((crs::k_elim_mf<T, (MT == 16 || MT == 32) ? MT : 16, EI>),
                               dim3((unsigned)(L.total * nsplit)), dim3(64), 0, st,
                               segs + L.seg0, L.nseg, L.total, nsplit, (const EI*)inA,
                               (const EI*)inB, (const EI*)iny, (cx<T>*)W, flags, mat, rhs);
        } else if (MT <= 32 && variant == 0) {
            hipLaunchKernelGGL((crs::k_elim_w<T, MT <= 32 ? MT : 32, EI>), dim3((unsigned)L.total), dim3(64), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const EI*)inA,
                               (const EI*)inB, (const EI*)iny, (cx<T>*)W, flags, mat, rhs);
        } else if constexpr (MT <= 32) { // blocks above 32 run the tiled kernels
            constexpr int PW = sizeof(T) == 8 ? 32 : 64;
            hipLaunchKernelGGL((crs::k_elim<T, MT, kNT, PW, EI>), dim3(grid_of(L.total)), dim3(kNT), 0,
                               st, segs + L.seg0, L.nseg, L.total, (const EI*)inA,
                               (const EI*)inB, (const EI*)iny, (cx<T>*)W, flags, mat, rhs);
        }
    }
    template <int MT>
    static void reduce(const Launch& L, const Seg* segs, const void* inA, const void* iny, void* W,
                       const unsigned long long* flags, int mat, int rhs, hipStream_t st,
                       int variant)
    {
        if ((MT == 16 || MT == 32) && variant == 0) {
            hipLaunchKernelGGL((crs::k_reduce_m<T, (MT == 16 || MT == 32) ? MT : 16, EI>), dim3((unsigned)L.total), dim3(64), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const EI*)inA,
                               (const EI*)iny, (cx<T>*)W, flags, mat, rhs);
        } else if (MT == 64) {
            hipLaunchKernelGGL((crs::k_reduce_t<T, 64, EI>), dim3((unsigned)L.total), dim3(64), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const EI*)inA,
                               (const EI*)iny, (cx<T>*)W, flags, mat, rhs);
        } else {
            hipLaunchKernelGGL((crs::k_reduce<T, MT, kNT, EI>), dim3(grid_of(L.total)), dim3(kNT), 0,
                               st, segs + L.seg0, L.nseg, L.total, (const EI*)inA,
                               (const EI*)iny, (cx<T>*)W, flags, mat, rhs);
        }
    }
    template <int MT>
    static void back(const Launch& L, const Seg* segs, const void* W, void* X,
                     const unsigned long long* flags, hipStream_t st, int variant, void* U,
                     int upd)
    {
        if ((MT == 16 || MT == 32) && variant == 0) {
            hipLaunchKernelGGL((crs::k_back_mf<T, (MT == 16 || MT == 32) ? MT : 16>), dim3((unsigned)L.total), dim3(64), 0, st,
                               segs + L.seg0, L.nseg, L.total, (const cx<T>*)W, (cx<T>*)X, flags,
                               (cx<double>*)U, upd);
        } else if constexpr (MT <= 32) { // blocks above 32 run the tiled kernels
            constexpr int PW = 32;
            hipLaunchKernelGGL((crs::k_back<T, MT, kNT, PW>), dim3(grid_of(L.total)), dim3(kNT), 0,
                               st, segs + L.seg0, L.nseg, L.total, (const cx<T>*)W, (cx<T>*)X,
                               flags, (cx<double>*)U, upd);
        }
    }
    template <int MT>
    static void grad(const Launch& L, const Seg* segs, const void* X, const void* Lam, void* gA,
                     void* gB, hipStream_t st)
    {
        if constexpr (MT <= 32) // blocks above 32 run k_grad_big
            hipLaunchKernelGGL((crs::k_grad<T, MT, kNT>), dim3(grid_of(L.total)), dim3(kNT), 0, st,
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
    const CvtJob* djobs;
    unsigned long long* flags;
    hipStream_t st;
};

Ctx make_ctx(const crsolve_plan* p, void* ws, void* stream)
{
    Ctx c;
    c.p = p;
    c.ws = (char*)ws;
    c.dsegs = (const Seg*)(c.ws + p->off_segs);
    c.djobs = (const CvtJob*)(c.ws + p->off_jobs);
    c.flags = (unsigned long long*)(c.ws + p->off_flags);
    c.st = (hipStream_t)stream;
    return c;
}

// Largest per-block extents over the segments of a launch of the tiled
// kernels: 16-row tiles S, 16-column strips of the right-hand side K16, and
// the 32-wide counts T32, K32 of the reduced-system tiles.
struct BigDims {
    int S = 0, K16 = 0, T32 = 0, K32 = 0;
};
BigDims big_dims(const crsolve_plan* p, const Launch& L)
{
    BigDims b;
    for (int i = L.seg0; i < L.seg0 + L.nseg; ++i) {
        const Seg& g = p->segs[i];
        b.S = std::max(b.S, (g.m + 15) / 16);
        b.K16 = std::max(b.K16, (g.k + 15) / 16);
        b.T32 = std::max(b.T32, (g.m + 31) / 32);
        b.K32 = std::max(b.K32, (g.k + 31) / 32);
    }
    return b;
}

// FP64 tiled forward substitutions of launches with at least this many blocks
// run one wave per strip (k_trsm_strip); fewer blocks, or FP32, take the
// work-group form with its shorter chain and shared L tiles.
constexpr int64_t kTrsmStripBlocks = 256;

// Tiled Cholesky launches of at most this many blocks (one per CU) run
// work-groups of eight waves.
constexpr int64_t kPotrfWideBlocks = 256;

// Grid of the tiled kernels: a multiple of 8 work-groups (see xcd_item).
unsigned grid8(int64_t items) { return (unsigned)((items + 7) / 8 * 8); }

// Levels of the one-wave MFMA classes (8 < m <= 32) with few blocks are bound
// by one block's chain of dependent steps, not by throughput.  There the
// elimination splits each block's strips over up to tail_waves / blocks
// waves, and launches of at most tail_blocks blocks form the reduced system
// one wave per 16 x 16 output tile.  Defaults 2048 and 1024 (measured on the
// N = 65536, m = 32 workload; 2048 is about the wave slots of the GPU's 1024
// SIMDs); the autotuner picks both per plan.

bool mf_class(int cls) { return cls == 2 || cls == 3; }

template <class T, class EI, bool RE>
void run_elim(const Ctx& c, const Launch& L, const void* A, const void* B, const void* y, int mat,
              int rhs)
{
    const void* inA = L.userAB ? A : c.ws;
    const void* inB = L.userAB ? B : c.ws;
    const void* iny = L.userY ? y : c.ws;
    if (tiled(L.cls)) {
        const BigDims b = big_dims(c.p, L);
        if (mat) {
            Timed tm(c.p, KID_POTRF, c.st, L.cls, L.f64);
            // levels with at most one block per CU spread the panel tiles over
            // eight waves instead of four
            const unsigned nthr = L.total <= kPotrfWideBlocks ? 512 : 256;
            if (L.total <= kPotrfWideBlocks)
                // few blocks (every tiled class): one block's chain of panels
                // sets the time, so the diagonal steps run ahead of the
                // trailing updates
                hipLaunchKernelGGL((crs::k_potrf_rl<T, EI, RE>), dim3((unsigned)L.total), dim3(512), 0,
                                   c.st, c.dsegs + L.seg0, L.nseg, L.total, (const EI*)inA,
                                   (cx<T>*)c.ws, c.flags);
            else if (L.cls == kBig)
                hipLaunchKernelGGL((crs::k_potrf_big<T, false, EI, RE>), dim3((unsigned)L.total), dim3(nthr), 0,
                                   c.st, c.dsegs + L.seg0, L.nseg, L.total, (const EI*)inA,
                                   (cx<T>*)c.ws, c.flags);
            else
                hipLaunchKernelGGL((crs::k_potrf_big<T, true, EI, RE>), dim3((unsigned)L.total), dim3(nthr), 0,
                                   c.st, c.dsegs + L.seg0, L.nseg, L.total, (const EI*)inA,
                                   (cx<T>*)c.ws, c.flags);
        }
        const int ns = (mat ? 2 * b.S : 0) + (rhs ? b.K16 : 0);
        if (ns > 0) {
            constexpr int NC = crs::trsm_strips<T>();
            const int ngrp = (ns + NC - 1) / NC;
            Timed tm(c.p, KID_TRSM, c.st, L.cls, L.f64);
            if (sizeof(T) == 8 && L.total >= kTrsmStripBlocks && L.cls == kBig)
                // the real form's single-MFMA steps take the deeper prefetch
                // (Poisson real form k_trsm 13.5 -> 13.2 ms; the complex form
                // measured slower with it, 14.0 -> 14.7 ms)
                hipLaunchKernelGGL((crs::k_trsm_strip<T, EI, RE, 1, RE ? 8 : 0>), dim3(grid8(L.total * ns)),
                                   dim3(64), 0, c.st, c.dsegs + L.seg0, L.nseg, L.total, ns, mat, rhs,
                                   (const EI*)inB, (const EI*)iny, (cx<T>*)c.ws, c.flags);
            else if (sizeof(T) == 8 && L.cls == kBig)
                // few blocks: every strip's chain of loads in flight eight
                // contraction steps deep
                hipLaunchKernelGGL((crs::k_trsm_strip<T, EI, RE, 1, 8>), dim3(grid8(L.total * ns)), dim3(64), 0,
                                   c.st, c.dsegs + L.seg0, L.nseg, L.total, ns, mat, rhs,
                                   (const EI*)inB, (const EI*)iny, (cx<T>*)c.ws, c.flags);
            else if (sizeof(T) == 8 && L.total >= kTrsmStripBlocks) {
                // blocks of 33..64: two strips per wave, ceil(S / 2) items per
                // B and ceil(K16 / 2) of y
                const int ni = (mat ? 2 * ((b.S + 1) / 2) : 0) + (rhs ? (b.K16 + 1) / 2 : 0);
                hipLaunchKernelGGL((crs::k_trsm_strip<T, EI, RE, 2>), dim3(grid8(L.total * ni)), dim3(64), 0,
                                   c.st, c.dsegs + L.seg0, L.nseg, L.total, ni, mat, rhs,
                                   (const EI*)inB, (const EI*)iny, (cx<T>*)c.ws, c.flags);
            }
            else
                hipLaunchKernelGGL((crs::k_trsm_big<T, EI, RE>), dim3(grid8(L.total * ngrp)), dim3(64 * b.S),
                                   0, c.st, c.dsegs + L.seg0, L.nseg, L.total, ngrp, mat, rhs,
                                   (const EI*)inB, (const EI*)iny, (cx<T>*)c.ws, c.flags);
        }
        return;
    }
    Timed tm(c.p, KID_ELIM, c.st, L.cls, L.f64);
    const int v = c.p->var[0][L.cls][L.f64];
    int nsplit = 1;
    if (mf_class(L.cls) && v == 0) {
        const BigDims b = big_dims(c.p, L);
        const int nst = (mat ? 2 * b.S : 0) + (rhs ? b.K16 : 0);
        nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(nst, c.p->tail_waves / L.total));
    }
#define CALL(MT) Disp<T, EI, RE>::template elim<MT>(L, c.dsegs, inA, inB, iny, c.ws, c.flags, mat, rhs, c.st, v, nsplit)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

template <class T, class EI, bool RE>
void run_reduce(const Ctx& c, const Launch& L, const void* A, const void* y, int mat, int rhs)
{
    const void* inA = L.userAB ? A : c.ws;
    const void* iny = L.userY ? y : c.ws;
    Timed tm(c.p, KID_REDUCE, c.st, L.cls, L.f64);
    const int v = c.p->var[1][L.cls][L.f64];
    if (L.cls == kBig || (tiled(L.cls) && v == 0)) {
        const BigDims b = big_dims(c.p, L);
        // blocks above 64: A' and B' from LDS-staged 64 x 64 tiles, y' in
        // 32 x 32 tiles (for m <= 64 the per-wave tiles are faster: the
        // LDS form would run one or two work-groups per block)
        const bool staged = mat && L.cls == kBig;
        if (staged) {
            const int T64 = (b.S + 3) / 4, nm = T64 * (T64 + 1) / 2 + T64 * T64;
            hipLaunchKernelGGL((crs::k_reduce_lds<T, EI, RE>), dim3(grid8(L.total * nm)), dim3(256), 0, c.st,
                               c.dsegs + L.seg0, L.nseg, L.total, nm, (const EI*)inA,
                               (cx<T>*)c.ws, c.flags);
        }
        const int mt = mat && !staged ? 1 : 0;
        if (mt) {
            // 32 < m <= 64: one wave per 16 x 16 tile (four times the waves of
            // the 32 x 32 tiles for these short contractions)
            const int nt = b.S * (b.S + 1) / 2 + b.S * b.S + (rhs ? b.S * b.K16 : 0);
            hipLaunchKernelGGL((crs::k_reduce_big<T, 1, EI, RE>), dim3(grid8(L.total * nt)), dim3(64), 0, c.st,
                               c.dsegs + L.seg0, L.nseg, L.total, nt, 1, rhs, (const EI*)inA,
                               (const EI*)iny, (cx<T>*)c.ws, c.flags);
            return;
        }
        if (!mt && rhs && b.K16 == 1) {
            // y' alone with at most 16 columns: 16 x 16 tiles waste half as
            // many MFMA columns as 32 x 32 ones
            const int nt = b.S;
            hipLaunchKernelGGL((crs::k_reduce_big<T, 1, EI, RE>), dim3(grid8(L.total * nt)), dim3(64), 0, c.st,
                               c.dsegs + L.seg0, L.nseg, L.total, nt, 0, rhs, (const EI*)inA,
                               (const EI*)iny, (cx<T>*)c.ws, c.flags);
            return;
        }
        const int nt = (mt ? b.T32 * (b.T32 + 1) / 2 + b.T32 * b.T32 : 0) + (rhs ? b.T32 * b.K32 : 0);
        if (nt > 0)
            hipLaunchKernelGGL((crs::k_reduce_big<T, 2, EI, RE>), dim3(grid8(L.total * nt)), dim3(64), 0, c.st,
                               c.dsegs + L.seg0, L.nseg, L.total, nt, mt, rhs, (const EI*)inA,
                               (const EI*)iny, (cx<T>*)c.ws, c.flags);
        return;
    }
    if (mf_class(L.cls) && L.total <= c.p->tail_blocks) {
        const BigDims b = big_dims(c.p, L);
        const int nt = (mat ? b.S * (b.S + 1) / 2 + b.S * b.S : 0) + (rhs ? b.S * b.K16 : 0);
        if (nt > 0)
            hipLaunchKernelGGL((crs::k_reduce_big<T, 1, EI, RE>), dim3(grid8(L.total * nt)), dim3(64), 0, c.st,
                               c.dsegs + L.seg0, L.nseg, L.total, nt, mat, rhs, (const EI*)inA,
                               (const EI*)iny, (cx<T>*)c.ws, c.flags);
        return;
    }
#define CALL(MT) Disp<T, EI, RE>::template reduce<MT>(L, c.dsegs, inA, iny, c.ws, c.flags, mat, rhs, c.st, v)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

// upd (mixed form): 0 plain back substitution; 1 / 2 the level-0 launches
// assign / add their corrections to the caller's FP64 x.
template <class T, bool RE>
void run_back(const Ctx& c, const Launch& L, void* x, int upd)
{
    void* X = L.userX ? x : c.ws;
    const int u = L.upd ? upd : 0;
    Timed tm(c.p, KID_BACK, c.st, L.cls, L.f64);
    if (tiled(L.cls)) {
        const BigDims b = big_dims(c.p, L);
        hipLaunchKernelGGL((crs::k_back_big<T, RE>), dim3(grid8(L.total * b.K16)), dim3(64 * b.S), 0, c.st,
                           c.dsegs + L.seg0, L.nseg, L.total, b.K16, (const cx<T>*)c.ws, (cx<T>*)X,
                           c.flags, (cx<double>*)x, u);
        return;
    }
    const int v = c.p->var[2][L.cls][L.f64];
#define CALL(MT) Disp<T>::template back<MT>(L, c.dsegs, c.ws, X, c.flags, c.st, v, x, u)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

template <class T>
void run_grad(const Ctx& c, const Launch& L, const void* x, const void* lam, void* gA, void* gB)
{
    Timed tm(c.p, KID_GRAD, c.st);
    if (tiled(L.cls)) {
        const BigDims b = big_dims(c.p, L);
        hipLaunchKernelGGL((crs::k_grad_big<T>), dim3(grid8(L.total * b.T32 * b.T32)), dim3(64), 0,
                           c.st, c.dsegs + L.seg0, L.nseg, L.total, b.T32 * b.T32, (const cx<T>*)x,
                           (const cx<T>*)lam, (cx<T>*)gA, (cx<T>*)gB);
        return;
    }
#define CALL(MT) Disp<T>::template grad<MT>(L, c.dsegs, x, lam, gA, gB, c.st)
    CRS_BY_CLASS(L.cls, CALL)
#undef CALL
}

void run_cvt(const Ctx& c, const CvtLaunch& L, const void* A, const void* B, const void* y)
{
    const void* src = L.user_src ? (L.which == 0 ? A : (L.which == 1 ? B : y)) : c.ws;
    Timed tm(c.p, KID_CONVERT, c.st);
    const int64_t per = 256 * crs::kCvtPer;
    const unsigned g = (unsigned)std::min<int64_t>((L.total + per - 1) / per, 1 << 16);
    const CvtJob* jb = c.djobs + L.job0;
    if (L.f64_src && !L.f64_dst)
        hipLaunchKernelGGL((crs::k_convert<double, float>), dim3(g), dim3(256), 0, c.st, jb,
                           L.njobs, L.total, (const cx<double>*)src, (cx<float>*)c.ws);
    else if (!L.f64_src && L.f64_dst)
        hipLaunchKernelGGL((crs::k_convert<float, double>), dim3(g), dim3(256), 0, c.st, jb,
                           L.njobs, L.total, (const cx<float>*)src, (cx<double>*)c.ws);
    else if (L.f64_src)
        hipLaunchKernelGGL((crs::k_convert<double, double>), dim3(g), dim3(256), 0, c.st, jb,
                           L.njobs, L.total, (const cx<double>*)src, (cx<double>*)c.ws);
    else
        hipLaunchKernelGGL((crs::k_convert<float, float>), dim3(g), dim3(256), 0, c.st, jb,
                           L.njobs, L.total, (const cx<float>*)src, (cx<float>*)c.ws);
}

__global__ void k_finalize(const unsigned long long* flags, crsolve_info* info, int n, int fb)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        unsigned long long f = flags[i];
        crsolve_info v;
        v.status = f != crs::kNoFail;
        v.level = v.status ? (int32_t)(f >> 40) : -1;
        v.block = v.status ? (int64_t)(f & ((1ull << 40) - 1)) : -1;
        v.refine_iters = 0;
        v.fp64_fallback = fb;
        v.rel_residual = 0.0;
        info[i] = v;
    }
}

// Real dtypes: x[e] = Re xc[e] over the unknowns of every system.
template <class T>
__global__ void k_real_out(const cx<T>* __restrict__ xc, T* __restrict__ x, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
        x[e] = xc[e].r;
}

// info[i].refine_iters / rel_residual from a host-filled table {iters, rel}.
__global__ void k_set_refine(const double* tab, crsolve_info* info, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        info[i].refine_iters = (int32_t)tab[2 * i];
        info[i].rel_residual = tab[2 * i + 1];
    }
}

// ------------------------------------------------------------------ plan build

struct WsAlloc {
    size_t off = 0;
    int64_t take(int64_t elems, size_t esz)
    {
        int64_t o = (int64_t)(off / esz);
        off = align_up(off + (size_t)elems * esz);
        return o;
    }
};

// Appends launches: for each level, one launch per (class, precision) with
// work; `count(s, l)` gives the work items of system s at level l.
template <class Count>
void add_launches(crsolve_plan* p, std::vector<Launch>& out, int nlev, Count count)
{
    for (int lvl = 0; lvl < nlev; ++lvl)
        for (int f = 0; f < 2; ++f)
            for (int c = 0; c < kNumCls; ++c) {
                Launch L{lvl, c, f, (int)p->segs.size(), 0, 0, false, false, false, false, false, false};
                for (int s = 0; s < p->batch; ++s) {
                    if (p->cls[s] != c || lvl >= (int)p->lv[s].size())
                        continue;
                    const LevelSpec& v = p->lv[s][lvl];
                    if (v.f64 != f)
                        continue;
                    int64_t cnt = count(s, lvl);
                    if (cnt <= 0)
                        continue;
                    Seg g;
                    std::memset(&g, 0, sizeof(g));
                    g.n = v.n;
                    g.m = p->m[s];
                    g.k = p->k[s];
                    g.level = lvl;
                    g.sys = s;
                    g.oL = v.oL; g.oP = v.oP; g.oQ = v.oQ; g.og = v.og;
                    g.oAo = v.oAo; g.oBo = v.oBo; g.oyo = v.oyo;
                    g.oA = v.oA; g.oB = v.oB; g.oy = v.oy;
                    g.ox = v.ox; g.xo = v.xo; g.xs = v.xs;
                    g.oD = v.oD;
                    g.oU = v.oU;
                    if (!v.pcr) {
                        g.d = 1;
                        g.e0 = 0; g.es = 2; g.ne = v.ne;
                        g.k0 = 1; g.ks = 2; g.nk = v.nk;
                        g.out_by_pos = 0;
                        g.ob0 = 1ll << lvl;
                        g.obs = 1ll << lvl;
                    } else {
                        g.d = v.d;
                        g.e0 = 0; g.es = 1; g.ne = v.ne;
                        g.k0 = 0; g.ks = 1; g.nk = v.nk;
                        g.out_by_pos = 1;
                        g.ob0 = v.obs;
                        g.obs = v.obs;
                    }
                    g.w0 = L.total;
                    L.total += cnt;
                    L.userAB = v.userAB;
                    L.userY = v.userY;
                    L.userX = v.userX;
                    L.in64 = v.in64;
                    L.upd = v.upd;
                    L.inreal = v.inreal;
                    p->segs.push_back(g);
                    ++L.nseg;
                }
                if (L.nseg)
                    out.push_back(L);
                else
                    p->segs.resize(L.seg0);
            }
}

// Conversion launches from a list of (src, dst, count) ranges.
struct JobIn {
    int64_t src, dst, count;
};
void add_cvt(crsolve_plan* p, std::vector<CvtLaunch>& out, const std::vector<JobIn>& in,
             int f64_src, int f64_dst, bool user_src, int which)
{
    if (in.empty())
        return;
    CvtLaunch L{f64_src, f64_dst, user_src, which, (int)p->jobs.size(), 0, 0};
    for (const JobIn& j : in) {
        if (j.count <= 0)
            continue;
        p->jobs.push_back(CvtJob{L.total, j.src, j.dst, j.count});
        L.total += j.count;
        ++L.njobs;
    }
    if (L.njobs)
        out.push_back(L);
    else
        p->jobs.resize(L.job0);
}

int build_plan(crsolve_plan* p)
{
    const bool refine = p->prec == CRSOLVE_PREC_FP32_REFINE;
    const bool f64native = p->dtype == CRSOLVE_C128 || p->dtype == CRSOLVE_R64;
    WsAlloc a;
    p->off_flags = a.off;
    a.off = align_up(a.off + sizeof(unsigned long long) * p->batch);
    p->lv.assign(p->batch, {});
    p->sw.assign(p->batch, -1);
    const size_t e32 = sizeof(cx<float>), e64 = sizeof(cx<double>);

    // residual norm partials and totals (FP64 inputs); for refinement also
    // the correction d (complex FP32, laid out like y), the residual r
    // (complex FP64, laid out like y), the info table and the fallback bits
    std::vector<int64_t> oxt(p->batch, 0);
    const bool io64 = refine || p->dtype == CRSOLVE_C128;
    if (io64) {
        p->off_part = a.off;
        // one pair of partial sums per residual work item
        int64_t nparts = 0;
        for (int s = 0; s < p->batch; ++s)
            nparts += (int64_t)p->N[s] * crs::resid_items(p->m[s], p->k[s]);
        a.off = align_up(a.off + sizeof(double) * 2 * (size_t)std::max<int64_t>(nparts, 1));
        p->off_norms = a.off;
        a.off = align_up(a.off + sizeof(double) * 2 * p->batch);
    }
    if (refine) {
        p->off_d32 = a.off;
        a.off = align_up(a.off + (size_t)p->toty * e32);
        p->off_r64 = a.off;
        a.off = align_up(a.off + (size_t)p->toty * e64);
        p->off_info = a.off;
        a.off = align_up(a.off + sizeof(double) * 2 * p->batch);
        p->off_fbits = a.off;
        a.off = align_up(a.off + sizeof(int32_t) * p->batch);
    }
    if (p->real) {
        // the unknowns in the complex layout of the levels; their real parts
        // go to the caller's real x at the end of every solve
        p->off_xc = a.off;
        a.off = align_up(a.off + (size_t)p->toty * (f64native ? e64 : e32));
    }

    int maxlev = 0;
    for (int s = 0; s < p->batch; ++s) {
        const int64_t mm = (int64_t)p->m[s] * p->m[s], mk = (int64_t)p->m[s] * p->k[s];
        const int64_t dtiles = (int64_t)((p->m[s] + 15) / 16) * 256; // inverse diagonal tiles
        std::vector<LevelSpec>& L = p->lv[s];
        if (p->sched == CRSOLVE_SCHED_CR) {
            // one-sided levels until the block count falls to hyb (if set)
            int v = p->N[s];
            for (; v > 0 && !(p->hyb > 0 && v <= p->hyb); v /= 2) {
                LevelSpec ls;
                ls.n = v;
                ls.ne = (v + 1) / 2;
                ls.nk = v / 2;
                ls.f64 = refine ? (v <= p->tail ? 1 : 0) : (f64native ? 1 : 0);
                L.push_back(ls);
            }
            const int ncr = (int)L.size(), nt = v; // Algorithm 1 tail of nt blocks
            int sw = -1;
            if (refine)
                for (size_t l = 0; l < L.size(); ++l)
                    if (L[l].f64) {
                        sw = (int)l;
                        break;
                    }
            p->sw[s] = sw;
            // factor storage and reduced systems, per level in its precision
            for (size_t l = 0; l < (size_t)ncr; ++l) {
                LevelSpec& v = L[l];
                const size_t es = v.f64 ? e64 : e32;
                v.oL = a.take(v.ne * mm, es);
                v.oP = a.take(v.ne * mm, es);
                v.oQ = a.take(v.ne * mm, es);
                v.oAo = a.take(v.nk * mm, es);
                v.oBo = a.take(std::max(v.nk - 1, 0) * mm, es);
                if (tiled(p->cls[s]))
                    v.oD = a.take(v.ne * dtiles, es);
            }
            for (size_t l = 0; l < (size_t)ncr; ++l) {
                LevelSpec& v = L[l];
                const size_t es = v.f64 ? e64 : e32;
                v.og = a.take(v.ne * mk, es);
                v.oyo = a.take(v.nk * mk, es);
            }
            if (nt > 0) {
                // Algorithm 1 in place on the nt blocks of level ncr: every
                // level keeps its own factors (so that a factorization can be
                // solved again), the reduced systems alternate between two
                // buffers
                const size_t es = f64native ? e64 : e32;
                const int D = pcr_depth(nt);
                int64_t bA[2], bB[2], by[2];
                for (int b = 0; b < 2; ++b) {
                    bA[b] = a.take((int64_t)nt * mm, es);
                    bB[b] = a.take((int64_t)nt * mm, es);
                    by[b] = a.take((int64_t)nt * mk, es);
                }
                for (int i = 0; i <= D; ++i) {
                    LevelSpec ls;
                    ls.n = ls.ne = nt;
                    ls.nk = i < D ? nt : 0;
                    ls.f64 = f64native ? 1 : 0;
                    ls.pcr = true;
                    ls.d = (int)std::min<int64_t>(1ll << i, (int64_t)1 << 30);
                    ls.obs = 1ll << ncr;
                    ls.oL = a.take((int64_t)nt * mm, es);
                    ls.oP = a.take((int64_t)nt * mm, es);
                    ls.oQ = a.take((int64_t)nt * mm, es);
                    ls.og = a.take((int64_t)nt * mk, es);
                    if (tiled(p->cls[s]))
                        ls.oD = a.take((int64_t)nt * dtiles, es);
                    ls.oAo = bA[(i + 1) & 1];
                    ls.oBo = bB[(i + 1) & 1];
                    ls.oyo = by[(i + 1) & 1];
                    L.push_back(ls);
                }
            }
            // level inputs: level 0 reads the caller's arrays (the mixed
            // form's right-hand side is y in the first pass and the FP64
            // residual, laid out like y, in the corrections; its FP32 level 0
            // rounds the FP64 inputs on load)
            for (size_t l = 0; l < L.size(); ++l) {
                LevelSpec& v = L[l];
                v.in64 = v.f64 || (refine && l == 0);
                v.inreal = p->real && l == 0;
                if (l == 0) {
                    v.userAB = v.userY = true;
                    v.oA = p->offA[s];
                    v.oB = p->offB[s];
                    v.oy = p->offy[s];
                } else if (v.pcr && (int)l > ncr) {
                    // later levels of the Algorithm 1 tail: the other buffer
                    v.oA = L[l - 1].oAo;
                    v.oB = L[l - 1].oBo;
                    v.oy = L[l - 1].oyo;
                } else if ((int)l == sw) {
                    // first FP64 level: its inputs are FP64 copies of the
                    // previous (FP32) level's reduced system
                    v.oA = a.take(v.n * mm, e64);
                    v.oB = a.take(std::max(v.n - 1, 0) * mm, e64);
                    v.oy = a.take(v.n * mk, e64);
                } else {
                    v.oA = L[l - 1].oAo;
                    v.oB = L[l - 1].oBo;
                    v.oy = L[l - 1].oyo;
                }
            }
            // unknowns
            if (refine && sw >= 0)
                oxt[s] = a.take((int64_t)L[sw].n * mk, e64);
            for (size_t l = 0; l < L.size(); ++l) {
                LevelSpec& v = L[l];
                if (refine && l == 0) {
                    // the corrections of level 0 go straight into the FP64 x
                    v.upd = true;
                    v.oU = p->offy[s];
                }
                if (!refine) {
                    // level l position p is block (p + 1) 2^l of x; the
                    // Algorithm 1 tail keeps the numbering of its first level
                    const int lx = v.pcr ? ncr : (int)l;
                    v.userX = !p->real;
                    v.ox = p->real ? (int64_t)(p->off_xc / (f64native ? e64 : e32)) + p->offy[s]
                                   : p->offy[s];
                    v.xo = (1ll << lx) - 1;
                    v.xs = 1ll << lx;
                } else if (sw < 0 || (int)l < sw) {
                    v.ox = (int64_t)(p->off_d32 / e32) + p->offy[s];
                    v.xo = (1ll << l) - 1;
                    v.xs = 1ll << l;
                } else {
                    v.ox = oxt[s];
                    v.xo = (1ll << (l - sw)) - 1;
                    v.xs = 1ll << (l - sw);
                }
            }
        } else {
            const int N = p->N[s], D = pcr_depth(N);
            const size_t es = e64;
            int64_t oL = a.take(N * mm, es), oP = a.take(N * mm, es), oQ = a.take(N * mm, es),
                    og = a.take(N * mk, es);
            const int64_t oD = tiled(p->cls[s]) ? a.take(N * dtiles, es) : 0;
            int64_t bA[2], bB[2], by[2];
            for (int b = 0; b < 2; ++b) {
                bA[b] = a.take(N * mm, es);
                bB[b] = a.take(N * mm, es);
                by[b] = a.take(N * mk, es);
            }
            for (int l = 0; l <= D; ++l) {
                LevelSpec v;
                v.n = N;
                v.ne = N;
                v.nk = l < D ? N : 0;
                v.f64 = 1;
                v.oL = oL; v.oP = oP; v.oQ = oQ; v.og = og; v.oD = oD;
                v.oAo = bA[(l + 1) & 1]; v.oBo = bB[(l + 1) & 1]; v.oyo = by[(l + 1) & 1];
                if (l == 0) {
                    v.userAB = v.userY = true;
                    v.oA = p->offA[s]; v.oB = p->offB[s]; v.oy = p->offy[s];
                } else {
                    v.oA = bA[l & 1]; v.oB = bB[l & 1]; v.oy = by[l & 1];
                }
                v.userX = true;
                v.ox = p->offy[s];
                v.xo = 0;
                v.xs = 1;
                v.pcr = true;
                v.d = (int)std::min<int64_t>(1ll << l, (int64_t)1 << 30);
                v.obs = 1;
                L.push_back(v);
            }
        }
        maxlev = std::max(maxlev, (int)L.size());
    }
    p->nlevels = maxlev;

    p->segs.clear();
    p->jobs.clear();
    p->elim.clear(); p->reduce.clear(); p->back.clear(); p->grad.clear(); p->resid.clear();
    add_launches(p, p->elim, maxlev, [&](int s, int l) -> int64_t { return p->lv[s][l].ne; });
    add_launches(p, p->reduce, maxlev, [&](int s, int l) -> int64_t { return p->lv[s][l].nk; });
    // Recovery of the unknowns: the one-sided schedule back-substitutes at
    // every level; Algorithm 1 only solves the uncoupled blocks of its last
    // level (reassembly is the identity on the in-place layout).
    add_launches(p, p->back, maxlev, [&](int s, int l) -> int64_t {
        if (p->lv[s][l].pcr && l + 1 != (int)p->lv[s].size())
            return 0;
        return p->lv[s][l].ne;
    });

    // whole-system segments: gradients or residuals (one work item per block
    // row) and norms (one per system)
    // first residual partial-sum pair of each system: one pair per (block
    // row, 16-row tile)
    std::vector<int64_t> rowbase(p->batch, 0);
    for (int s = 1; s < p->batch; ++s)
        rowbase[s] = rowbase[s - 1] + (int64_t)p->N[s - 1] * crs::resid_items(p->m[s - 1], p->k[s - 1]);
    auto sys_seg = [&](int s) {
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
        g.ob0 = rowbase[s];
        return g;
    };
    for (int kind = 0; kind < 2; ++kind)
        for (int f = 0; f < 2; ++f)
            for (int c = 0; c < kNumCls; ++c) {
                // kind 0, gradients: one launch per class in the plan's dtype;
                // kind 1, residuals (FP64 inputs): one launch per class and
                // level-0 precision
                if (kind == 0 && refine)
                    continue;
                if (kind == 1 && !io64)
                    continue;
                Launch L{0, c, f, (int)p->segs.size(), 0, 0, false, false, false, false, false, false};
                for (int s = 0; s < p->batch; ++s) {
                    if (p->cls[s] != c || (f == 1) != (p->lv[s][0].f64 == 1))
                        continue;
                    Seg g = sys_seg(s);
                    if (refine) // r lands in the FP64 residual buffer, laid out like y
                        g.og = (int64_t)(p->off_r64 / e64) + p->offy[s];
                    g.w0 = L.total;
                    // gradients: one work item per block row; residuals:
                    // resid_items per block row
                    L.total += kind == 0 ? (int64_t)p->N[s]
                                         : (int64_t)p->N[s] * crs::resid_items(p->m[s], p->k[s]);
                    p->segs.push_back(g);
                    ++L.nseg;
                }
                if (L.nseg)
                    (kind == 0 ? p->grad : p->resid).push_back(L);
                else
                    p->segs.resize(L.seg0);
            }
    p->norm_seg0 = (int)p->segs.size();
    for (int s = 0; s < p->batch; ++s)
        p->segs.push_back(sys_seg(s));

    // conversion jobs (refine)
    p->cvt_factor_sw.assign(maxlev + 1, {});
    p->cvt_solve_sw.assign(maxlev + 1, {});
    p->scatter_sw.assign(maxlev + 1, {});
    if (refine) {
        for (int l = 1; l <= maxlev; ++l) {
            std::vector<JobIn> fa, fbv, fy;
            for (int s = 0; s < p->batch; ++s) {
                if (p->sw[s] != l)
                    continue;
                const int64_t mm = (int64_t)p->m[s] * p->m[s], mk = (int64_t)p->m[s] * p->k[s];
                const LevelSpec &pv = p->lv[s][l - 1], &cv = p->lv[s][l];
                // source offsets count FP32 elements, destination offsets FP64
                // elements, both from the start of the workspace
                fa.push_back({pv.oAo, cv.oA, (int64_t)cv.n * mm});
                fbv.push_back({pv.oBo, cv.oB, (int64_t)std::max(cv.n - 1, 0) * mm});
                fy.push_back({pv.oyo, cv.oy, (int64_t)cv.n * mk});
            }
            add_cvt(p, p->cvt_factor_sw[l], fa, 0, 1, false, 0);
            add_cvt(p, p->cvt_factor_sw[l], fbv, 0, 1, false, 1);
            add_cvt(p, p->cvt_solve_sw[l], fy, 0, 1, false, 2);
        }
        // level 0 of a system that is FP64 throughout moves its corrections
        // into x itself (no scatter)
        for (int l = 1; l <= maxlev; ++l) {
            std::vector<JobIn> sc;
            for (int s = 0; s < p->batch; ++s) {
                if (p->sw[s] != l)
                    continue;
                const int64_t mk = (int64_t)p->m[s] * p->k[s];
                const int64_t d0 = (int64_t)(p->off_d32 / e32) + p->offy[s];
                for (int j = 0; j < p->lv[s][l].n; ++j)
                    sc.push_back({oxt[s] + j * mk, d0 + (((int64_t)(j + 1) << l) - 1) * mk, mk});
            }
            add_cvt(p, p->scatter_sw[l], sc, 1, 0, false, 2);
        }
    }

    p->off_segs = a.off;
    a.off = align_up(a.off + sizeof(Seg) * p->segs.size());
    p->off_jobs = a.off;
    a.off = align_up(a.off + sizeof(CvtJob) * std::max<size_t>(p->jobs.size(), 1));
    if (refine) {
        size_t big = 0;
        for (const auto& q : p->fbs)
            big = std::max(big, q->ws_bytes);
        p->off_fb = a.off;
        a.off = align_up(a.off + big);
    }
    p->ws_bytes = a.off;
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

bool any_B(const crsolve_plan* p) { return p->totB > 0; }

size_t io_esz(const crsolve_plan* p)
{
    if (p->dtype == CRSOLVE_R64)
        return 8;
    if (p->dtype == CRSOLVE_R32)
        return 4;
    return (p->dtype == CRSOLVE_C128 || p->prec == CRSOLVE_PREC_FP32_REFINE) ? 16 : 8;
}

int upload(const crsolve_plan* p, char* ws, hipStream_t st)
{
    if (hipMemcpyAsync(ws + p->off_segs, p->segs.data(), sizeof(Seg) * p->segs.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return CRSOLVE_EHIP;
    if (!p->jobs.empty() &&
        hipMemcpyAsync(ws + p->off_jobs, p->jobs.data(), sizeof(CvtJob) * p->jobs.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess)
        return CRSOLVE_EHIP;
    return CRSOLVE_OK;
}

int last_err() { return hipGetLastError() == hipSuccess ? CRSOLVE_OK : CRSOLVE_EHIP; }

// All levels downwards: matrix part (mat), right-hand side (rhs) or both.
void levels_down(const Ctx& c, const void* A, const void* B, const void* y, int mat, int rhs)
{
    const crsolve_plan* p = c.p;
    size_t ie = 0, ir = 0;
    for (int l = 0; l < p->nlevels; ++l) {
        for (; ie < p->elim.size() && p->elim[ie].level == l; ++ie) {
            const Launch& L = p->elim[ie];
            const bool re = p->real;
            if (L.f64 && L.inreal)
                run_elim<double, crs::rl<double>, true>(c, L, A, B, y, mat, rhs);
            else if (L.f64 && re)
                run_elim<double, cx<double>, true>(c, L, A, B, y, mat, rhs);
            else if (L.f64)
                run_elim<double, cx<double>, false>(c, L, A, B, y, mat, rhs);
            else if (L.inreal)
                run_elim<float, crs::rl<float>, true>(c, L, A, B, y, mat, rhs);
            else if (re)
                run_elim<float, cx<float>, true>(c, L, A, B, y, mat, rhs);
            else if (L.in64)
                run_elim<float, cx<double>, false>(c, L, A, B, y, mat, rhs);
            else
                run_elim<float, cx<float>, false>(c, L, A, B, y, mat, rhs);
        }
        for (; ir < p->reduce.size() && p->reduce[ir].level == l; ++ir) {
            const Launch& L = p->reduce[ir];
            const bool re = p->real;
            if (L.f64 && L.inreal)
                run_reduce<double, crs::rl<double>, true>(c, L, A, y, mat, rhs);
            else if (L.f64 && re)
                run_reduce<double, cx<double>, true>(c, L, A, y, mat, rhs);
            else if (L.f64)
                run_reduce<double, cx<double>, false>(c, L, A, y, mat, rhs);
            else if (L.inreal)
                run_reduce<float, crs::rl<float>, true>(c, L, A, y, mat, rhs);
            else if (re)
                run_reduce<float, cx<float>, true>(c, L, A, y, mat, rhs);
            else if (L.in64)
                run_reduce<float, cx<double>, false>(c, L, A, y, mat, rhs);
            else
                run_reduce<float, cx<float>, false>(c, L, A, y, mat, rhs);
        }
        if (l + 1 < (int)p->cvt_factor_sw.size()) {
            if (mat)
                for (const CvtLaunch& cl : p->cvt_factor_sw[l + 1])
                    run_cvt(c, cl, A, B, y);
            if (rhs)
                for (const CvtLaunch& cl : p->cvt_solve_sw[l + 1])
                    run_cvt(c, cl, A, B, y);
        }
    }
}

// All levels upwards.  Before the back substitution of level l (FP32), the
// unknowns of systems whose FP64 tail starts at level l + 1 move into the
// FP32 correction.  upd: see run_back.
void levels_up(const Ctx& c, void* x, int upd = 0)
{
    const crsolve_plan* p = c.p;
    const int nsc = (int)p->scatter_sw.size();
    int next = p->nlevels; // scatter lists of levels >= next are done
    for (size_t i = p->back.size(); i-- > 0;) {
        const Launch& L = p->back[i];
        for (; next > L.level + 1; --next)
            if (next - 1 < nsc && next - 1 > L.level)
                for (const CvtLaunch& cl : p->scatter_sw[next - 1])
                    run_cvt(c, cl, nullptr, nullptr, nullptr);
        if (L.f64)
            p->real ? run_back<double, true>(c, L, x, upd) : run_back<double, false>(c, L, x, upd);
        else
            p->real ? run_back<float, true>(c, L, x, upd) : run_back<float, false>(c, L, x, upd);
    }
    for (; next > 0; --next)
        if (next - 1 < nsc)
            for (const CvtLaunch& cl : p->scatter_sw[next - 1])
                run_cvt(c, cl, nullptr, nullptr, nullptr);
    if (p->real) {
        Timed tm(p, KID_REALOUT, c.st);
        const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((p->toty + 255) / 256, 1 << 16));
        if (p->dtype == CRSOLVE_R64)
            hipLaunchKernelGGL(k_real_out<double>, dim3(g), dim3(256), 0, c.st,
                               (const cx<double>*)(c.ws + p->off_xc), (double*)x, p->toty);
        else
            hipLaunchKernelGGL(k_real_out<float>, dim3(g), dim3(256), 0, c.st,
                               (const cx<float>*)(c.ws + p->off_xc), (float*)x, p->toty);
    }
}

void finalize(const Ctx& c, crsolve_info* info, int fb)
{
    if (!info)
        return;
    int n = c.p->batch;
    Timed tm(c.p, KID_FINAL, c.st);
    hipLaunchKernelGGL(k_finalize, dim3((n + 255) / 256), dim3(256), 0, c.st, c.flags, info, n, fb);
}

void init_flags(const Ctx& c)
{
    int n = c.p->batch;
    Timed tm(c.p, KID_FLAGS, c.st);
    hipLaunchKernelGGL(crs::k_flags_init, dim3((n + 255) / 256), dim3(256), 0, c.st, c.flags, n);
}

// --------------------------------------------------------------- mixed form

void residual(const Ctx& c, const void* A, const void* B, const void* x, const void* y,
              bool store_r)
{
    const crsolve_plan* p = c.p;
    double* part = (double*)(c.ws + p->off_part);
    cx<double>* R = store_r ? (cx<double>*)c.ws : nullptr;
    for (const Launch& L : p->resid) {
        Timed tm(p, KID_RESIDUAL, c.st);
        // row tiles per wave: one up to m = 16, then groups of two (four
        // would leave one wave per SIMD)
        const auto* Ad = (const cx<double>*)A;
        const auto* Bd = (const cx<double>*)B;
        const auto* Xd = (const cx<double>*)x;
        const auto* Yd = (const cx<double>*)y;
        if (L.cls <= 2)
            hipLaunchKernelGGL(crs::k_residual<1>, dim3(grid8(L.total)), dim3(64), 0, c.st,
                               c.dsegs + L.seg0, L.nseg, L.total, Ad, Bd, Xd, Yd, R, part);
        else
            hipLaunchKernelGGL(crs::k_residual<2>, dim3(grid8(L.total)), dim3(64), 0, c.st,
                               c.dsegs + L.seg0, L.nseg, L.total, Ad, Bd, Xd, Yd, R, part);
    }
    Timed tm(p, KID_NORMS, c.st);
    hipLaunchKernelGGL(crs::k_norms, dim3(p->batch), dim3(256), 0, c.st, c.dsegs + p->norm_seg0,
                       p->batch, (const double*)part, (double*)(c.ws + p->off_norms));
}

int read_norms(const Ctx& c, std::vector<double>& h)
{
    h.resize(2 * c.p->batch);
    if (hipMemcpyAsync(h.data(), c.ws + c.p->off_norms, sizeof(double) * h.size(),
                       hipMemcpyDeviceToHost, c.st) != hipSuccess)
        return CRSOLVE_EHIP;
    if (hipStreamSynchronize(c.st) != hipSuccess)
        return CRSOLVE_EHIP;
    return CRSOLVE_OK;
}

int write_refine_info(const Ctx& c, crsolve_info* info, const std::vector<double>& tab)
{
    if (!info)
        return CRSOLVE_OK;
    double* d = (double*)(c.ws + c.p->off_info);
    if (hipMemcpyAsync(d, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, c.st) !=
        hipSuccess)
        return CRSOLVE_EHIP;
    int n = c.p->batch;
    hipLaunchKernelGGL(k_set_refine, dim3((n + 255) / 256), dim3(256), 0, c.st, (const double*)d,
                       info, n);
    // the host table must outlive the copy
    if (hipStreamSynchronize(c.st) != hipSuccess)
        return CRSOLVE_EHIP;
    return CRSOLVE_OK;
}

// Records `enqueue` once per key into a HIP graph on the plan's capture
// stream (tables are uploaded first, outside the recording, so the graph
// holds kernel nodes only) and launches the graph on `st`.
template <class F>
int with_graph(const crsolve_plan* p, const std::vector<const void*>& key, char* ws,
               hipStream_t st, F enqueue)
{
    for (const crsolve_plan::GraphEntry& g : p->graphs)
        if (g.key == key)
            return hipGraphLaunch(g.exec, st) == hipSuccess ? CRSOLVE_OK : CRSOLVE_EHIP;
    int rc = upload(p, ws, st);
    if (rc)
        return rc;
    if (hipStreamSynchronize(st) != hipSuccess)
        return CRSOLVE_EHIP;
    if (!p->cap_stream && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return CRSOLVE_EHIP;
    const crsolve_plan* tp = tplan(p);
    const bool timing = tp->timing;
    tp->timing = false;
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        tp->timing = timing;
        return CRSOLVE_EHIP;
    }
    enqueue(make_ctx(p, ws, p->cap_stream));
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap_stream, &g);
    tp->timing = timing;
    if (ec != hipSuccess || !g)
        return CRSOLVE_EHIP;
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return CRSOLVE_EHIP;
    }
    (void)hipGraphDestroy(g);
    p->graphs.push_back({key, e});
    return hipGraphLaunch(e, st) == hipSuccess ? CRSOLVE_OK : CRSOLVE_EHIP;
}

std::vector<const void*> gkey(intptr_t kind, std::initializer_list<const void*> ptrs)
{
    std::vector<const void*> k{(const void*)kind};
    k.insert(k.end(), ptrs.begin(), ptrs.end());
    return k;
}

void enqueue_native_fs(const Ctx& c, const void* A, const void* B, const void* y, void* x,
                       crsolve_info* info)
{
    init_flags(c);
    levels_down(c, A, B, y, 1, 1);
    levels_up(c, x);
    finalize(c, info, 0);
}

void enqueue_refine_factor(const Ctx& c, const void* A, const void* B)
{
    init_flags(c);
    levels_down(c, A, B, nullptr, 1, 0);
}

// One solve pass of the mixed form: d = A^{-1} r with the mixed factors
// (first pass: r = y, read from the caller's y; later passes: the FP64
// residual), x = d or x += d inside the level-0 back substitution, then the
// FP64 residual and its norms.
void enqueue_refine_pass(const Ctx& c, const void* A, const void* B, const void* y, void* x,
                         bool first)
{
    levels_down(c, nullptr, nullptr, first ? y : (const void*)(c.ws + c.p->off_r64), 0, 1);
    levels_up(c, x, first ? 1 : 2);
    residual(c, A, B, x, y, true);
}

// The factorization fused with the first solve pass of the mixed form: all
// levels down with matrix and right-hand side together (level 0 reads the
// caller's FP64 A, B, y), back substitution with x = d at level 0, then the
// FP64 residual and its norms.
void enqueue_refine_fused(const Ctx& c, const void* A, const void* B, const void* y, void* x)
{
    init_flags(c);
    levels_down(c, A, B, y, 1, 1);
    levels_up(c, x, 1);
    residual(c, A, B, x, y, true);
}

// Relative residual of system s from the norm pairs read back by read_norms.
double rel_of(const std::vector<double>& nh, int s)
{
    return nh[2 * s + 1] > 0 ? std::sqrt(nh[2 * s] / nh[2 * s + 1]) : 0.0;
}

// Refinement after a first pass whose residual norms are in the workspace:
// d = A^{-1} r with the mixed factors and x += d while some active system
// misses rtol.  A system leaves the loop for the FP64 fallback (fb[s] = 1)
// when its residual fails to decrease from one pass to the next (stalled,
// diverging or NaN) or when it still misses rtol after max_refine passes.
// tab receives {corrections applied, relative residual} per system.
template <class Pass>
int refine_iterate(const crsolve_plan* p, const Ctx& c, Pass pass, std::vector<char>& fb,
                   std::vector<double>& tab)
{
    std::vector<double> nh, prev(p->batch, 0.0);
    tab.assign(2 * p->batch, 0.0);
    int it = 0, rc;
    for (;;) {
        if ((rc = read_norms(c, nh)))
            return rc;
        bool done = true;
        for (int s = 0; s < p->batch; ++s) {
            if (fb[s])
                continue;
            const double rel = rel_of(nh, s);
            tab[2 * s] = it;
            tab[2 * s + 1] = rel;
            if (rel <= p->rtol)
                continue;
            if (it > 0 && !(rel < prev[s])) {
                fb[s] = 1; // no progress: FP32 cannot refine this system
                continue;
            }
            prev[s] = rel;
            done = false;
        }
        if (done)
            break;
        if (it >= p->max_refine) {
            for (int s = 0; s < p->batch; ++s)
                if (!fb[s] && !(tab[2 * s + 1] <= p->rtol))
                    fb[s] = 1;
            break;
        }
        if ((rc = pass(false)))
            return rc;
        ++it;
    }
    return CRSOLVE_OK;
}

// The one-system FP64 plan of system s in the fallback region: factor
// (y == nullptr) or factor and solve, then that system's info record
// (fp64_fallback = fbflag).
void fallback_sys(const crsolve_plan* p, char* ws, hipStream_t st, int s, const void* A,
                  const void* B, const void* y, void* x, crsolve_info* info, int fbflag)
{
    const crsolve_plan* q = p->fbs[s].get();
    Ctx cf = make_ctx(q, ws + p->off_fb, st);
    (void)upload(q, cf.ws, st);
    const size_t e = sizeof(cx<double>);
    const char* As = (const char*)A + (size_t)p->offA[s] * e;
    const char* Bs = (const char*)B + (size_t)p->offB[s] * e;
    init_flags(cf);
    if (y) {
        levels_down(cf, As, Bs, (const char*)y + (size_t)p->offy[s] * e, 1, 1);
        levels_up(cf, (char*)x + (size_t)p->offy[s] * e);
    } else {
        levels_down(cf, As, Bs, nullptr, 1, 0);
    }
    finalize(cf, info ? info + s : nullptr, fbflag);
}

// Fallback bits of the systems (the workspace keeps them for later solves).
int write_fbits(const Ctx& c, const std::vector<char>& fb)
{
    std::vector<int32_t> h(fb.begin(), fb.end());
    if (hipMemcpyAsync(c.ws + c.p->off_fbits, h.data(), sizeof(int32_t) * h.size(),
                       hipMemcpyHostToDevice, c.st) != hipSuccess ||
        hipStreamSynchronize(c.st) != hipSuccess)
        return CRSOLVE_EHIP;
    return CRSOLVE_OK;
}

int read_fbits(const Ctx& c, std::vector<char>& fb)
{
    std::vector<int32_t> h(c.p->batch);
    if (hipMemcpyAsync(h.data(), c.ws + c.p->off_fbits, sizeof(int32_t) * h.size(),
                       hipMemcpyDeviceToHost, c.st) != hipSuccess ||
        hipStreamSynchronize(c.st) != hipSuccess)
        return CRSOLVE_EHIP;
    fb.assign(h.begin(), h.end());
    return CRSOLVE_OK;
}

int read_flags(const Ctx& c, std::vector<unsigned long long>& fl)
{
    fl.resize(c.p->batch);
    if (hipMemcpyAsync(fl.data(), c.flags, sizeof(unsigned long long) * fl.size(),
                       hipMemcpyDeviceToHost, c.st) != hipSuccess ||
        hipStreamSynchronize(c.st) != hipSuccess)
        return CRSOLVE_EHIP;
    return CRSOLVE_OK;
}

// After the refinement: the systems marked in fb are solved by their FP64
// plans; the residuals of those are measured for the record; the info
// records get {corrections, residual} (no correction counts for a fallback
// system) and the workspace keeps the fallback bits.
int finish_refine(const crsolve_plan* p, const Ctx& c, const void* A, const void* B,
                  const void* y, void* x, crsolve_info* info, const std::vector<char>& fb,
                  std::vector<double>& tab)
{
    int rc;
    bool any = false;
    for (int s = 0; s < p->batch; ++s)
        if (fb[s]) {
            fallback_sys(p, c.ws, c.st, s, A, B, y, x, info, 1);
            any = true;
        }
    if (any) {
        residual(c, A, B, x, y, false);
        std::vector<double> nh;
        if ((rc = read_norms(c, nh)))
            return rc;
        for (int s = 0; s < p->batch; ++s)
            if (fb[s]) {
                tab[2 * s] = 0;
                tab[2 * s + 1] = rel_of(nh, s);
            }
    }
    if ((rc = write_fbits(c, fb)))
        return rc;
    if ((rc = write_refine_info(c, info, tab)))
        return rc;
    return last_err();
}

// crsolve_factor_solve of the mixed form: the fused first pass, one
// synchronization for the breakdown flags and the residual norms, the
// refinement passes, then the FP64 fallback of the systems that need it.
int factor_solve_refine(const crsolve_plan* p, const void* A, const void* B, const void* y,
                        void* x, char* ws, crsolve_info* info, hipStream_t st)
{
    Ctx c = make_ctx(p, ws, st);
    int rc;
    if (p->graphs_on) {
        rc = with_graph(p, gkey(4, {A, B, y, x, ws}), ws, st,
                        [&](const Ctx& g) { enqueue_refine_fused(g, A, B, y, x); });
        if (rc)
            return rc;
    } else {
        if ((rc = upload(p, ws, st)))
            return rc;
        enqueue_refine_fused(c, A, B, y, x);
    }
    std::vector<unsigned long long> fl;
    if ((rc = read_flags(c, fl)))
        return rc;
    std::vector<char> fb(p->batch, 0);
    for (int s = 0; s < p->batch; ++s)
        fb[s] = fl[s] != crs::kNoFail;
    finalize(c, info, 0);
    auto pass = [&](bool first) -> int {
        if (!p->graphs_on) {
            enqueue_refine_pass(c, A, B, y, x, first);
            return CRSOLVE_OK;
        }
        return with_graph(p, gkey(3, {A, B, y, x, ws}), ws, st,
                          [&](const Ctx& g) { enqueue_refine_pass(g, A, B, y, x, first); });
    };
    std::vector<double> tab;
    if ((rc = refine_iterate(p, c, pass, fb, tab)))
        return rc;
    return finish_refine(p, c, A, B, y, x, info, fb, tab);
}

// FP32 factorization with FP64 tail.  Systems whose FP32 factorization broke
// down are factored by their FP64 plans (for their info record; a later
// solve redoes it, as the fallback region holds one system at a time) and
// marked for the FP64 path.  With verdict64 (the definiteness test) every
// system is factored in FP64 and its record is the FP64 one; a system that
// fails there is marked too.
int factor_refine(const crsolve_plan* p, const void* A, const void* B, char* ws,
                  crsolve_info* info, hipStream_t st, bool verdict64)
{
    Ctx c = make_ctx(p, ws, st);
    int rc;
    if (p->graphs_on) {
        rc = with_graph(p, gkey(1, {A, B, ws}), ws, st,
                        [&](const Ctx& g) { enqueue_refine_factor(g, A, B); });
        if (rc)
            return rc;
    } else {
        if ((rc = upload(p, ws, st)))
            return rc;
        enqueue_refine_factor(c, A, B);
    }
    std::vector<unsigned long long> fl;
    if ((rc = read_flags(c, fl)))
        return rc;
    finalize(c, info, 0);
    std::vector<char> fb(p->batch, 0);
    for (int s = 0; s < p->batch; ++s) {
        const bool f32fail = fl[s] != crs::kNoFail;
        if (!f32fail && !verdict64)
            continue;
        fallback_sys(p, ws, st, s, A, B, nullptr, nullptr, info, f32fail ? 1 : 0);
        fb[s] = f32fail;
        if (verdict64 && !f32fail) {
            // the FP64 verdict of a system the FP32 factorization passed
            unsigned long long f64 = 0;
            if (hipMemcpyAsync(&f64, ws + p->off_fb + p->fbs[s]->off_flags, sizeof(f64),
                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return CRSOLVE_EHIP;
            fb[s] = f64 != crs::kNoFail;
        }
    }
    if ((rc = write_fbits(c, fb)))
        return rc;
    return last_err();
}

int solve_refine(const crsolve_plan* p, char* ws, const void* A, const void* B, const void* y,
                 void* x, crsolve_info* info, hipStream_t st)
{
    Ctx c = make_ctx(p, ws, st);
    int rc = upload(p, ws, st);
    if (rc)
        return rc;
    std::vector<char> fb;
    if ((rc = read_fbits(c, fb)))
        return rc;
    finalize(c, info, 0);
    auto pass = [&](bool first) -> int {
        if (!p->graphs_on) {
            enqueue_refine_pass(c, A, B, y, x, first);
            return CRSOLVE_OK;
        }
        return with_graph(p, gkey(first ? 2 : 3, {A, B, y, x, ws}), ws, st,
                          [&](const Ctx& g) { enqueue_refine_pass(g, A, B, y, x, first); });
    };
    // x_0 = A^{-1} y with the mixed factors, then its residual
    if ((rc = pass(true)))
        return rc;
    std::vector<double> tab;
    if ((rc = refine_iterate(p, c, pass, fb, tab)))
        return rc;
    return finish_refine(p, c, A, B, y, x, info, fb, tab);
}

int validate(const crsolve_desc* d)
{
    if (!d || d->batch < 1 || !d->N || !d->m || !d->k)
        return CRSOLVE_EINVAL;
    if (d->dtype != CRSOLVE_C128 && d->dtype != CRSOLVE_C64 && d->dtype != CRSOLVE_R64 &&
        d->dtype != CRSOLVE_R32)
        return CRSOLVE_EINVAL;
    if (d->precision != CRSOLVE_PREC_NATIVE && d->precision != CRSOLVE_PREC_FP32_REFINE)
        return CRSOLVE_EINVAL;
    if (d->schedule != CRSOLVE_SCHED_CR && d->schedule != CRSOLVE_SCHED_PCR)
        return CRSOLVE_EINVAL;
    if (d->precision == CRSOLVE_PREC_FP32_REFINE &&
        (d->dtype != CRSOLVE_C128 || d->schedule != CRSOLVE_SCHED_CR))
        return CRSOLVE_EUNSUPPORTED;
    if (d->precision == CRSOLVE_PREC_FP32_REFINE && (d->max_refine < 0 || !(d->rtol >= 0)))
        return CRSOLVE_EINVAL;
    if (d->schedule == CRSOLVE_SCHED_PCR &&
        (d->dtype != CRSOLVE_C128 || d->precision != CRSOLVE_PREC_NATIVE))
        return CRSOLVE_EUNSUPPORTED;
    if (d->pcr_tail_blocks < 0)
        return CRSOLVE_EINVAL;
    if ((d->dtype == CRSOLVE_R64 || d->dtype == CRSOLVE_R32) &&
        (d->precision != CRSOLVE_PREC_NATIVE || d->schedule != CRSOLVE_SCHED_CR))
        return CRSOLVE_EUNSUPPORTED;
    if (d->pcr_tail_blocks > 0 && d->precision != CRSOLVE_PREC_NATIVE &&
        d->schedule == CRSOLVE_SCHED_CR)
        return CRSOLVE_EUNSUPPORTED;
    for (int s = 0; s < d->batch; ++s) {
        if (d->N[s] < 1 || d->m[s] < 1 || d->k[s] < 1)
            return CRSOLVE_EINVAL;
        if (d->m[s] > kClsM[kNumCls - 1])
            return CRSOLVE_EUNSUPPORTED;
        if (d->m[s] > 64 && d->N[s] > (1 << 24))
            return CRSOLVE_EUNSUPPORTED; // keeps the tiled kernels' work-item counts in range
        if ((int64_t)d->N[s] >= (1ll << 30))
            return CRSOLVE_EUNSUPPORTED;
    }
    return CRSOLVE_OK;
}

crsolve_plan* new_plan(const crsolve_desc* d, crsolve_precision prec, int* rc)
{
    crsolve_plan* p = new (std::nothrow) crsolve_plan();
    if (!p) {
        *rc = CRSOLVE_EINVAL;
        return nullptr;
    }
    p->batch = d->batch;
    p->N.assign(d->N, d->N + d->batch);
    p->m.assign(d->m, d->m + d->batch);
    p->k.assign(d->k, d->k + d->batch);
    p->dtype = d->dtype;
    p->real = d->dtype == CRSOLVE_R64 || d->dtype == CRSOLVE_R32;
    p->prec = prec;
    p->sched = d->schedule;
    p->rtol = d->rtol;
    p->max_refine = d->max_refine;
    p->tail = d->fp64_tail_blocks;
    p->hyb = d->schedule == CRSOLVE_SCHED_CR ? d->pcr_tail_blocks : 0;
    p->cls.resize(p->batch);
    int64_t oa = 0, ob = 0, oy = 0, on = 0;
    for (int s = 0; s < p->batch; ++s) {
        p->cls[s] = cls_of(p->m[s]);
        p->offA.push_back(oa);
        p->offB.push_back(ob);
        p->offy.push_back(oy);
        oa += (int64_t)p->N[s] * p->m[s] * p->m[s];
        ob += (int64_t)(p->N[s] - 1) * p->m[s] * p->m[s];
        oy += (int64_t)p->N[s] * p->m[s] * p->k[s];
        on += p->N[s];
    }
    p->totA = oa;
    p->totB = ob;
    p->toty = oy;
    p->totN = on;
    if (prec == CRSOLVE_PREC_FP32_REFINE) {
        for (int s = 0; s < p->batch; ++s) {
            crsolve_desc dn = *d;
            dn.batch = 1;
            dn.N = d->N + s;
            dn.m = d->m + s;
            dn.k = d->k + s;
            dn.precision = CRSOLVE_PREC_NATIVE;
            dn.dtype = CRSOLVE_C128;
            p->fbs.emplace_back(new_plan(&dn, CRSOLVE_PREC_NATIVE, rc));
            if (!p->fbs.back()) {
                delete p;
                return nullptr;
            }
            p->fbs.back()->timing_parent = p;
        }
    }
    *rc = build_plan(p);
    if (*rc != CRSOLVE_OK) {
        delete p;
        return nullptr;
    }
    return p;
}

// ------------------------------------------------- no-allocation entry point

// Workspace of crsolve_factor_solve_noalloc: a file-scope device array that
// every GPU the library runs on holds from module load to process end.  In
// host code its name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, looked up once per device.
constexpr size_t kScratchBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr; // per device id, null until looked up

int scratch_ptr(void** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return CRSOLVE_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((size_t)dev >= g_scratch_ptr.size())
        g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return CRSOLVE_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CRSOLVE_OK;
}

} // namespace

// ======================================================================= C ABI

extern "C" {

int crsolve_plan_create(const crsolve_desc* d, crsolve_plan** out)
{
    if (!out)
        return CRSOLVE_EINVAL;
    int rc = validate(d);
    if (rc)
        return rc;
    crsolve_plan* p = new_plan(d, d->precision, &rc);
    if (!p)
        return rc ? rc : CRSOLVE_EINVAL;
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
        cnt[p->reckid[i] & 255] += 1;
        ms[p->reckid[i] & 255] += t;
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

int crsolve_residual(const crsolve_plan* p, void* ws, size_t ws_bytes, const void* A,
                     const void* B, const void* x, const void* y, double* rel, void* stream)
{
    if (!p || !rel)
        return CRSOLVE_EINVAL;
    if (p->resid.empty())
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!aligned(A, 16) || (any_B(p) && !aligned(B, 16)) || !aligned(x, 16) || !aligned(y, 16))
        return CRSOLVE_EINVAL;
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    residual(c, A, B, x, y, false);
    std::vector<double> nh;
    if ((rc = read_norms(c, nh)))
        return rc;
    for (int s = 0; s < p->batch; ++s)
        rel[s] = nh[2 * s + 1] > 0 ? std::sqrt(nh[2 * s] / nh[2 * s + 1]) : 0.0;
    return last_err();
}

int crsolve_set_graphs(crsolve_plan* p, int enable)
{
    if (!p)
        return CRSOLVE_EINVAL;
    p->graphs_on = enable != 0;
    if (!enable)
        p->drop_graphs();
    return CRSOLVE_OK;
}

int crsolve_set_tuning(crsolve_plan* p, const char* choice)
{
    if (!p || !choice)
        return CRSOLVE_EINVAL;
    // tokens "r<role>c<class>f<precision>=<variant>;", "tw=<waves>;",
    // "tb=<blocks>;"
    const char* q = choice;
    while (*q) {
        int r, c, f, v, n = 0;
        long long lv = 0;
        if (std::sscanf(q, "tw=%lld;%n", &lv, &n) == 1 && n > 0) {
            if (lv < 1 || lv > (1ll << 20))
                return CRSOLVE_EINVAL;
            p->tail_waves = lv;
            q += n;
            continue;
        }
        n = 0;
        if (std::sscanf(q, "tb=%lld;%n", &lv, &n) == 1 && n > 0) {
            if (lv < 0 || lv > (1ll << 30))
                return CRSOLVE_EINVAL;
            p->tail_blocks = lv;
            q += n;
            continue;
        }
        n = 0;
        if (std::sscanf(q, "r%dc%df%d=%d;%n", &r, &c, &f, &v, &n) != 4 || n == 0)
            return CRSOLVE_EINVAL;
        if (r < 0 || r > 2 || c < 0 || c >= kNumCls || f < 0 || f > 1 || v < 0 || v > 1)
            return CRSOLVE_EINVAL;
        p->var[r][c][f] = v;
        q += n;
    }
    p->drop_graphs();
    return CRSOLVE_OK;
}

int crsolve_autotune(crsolve_plan* p, const void* A, const void* B, const void* y, void* ws,
                     size_t ws_bytes, void* x, void* stream, char* choice, size_t cap)
{
    if (!p || !choice || cap < 2)
        return CRSOLVE_EINVAL;
    if (p->sched != CRSOLVE_SCHED_CR || p->prec != CRSOLVE_PREC_NATIVE)
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    const size_t es = io_esz(p);
    if (!aligned(A, es) || (any_B(p) && !aligned(B, es)) || !aligned(y, es) || !aligned(x, es))
        return CRSOLVE_EINVAL;
    const bool graphs = p->graphs_on;
    p->graphs_on = false;
    hipStream_t st = (hipStream_t)stream;
    double t[2][3][kNumCls][2] = {};
    bool seen[3][kNumCls][2] = {};
    for (int v = 0; v < 2; ++v) {
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < kNumCls; ++c)
                for (int f = 0; f < 2; ++f)
                    p->var[r][c][f] = v;
        Ctx c = make_ctx(p, ws, st);
        for (int rep = 0; rep < 3; ++rep) {
            if (rep == 1)
                crsolve_timing_enable(p, 1);
            if ((rc = upload(p, c.ws, st)))
                return rc;
            enqueue_native_fs(c, A, B, y, x, nullptr);
        }
        if (hipStreamSynchronize(st) != hipSuccess)
            return CRSOLVE_EHIP;
        for (size_t i = 0; i < p->reckid.size(); ++i) {
            const int kid = p->reckid[i] & 255, cls = (p->reckid[i] >> 8) & 15,
                      f64 = (p->reckid[i] >> 12) & 1;
            if (kid > KID_BACK)
                continue;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p->evpool[2 * i], p->evpool[2 * i + 1]) != hipSuccess)
                return CRSOLVE_EHIP;
            t[v][kid][cls][f64] += ms;
            seen[kid][cls][f64] = true;
        }
        crsolve_timing_enable(p, 0);
    }
    std::string out;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < kNumCls; ++c)
            for (int f = 0; f < 2; ++f) {
                // tiled classes have one elimination and one back-substitution
                // kernel, and above 64 one reduced-system form as well
                const bool tuned = seen[r][c][f] && !(tiled(c) && r != 1) && c != kBig;
                const int v = (tuned && t[1][r][c][f] < t[0][r][c][f]) ? 1 : 0;
                p->var[r][c][f] = v;
                if (tuned)
                    out += "r" + std::to_string(r) + "c" + std::to_string(c) + "f" +
                           std::to_string(f) + "=" + std::to_string(v) + ";";
            }
    // launch shapes of the few-block levels of the one-wave MFMA classes:
    // whole steps timed for each pair, the fastest kept
    bool mf = false;
    for (int s = 0; s < p->batch; ++s)
        mf |= mf_class(p->cls[s]);
    if (mf) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return CRSOLVE_EHIP;
        const int64_t cw[3] = {1024, 2048, 4096}, cb[3] = {512, 1024, 2048};
        float best = 0.f;
        int64_t bw = p->tail_waves, bb = p->tail_blocks;
        Ctx c = make_ctx(p, ws, st);
        for (int i = 0; i < 3 && rc == CRSOLVE_OK; ++i)
            for (int j = 0; j < 3 && rc == CRSOLVE_OK; ++j) {
                p->tail_waves = cw[i];
                p->tail_blocks = cb[j];
                float tmin = 0.f;
                for (int rep = 0; rep < 3; ++rep) {
                    if ((rc = upload(p, c.ws, st)))
                        break;
                    (void)hipEventRecord(e0, st);
                    enqueue_native_fs(c, A, B, y, x, nullptr);
                    (void)hipEventRecord(e1, st);
                    float ms = 0.f;
                    if (hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        rc = CRSOLVE_EHIP;
                        break;
                    }
                    if (rep > 0 && (rep == 1 || ms < tmin))
                        tmin = ms;
                }
                if (rc == CRSOLVE_OK && (best == 0.f || tmin < best)) {
                    best = tmin;
                    bw = cw[i];
                    bb = cb[j];
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc)
            return rc;
        p->tail_waves = bw;
        p->tail_blocks = bb;
        out += "tw=" + std::to_string(bw) + ";tb=" + std::to_string(bb) + ";";
    }
    p->drop_graphs();
    p->graphs_on = graphs;
    p->mark_factored(ws);
    if (out.size() + 1 > cap)
        return CRSOLVE_EINVAL;
    std::memcpy(choice, out.c_str(), out.size() + 1);
    return last_err();
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

namespace {
int factor_entry(crsolve_plan* p, const void* A, const void* B, void* ws, size_t ws_bytes,
                 crsolve_info* info, void* stream, bool verdict64)
{
    if (!p)
        return CRSOLVE_EINVAL;
    if (p->sched != CRSOLVE_SCHED_CR)
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!aligned(A, io_esz(p)) || (any_B(p) && !aligned(B, io_esz(p))))
        return CRSOLVE_EINVAL;
    if (p->prec == CRSOLVE_PREC_FP32_REFINE) {
        rc = factor_refine(p, A, B, (char*)ws, info, (hipStream_t)stream, verdict64);
    } else {
        Ctx c = make_ctx(p, ws, stream);
        if ((rc = upload(p, c.ws, c.st)))
            return rc;
        init_flags(c);
        levels_down(c, A, B, nullptr, 1, 0);
        finalize(c, info, 0);
        rc = last_err();
    }
    if (rc == CRSOLVE_OK)
        p->mark_factored(ws);
    return rc;
}
} // namespace

int crsolve_factor(crsolve_plan* p, const void* A, const void* B, void* ws, size_t ws_bytes,
                   crsolve_info* info, void* stream)
{
    return factor_entry(p, A, B, ws, ws_bytes, info, stream, false);
}

int crsolve_check_hpd(crsolve_plan* p, const void* A, const void* B, void* ws, size_t ws_bytes,
                      crsolve_info* info, void* stream)
{
    // the factorization is the test: its flag is the verdict (FP64's for the
    // mixed form)
    return factor_entry(p, A, B, ws, ws_bytes, info, stream, true);
}

int crsolve_solve(const crsolve_plan* p, void* ws, size_t ws_bytes, const void* A, const void* B,
                  const void* y, void* x, crsolve_info* info, void* stream)
{
    if (!p)
        return CRSOLVE_EINVAL;
    if (p->sched != CRSOLVE_SCHED_CR)
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!p->is_factored(ws))
        return CRSOLVE_ESTATE;
    if (!aligned(y, io_esz(p)) || !aligned(x, io_esz(p)))
        return CRSOLVE_EINVAL;
    if (p->prec == CRSOLVE_PREC_FP32_REFINE) {
        if (!aligned(A, 16) || (any_B(p) && !aligned(B, 16)))
            return CRSOLVE_EINVAL;
        return solve_refine(p, (char*)ws, A, B, y, x, info, (hipStream_t)stream);
    }
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    levels_down(c, nullptr, nullptr, y, 0, 1);
    levels_up(c, x);
    finalize(c, info, 0);
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
    const size_t es = io_esz(p);
    if (!aligned(A, es) || (any_B(p) && !aligned(B, es)) || !aligned(y, es) || !aligned(x, es))
        return CRSOLVE_EINVAL;
    if (p->prec == CRSOLVE_PREC_FP32_REFINE) {
        rc = factor_solve_refine(p, A, B, y, x, (char*)ws, info, (hipStream_t)stream);
    } else if (p->graphs_on) {
        rc = with_graph(p, gkey(0, {A, B, y, x, ws, info}), (char*)ws, (hipStream_t)stream,
                        [&](const Ctx& g) { enqueue_native_fs(g, A, B, y, x, info); });
        rc = rc ? rc : last_err();
    } else {
        Ctx c = make_ctx(p, ws, stream);
        if ((rc = upload(p, c.ws, c.st)))
            return rc;
        enqueue_native_fs(c, A, B, y, x, info);
        rc = last_err();
    }
    if (rc == CRSOLVE_OK && p->sched == CRSOLVE_SCHED_CR)
        p->mark_factored(ws);
    return rc;
}

int crsolve_factor_solve_noalloc(crsolve_plan* p, const void* A, const void* B, const void* y,
                                 void* x, crsolve_info* info, void* stream)
{
    if (!p)
        return CRSOLVE_EINVAL;
    if (p->prec != CRSOLVE_PREC_NATIVE)
        return CRSOLVE_EUNSUPPORTED;
    if (p->ws_bytes > kScratchBytes)
        return CRSOLVE_EWORKSPACE;
    const size_t es = io_esz(p);
    if (!aligned(A, es) || (any_B(p) && !aligned(B, es)) || !aligned(y, es) || !aligned(x, es))
        return CRSOLVE_EINVAL;
    void* ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc)
        return rc;
    // eager launches only: no graph, no timing events
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    const bool timing = tplan(p)->timing;
    tplan(p)->timing = false;
    enqueue_native_fs(c, A, B, y, x, info);
    tplan(p)->timing = timing;
    return last_err();
}

int crsolve_backward(const crsolve_plan* p, void* ws, size_t ws_bytes, const void* x,
                     const void* grad_x, void* grad_y, void* grad_A, void* grad_B, void* stream)
{
    if (!p)
        return CRSOLVE_EINVAL;
    if (p->sched != CRSOLVE_SCHED_CR || p->prec != CRSOLVE_PREC_NATIVE || p->real)
        return CRSOLVE_EUNSUPPORTED;
    int rc = check_ws(p, ws, ws_bytes);
    if (rc)
        return rc;
    if (!p->is_factored(ws))
        return CRSOLVE_ESTATE;
    const size_t es = io_esz(p);
    if (!aligned(x, es) || !aligned(grad_x, es) || !aligned(grad_y, es) || !aligned(grad_A, es) ||
        (any_B(p) && !aligned(grad_B, es)))
        return CRSOLVE_EINVAL;
    Ctx c = make_ctx(p, ws, stream);
    if ((rc = upload(p, c.ws, c.st)))
        return rc;
    // lam = A^{-1} grad_x with the stored factors, written straight into grad_y
    levels_down(c, nullptr, nullptr, grad_x, 0, 1);
    levels_up(c, grad_y);
    for (const Launch& L : p->grad) {
        if (L.f64)
            run_grad<double>(c, L, x, grad_y, grad_A, grad_B);
        else
            run_grad<float>(c, L, x, grad_y, grad_A, grad_B);
    }
    return last_err();
}

} // extern "C"
