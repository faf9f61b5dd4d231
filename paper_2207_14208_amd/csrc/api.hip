// Host side of the C ABI: argument checks, allocation of the level
// hierarchy, work lists, the cycle launch sequence, hipGraph capture and
// replay, batches and the single-step entry points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "bcmg_internal.h"
#include "launch.h"
#include "mem.h"

using namespace bcmg;

namespace {

thread_local std::string g_err;

bcmg_status fail(bcmg_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(e_ == hipErrorOutOfMemory ? BCMG_ERR_OOM : BCMG_ERR_DEVICE, "%s: %s", #expr,   \
                        hipGetErrorString(e_));                                                        \
    } while (0)

// finest-level red-black sweep timing (bcmg_timing_*): while enabled, batches
// launch their cycles directly (no graph: events recorded during capture
// cannot be timed) with an event pair around every finest-level sweep; the
// durations are summed after each synchronised step.
struct Timing {
    bool on = false;
    long long launches = 0;
    double ms = 0.0;
    long long nodes = 0;
} g_timing;

}  // namespace

struct LevelH {
    int N = 0, n = 0;
    long long nn = 0;
    double h = 0.0;
    long long ni = 0, ng = 0, nb = 0;
    uint8_t *cls = nullptr;
    double *phi = nullptr;
    int *gidx = nullptr, *gcode = nullptr, *gfb = nullptr;
    double *gtau = nullptr, *gdtau = nullptr, *geta = nullptr, *gn = nullptr, *gq = nullptr;
    double *gnd = nullptr;                 // Neumann derivative coefficients [3*ng] (Neumann problems only)
    int *bidx = nullptr;
    long long ne = 0, nr = 0;              // entries of the extension / restriction rows
    int *bneed = nullptr;                  // band entries read by the prolongation (levels >= 1)
    long long nbn = 0;
    int *ilist = nullptr;                  // INSIDE nodes, even i+j+k first (levels up to kListNodes nodes)
    int nred = 0;
    int *eptr = nullptr, *eidx = nullptr;  // extension rows (CSR over ghost-list indices)
    double *ecoef = nullptr;
    int *rptr = nullptr, *ridx = nullptr;  // restriction rows of this level's ghosts (levels >= 1)
    double *rcoef = nullptr;
    void *u = nullptr, *rhs = nullptr, *r = nullptr;
    long long half = 0;  // u, rhs and r stored split by node parity (see NodeArr): (nn + 1) / 2, else 0
    double *gnew = nullptr;
    std::vector<Item> segs;  // desc field 0; patched when copied into a table
    // coarsest level
    int nc = 0, singular = 0;
    double *ainv = nullptr;
    int *cmap = nullptr;
};

struct bcmg_problem {
    int d = 0, N = 0, L = 0;
    bcmg_options opt{};
    hipStream_t stream = nullptr;
    MemSource mem;            // where its device memory comes from (fixed at setup)
    int device = 0;           // device current at setup
    int fp32 = 0;
    LevelH lev[kMaxLevels];
    double *rhs64 = nullptr;  // finest FP64 right-hand side (f on INSIDE, g(Q) on GHOST)
    double *r64 = nullptr;    // finest FP64 residual scratch
    std::vector<void *> allocs;
    char *arena = nullptr;       // current zeroed chunk that small arrays are carved from
    size_t arena_used = 0, arena_size = 0;
    long long bytes = 0;
    // single-step entry points
    Desc *d_step = nullptr;   // [L]
    SlotState *d_stepst = nullptr;
    Item *d_stepitems = nullptr;  // per level: segs, gch, bch
    std::vector<int> off_seg, off_gch, off_bch, n_seg, n_gch, n_bch;
    double *d_partials = nullptr;
    size_t partials_cap = 0;
    NormRange *d_range = nullptr;
    double *d_out = nullptr;
    Desc *h_stage = nullptr;  // pinned staging for descriptor uploads
    int *d_lvl = nullptr;     // [1] index of the coarsest level (the coarse-solve list)
    bcmg_batch *solo = nullptr;
};

struct Lists {
    Item *segs = nullptr;
    int nseg = 0;
    Item *gch = nullptr;
    int ngch = 0;
    Item *bch = nullptr;
    int nbch = 0;
    Item *csegs = nullptr;
    int ncseg = 0;
    Item *cbch = nullptr;  // band chunks of the next coarser level (its extension before prolongation)
    int ncbch = 0;
    Item *cgch = nullptr;  // ghost chunks of the next coarser level (restriction)
    int ncgch = 0;
    // segments of the problems whose finest level this is: the first red
    // half-sweep of the pre-smoothing runs on them only (on the others the
    // restriction into the level has done it)
    Item *rsegs = nullptr;
    int nrseg = 0;
    bool split = false;  // every problem's level here has split storage (paired sweeps pay there)
};

struct bcmg_batch {
    int cap = 0;
    MemSource mem;                      // where its device memory comes from (fixed at creation)
    hipStream_t stream = nullptr;       // private non-blocking stream (graph capture needs one)
    hipStream_t user_stream = nullptr;  // caller's stream, joined at every entry
    hipEvent_t join = nullptr;
    long long fine_inside = 0;          // INSIDE nodes on the finest aligned level
    int d = 0, fp32 = 0, nu1 = 2, nu2 = 1, K = 4, max_hist = 0;
    int wcycle = 0, jacobi = 0;         // cycle shape and interior smoother shared by the slots
    int neu = 0;                        // some slot has Neumann ghost rows (set at rebuild)
    std::vector<bcmg_problem *> prob;
    std::vector<double *> u;
    std::vector<double> rtol;
    // device state
    SlotState *d_state = nullptr;
    SlotState *h_state = nullptr;  // pinned mirror
    double *d_rtol2 = nullptr;
    double *d_hist = nullptr;
    int hist_stride = 0;
    NormRange *d_ranges = nullptr;
    // rebuilt on membership change
    Desc *d_desc = nullptr;
    size_t desc_cap = 0;
    Desc *d_outer = nullptr;
    float **d_eptr = nullptr;
    Item *d_items = nullptr;
    size_t items_cap = 0;
    int *d_coarse = nullptr;
    int ncoarse = 0;
    std::vector<int> desc_base;  // per slot: index of its finest level's descriptor in d_desc (-1: empty)
    double *d_partials = nullptr;
    size_t partials_cap = 0;
    // norm of the finest residual by norm_blocks workgroups per slot (block
    // sums and per-slot arrival counters, zero between launches)
    int norm_blocks = 1;
    double *d_norm_blk = nullptr;
    int *d_norm_cnt = nullptr;
    size_t norm_cap = 0;
    int A = 0;
    std::vector<Lists> lv;
    Item *fsegs = nullptr, *fgch = nullptr;
    int nfseg = 0, nfgch = 0;
    int Ac = 0;                    // aligned levels 0..Ac run in the per-problem coarse workgroup
    long long coarse_nodes = kCoarseNodes;
    int pair_segs = kSweepPairSegs;  // FP32 sweeps of split levels over this many segments take four per wavefront
    CoarseProg *d_progs = nullptr;
    int nprog = 0;
    LdsProg *d_lprogs = nullptr;   // the same programs with their levels staged in LDS
    uint32_t *d_limage = nullptr;  // their images (the LDS part fixed during a solve)
    size_t limage_cap = 0;         //   capacity in words
    size_t lds_bytes = 0;          // dynamic LDS per workgroup of k_coarse_lds (0: LDS path off)
    size_t lds_budget = 0;
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_cycles = 0;
    // bcmg_solve's blocks of j cycles with one check after them (j = 2..)
    hipGraph_t bgraph[kMaxCheckInterval + 1] = {};
    hipGraphExec_t bexec[kMaxCheckInterval + 1] = {};
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;  // timing events of direct launches
};

namespace {

// Setup phase timer: with BCMG_SETUP_TIMING=1 in the environment, setup
// prints the wall time of its phases (after a stream synchronisation) to
// stderr.
struct PhaseTimer {
    bool on = false;
    hipStream_t s = nullptr;
    std::chrono::steady_clock::time_point t;
    explicit PhaseTimer(hipStream_t st) : s(st) {
        const char *e = getenv("BCMG_SETUP_TIMING");
        on = e && e[0] == '1';
        t = std::chrono::steady_clock::now();
    }
    void mark(const char *what, int level = -1) {
        if (!on) return;
        hipStreamSynchronize(s);
        const auto now = std::chrono::steady_clock::now();
        fprintf(stderr, "bcmg setup %-14s level %2d %8.3f ms\n", what, level,
                std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};
thread_local PhaseTimer *t_phase = nullptr;

// roctx range over a host-side phase (setup, its levels, solves, batch
// steps, the cycles between two host checks); seen by rocprofv3
// --marker-trace, free without a profiler attached
struct TraceRange {
    explicit TraceRange(const char *fmt, ...) __attribute__((format(printf, 2, 3))) {
        char msg[96];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(msg, sizeof msg, fmt, ap);
        va_end(ap);
        roctxRangePushA(msg);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};
#define PHASE(what, level) \
    do {                   \
        if (t_phase) t_phase->mark(what, level); \
    } while (0)

// Zeroed device memory owned by the problem.  Small arrays are carved from
// zeroed 4 MiB chunks (a problem has ~25 arrays per level: one allocation,
// one fill and one free per chunk instead of per array); large arrays get
// their own allocation.  All come from the problem's memory source.
constexpr size_t kArenaChunk = 4u << 20;

static bcmg_status dalloc_raw(bcmg_problem *P, void **out, size_t bytes) {
    hipError_t e = mem_alloc(P->mem, out, bytes, P->stream);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(BCMG_ERR_OOM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    e = hipMemsetAsync(*out, 0, bytes, P->stream);
    if (e != hipSuccess) return fail(BCMG_ERR_DEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
    P->allocs.push_back(*out);
    P->bytes += (long long)bytes;
    return BCMG_OK;
}

bcmg_status dalloc(bcmg_problem *P, void **out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes > kArenaChunk / 4) return dalloc_raw(P, out, bytes);
    if (!P->arena || P->arena_used + bytes > P->arena_size) {
        void *chunk = nullptr;
        bcmg_status st = dalloc_raw(P, &chunk, kArenaChunk);
        if (st) return st;
        P->arena = (char *)chunk;
        P->arena_used = 0;
        P->arena_size = kArenaChunk;
    }
    *out = P->arena + P->arena_used;
    P->arena_used += bytes;
    return BCMG_OK;
}

template <typename T>
bcmg_status dalloc_t(bcmg_problem *P, T **out, size_t count) {
    void *p = nullptr;
    bcmg_status s = dalloc(P, &p, count * sizeof(T));
    *out = (T *)p;
    return s;
}

void free_problem_memory(bcmg_problem *P) {
    for (void *p : P->allocs) mem_free(P->mem, p, P->stream);
    P->allocs.clear();
    if (P->h_stage) hipHostFree(P->h_stage);
    P->h_stage = nullptr;
}

Item seg_item(int desc, long long start, int x0, int len, int j, int k) {
    Item it;
    it.x = desc;
    it.y = (int)start;
    it.z = x0 | (len << 16);
    it.w = j | (k << 16);
    return it;
}

void append_chunks(std::vector<Item> &out, int desc, long long count) {
    for (long long b = 0; b < count; b += kChunk) {
        Item it;
        it.x = desc;
        it.y = (int)b;
        it.z = (int)std::min<long long>(kChunk, count - b);
        it.w = 0;
        out.push_back(it);
    }
}

Desc make_desc(const bcmg_problem *P, int l, void *u, void *rhs, void *r, int slot) {
    const LevelH &V = P->lev[l];
    Desc D;
    memset(&D, 0, sizeof D);
    D.d = P->d;
    D.n = V.n;
    D.N = V.N;
    D.level = l;
    D.nn = V.nn;
    D.sy = P->d >= 2 ? V.n : 0;
    D.sz = P->d >= 3 ? (long long)V.n * V.n : 0;
    D.h = V.h;
    D.h2 = V.h * V.h;
    D.cls = V.cls;
    D.ng = (int)V.ng;
    D.nb = (int)V.nb;
    D.gidx = V.gidx;
    D.gcode = V.gcode;
    D.gtau = V.gtau;
    D.gdtau = V.gdtau;
    D.bidx = V.bidx;
    D.bneed = V.bneed;
    D.nbn = (int)V.nbn;
    D.eptr = V.eptr;
    D.eidx = V.eidx;
    D.ecoef = V.ecoef;
    D.rptr = V.rptr;
    D.ridx = V.ridx;
    D.rcoef = V.rcoef;
    D.ilist = V.ilist;
    D.ni = (int)V.ni;
    D.nred = V.nred;
    D.u = u;
    D.rhs = rhs;
    D.r = r;
    // the level's own arrays carry its storage order; other arrays (the
    // caller's u, the FP64 right-hand side) are in the natural order
    D.half_u = V.half && (u == V.u || u == V.rhs || u == V.r) ? V.half : 0;
    D.half_r = V.half && (r == V.u || r == V.rhs || r == V.r) ? V.half : 0;
    D.gnew = V.gnew;
    D.nc = V.nc;
    D.singular = V.singular;
    D.ainv = V.ainv;
    D.cmap = V.cmap;
    D.slot = slot;
    D.restrict_mode = P->opt.restrict_mode;
    D.gnd = P->opt.bc == BCMG_BC_NEUMANN ? V.gnd : nullptr;
    D.reaction = P->opt.reaction;
    return D;
}

// Setup temporaries: returned to the memory source on every exit path.
struct Temps {
    hipStream_t s;
    std::vector<void *> held;
    explicit Temps(hipStream_t st) : s(st) {}
    Temps(const Temps &) = delete;
    Temps &operator=(const Temps &) = delete;
    ~Temps() {
        for (void *p : held) scratch_free(p, s);
    }
    template <typename T>
    hipError_t get(T **p, size_t bytes) {
        void *q = nullptr;
        const hipError_t e = scratch_alloc(&q, bytes, s);
        *p = (T *)q;
        if (e == hipSuccess) held.push_back(q);
        return e;
    }
    void put(void *p) {
        auto it = std::find(held.begin(), held.end(), p);
        if (it == held.end()) return;
        held.erase(it);
        scratch_free(p, s);
    }
};

// ------------------------------------------------------------------ setup
// Extension rows of a level: K sweeps of count, prefix sum and write; the
// rows of the last sweep are kept (see k_erow).
bcmg_status build_ext_rows(bcmg_problem *P, LevelH &V, const int *bref, const double *bw, int *h_total) {
    hipStream_t s = P->stream;
    const int nb = (int)V.nb, K = P->opt.ext_iters;
    bcmg_status st;
    if (nb == 0 || K == 0) {  // eptr is zero-filled: every row empty
        if ((st = dalloc_t(P, &V.eidx, 1)) || (st = dalloc_t(P, &V.ecoef, 1))) return st;
        return BCMG_OK;
    }
    Temps tmp(s);
    int *counts = nullptr, *pptr = nullptr, *pidx = nullptr;
    double *pcf = nullptr;
    HIPCHK(tmp.get(&counts, sizeof(int) * nb));
    for (int j = 1; j <= K; j++) {
        int *optr = j == K ? V.eptr : nullptr;
        if (!optr) HIPCHK(tmp.get(&optr, sizeof(int) * (nb + 1)));
        launch_erow(P->d, V.N, V.cls, V.gidx, (int)V.ng, V.bidx, nb, bref, bw, j, pptr, pidx, pcf, nullptr, counts,
                    nullptr, nullptr, s);
        HIPCHK(launch_scan(counts, nb, optr, s));
        HIPCHK(hipMemcpyAsync(h_total, optr + nb, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const size_t tot = (size_t)std::max(*h_total, 1);
        int *oidx = nullptr;
        double *ocf = nullptr;
        if (j == K) {
            V.ne = *h_total;
            if ((st = dalloc_t(P, &V.eidx, tot)) || (st = dalloc_t(P, &V.ecoef, tot))) return st;
            oidx = V.eidx;
            ocf = V.ecoef;
        } else {
            HIPCHK(tmp.get(&oidx, sizeof(int) * tot));
            HIPCHK(tmp.get(&ocf, sizeof(double) * tot));
        }
        launch_erow(P->d, V.N, V.cls, V.gidx, (int)V.ng, V.bidx, nb, bref, bw, j, pptr, pidx, pcf, optr, counts,
                    oidx, ocf, s);
        if (pptr) {
            tmp.put(pptr);
            tmp.put(pidx);
            tmp.put(pcf);
        }
        pptr = j == K ? nullptr : optr;
        pidx = j == K ? nullptr : oidx;
        pcf = j == K ? nullptr : ocf;
    }
    HIPCHK(hipStreamSynchronize(s));
    return BCMG_OK;
}

// Band entries of level l >= 1 whose extended values the prolongation to
// level l-1 reads (see k_need_mark).
bcmg_status build_needed_band(bcmg_problem *P, int l, int *counts, int *offsets, int *total_dev, int *h_total) {
    hipStream_t s = P->stream;
    LevelH &C = P->lev[l];
    const LevelH &F = P->lev[l - 1];
    bcmg_status st;
    const size_t nb = (size_t)std::max<long long>(C.nb, 1);
    if ((st = dalloc_t(P, &C.bneed, nb))) return st;
    if (C.nb == 0) return BCMG_OK;
    Temps tmp(s);
    uint8_t *mark = nullptr, *flag = nullptr;
    HIPCHK(tmp.get(&mark, (size_t)C.nn));
    HIPCHK(tmp.get(&flag, nb));
    HIPCHK(hipMemsetAsync(mark, 0, (size_t)C.nn, s));
    launch_need_mark(P->d, F.N, F.cls, C.cls, mark, F.nn, s);
    launch_need_flags(C.bidx, (int)C.nb, mark, flag, s);
    HIPCHK(launch_compact(flag, (long long)C.nb, 1, counts, offsets, C.bneed, total_dev, s));
    HIPCHK(hipMemcpyAsync(h_total, total_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    C.nbn = *h_total;
    return BCMG_OK;
}

// Restriction rows of the ghosts of level l >= 1 over the ghosts of level l-1.
bcmg_status build_restrict_rows(bcmg_problem *P, int l, int *h_total) {
    hipStream_t s = P->stream;
    LevelH &C = P->lev[l];
    const LevelH &F = P->lev[l - 1];
    const int ng = (int)C.ng;
    bcmg_status st;
    if ((st = dalloc_t(P, &C.rptr, (size_t)ng + 1))) return st;
    if (ng == 0) {
        if ((st = dalloc_t(P, &C.ridx, 1)) || (st = dalloc_t(P, &C.rcoef, 1))) return st;
        return BCMG_OK;
    }
    Temps tmp(s);
    int *counts = nullptr;
    HIPCHK(tmp.get(&counts, sizeof(int) * ng));
    launch_rrow(P->d, C.N, C.gidx, ng, F.N, F.cls, F.gidx, (int)F.ng, F.bidx, (int)F.nb, F.eptr, F.eidx, F.ecoef,
                P->opt.restrict_mode, nullptr, counts, nullptr, nullptr, s);
    HIPCHK(launch_scan(counts, ng, C.rptr, s));
    HIPCHK(hipMemcpyAsync(h_total, C.rptr + ng, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const size_t tot = (size_t)std::max(*h_total, 1);
    C.nr = *h_total;
    if ((st = dalloc_t(P, &C.ridx, tot)) || (st = dalloc_t(P, &C.rcoef, tot))) return st;
    launch_rrow(P->d, C.N, C.gidx, ng, F.N, F.cls, F.gidx, (int)F.ng, F.bidx, (int)F.nb, F.eptr, F.eidx, F.ecoef,
                P->opt.restrict_mode, C.rptr, counts, C.ridx, C.rcoef, s);
    HIPCHK(hipStreamSynchronize(s));
    return BCMG_OK;
}

bcmg_status setup_level(bcmg_problem *P, int l, int *scratch_counts, int *scratch_offsets, int *total_dev,
                        int *h_total) {
    LevelH &V = P->lev[l];
    const TraceRange tr("bcmg_setup level %d (N=%d)", l, V.N);
    const int d = P->d;
    hipStream_t s = P->stream;
    bcmg_status st;
    launch_classify(d, V.n, V.phi, V.cls, s);
    PHASE("classify", l);
    // counts of INSIDE and GHOST nodes, ghost list
    HIPCHK(launch_compact(V.cls, V.nn, C_INSIDE, scratch_counts, scratch_offsets, nullptr, total_dev, s));
    HIPCHK(hipMemcpyAsync(h_total, total_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    V.ni = *h_total;
    if (l == 0 && V.ni == 0) return fail(BCMG_ERR_INVALID, "phi < 0 at no node: the domain holds no unknowns");
    HIPCHK(launch_compact(V.cls, V.nn, C_GHOST, scratch_counts, scratch_offsets, nullptr, total_dev, s));
    HIPCHK(hipMemcpyAsync(h_total, total_dev, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    V.ng = *h_total;
    const size_t ng = (size_t)std::max<long long>(V.ng, 1);
    if ((st = dalloc_t(P, &V.gidx, ng)) || (st = dalloc_t(P, &V.gcode, ng)) || (st = dalloc_t(P, &V.gfb, ng)) ||
        (st = dalloc_t(P, &V.gtau, 3 * ng)) || (st = dalloc_t(P, &V.gdtau, ng)) || (st = dalloc_t(P, &V.geta, ng)) ||
        (st = dalloc_t(P, &V.gn, 3 * ng)) || (st = dalloc_t(P, &V.gq, 3 * ng)) || (st = dalloc_t(P, &V.gnew, ng)))
        return st;
    if (P->opt.bc == BCMG_BC_NEUMANN && (st = dalloc_t(P, &V.gnd, 3 * ng))) return st;
    HIPCHK(launch_compact(V.cls, V.nn, C_GHOST, scratch_counts, scratch_offsets, V.gidx, total_dev, s));
    PHASE("ghost list", l);
    launch_ghost_geometry(d, V.N, l, V.h, V.phi, V.cls, V.gidx, (int)V.ng, P->opt.dtau_mode, P->opt.dtau_const,
                          P->opt.bc, V.gcode, V.gtau, V.gdtau, V.geta, V.gn, V.gq, V.gfb, V.gnd, s);
    PHASE("geometry", l);
    // extension band (only levels that restrict or receive a prolongation need it)
    {
        Temps tmp(s);
        uint8_t *mark = nullptr;
        HIPCHK(tmp.get(&mark, (size_t)V.nn));
        HIPCHK(hipMemsetAsync(mark, 0, (size_t)V.nn, s));
        launch_band_mark(d, V.N, V.cls, V.gidx, (int)V.ng, P->opt.ext_iters, mark, s);
        HIPCHK(launch_compact(mark, V.nn, 1, scratch_counts, scratch_offsets, nullptr, total_dev, s));
        HIPCHK(hipMemcpyAsync(h_total, total_dev, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        V.nb = *h_total;
        const size_t nb = (size_t)std::max<long long>(V.nb, 1);
        int *bref = nullptr;
        double *bw = nullptr;
        if ((st = dalloc_t(P, &V.bidx, nb)) || (st = dalloc_t(P, &V.eptr, nb + 1))) return st;
        HIPCHK(tmp.get(&bref, sizeof(int) * 3 * nb));
        HIPCHK(tmp.get(&bw, sizeof(double) * 3 * nb));
        HIPCHK(launch_compact(mark, V.nn, 1, scratch_counts, scratch_offsets, V.bidx, total_dev, s));
        launch_band_records(d, V.N, V.h, V.phi, V.cls, V.bidx, (int)V.nb, bref, bw, s);
        tmp.put(mark);
        PHASE("band", l);
        st = build_ext_rows(P, V, bref, bw, h_total);
        PHASE("ext rows", l);
        if (st) return st;
    }
    // row segments of INSIDE/GHOST nodes
    {
        Temps tmp(s);
        long long rows = 1;
        for (int k = 1; k < d; k++) rows *= V.n;
        int *ext = nullptr;
        HIPCHK(tmp.get(&ext, sizeof(int) * 4 * rows));
        launch_row_extent(d, V.n, V.cls, ext, ext + rows, ext + 2 * rows, ext + 3 * rows, s);
        std::vector<int> h(4 * rows);
        HIPCHK(hipMemcpyAsync(h.data(), ext, sizeof(int) * 4 * rows, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        V.segs.clear();
        for (long long r = 0; r < rows; r++) {
            const int lo = h[r], hi = h[rows + r];
            if (lo < 0) continue;
            const int j = d >= 2 ? (int)(r % V.n) : 0;
            const int k = d >= 3 ? (int)(r / V.n) : 0;
            const int ia = h[2 * rows + r], ib = h[3 * rows + r];
            for (int x = lo; x <= hi; x += P->opt.seg_len) {
                const int len = std::min(P->opt.seg_len, hi - x + 1);
                Item it = seg_item(0, r * V.n + x, x, len, j, k);
                if (ib >= 0 && ia <= x && x + len - 1 <= ib) it.z |= kSegAllInside;
                V.segs.push_back(it);
            }
        }
    }
    PHASE("segments", l);
    // colour-sorted INSIDE list of a small level (the LDS coarse cycle walks it)
    if (V.nn <= kListNodes) {
        std::vector<uint8_t> hc((size_t)V.nn);
        HIPCHK(hipMemcpyAsync(hc.data(), V.cls, (size_t)V.nn, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int> red, black;
        for (long long p = 0; p < V.nn; p++) {
            if (hc[p] != C_INSIDE) continue;
            long long q = p;
            int par = 0;
            for (int k = 0; k < d; k++) {
                par += (int)(q % V.n);
                q /= V.n;
            }
            ((par & 1) ? black : red).push_back((int)p);
        }
        V.nred = (int)red.size();
        red.insert(red.end(), black.begin(), black.end());
        if ((st = dalloc_t(P, &V.ilist, std::max<size_t>(red.size(), 1)))) return st;
        if (!red.empty())
            HIPCHK(hipMemcpyAsync(V.ilist, red.data(), sizeof(int) * red.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    // level arrays (cycle precision); the finest FP64 level uses caller memory for u
    const size_t esz = P->fp32 ? 4 : 8;
    const long long split_min = l == 0 ? kSplitMinNodes : kSplitMinCoarseNodes;
    if (P->fp32 && P->opt.layout == BCMG_LAYOUT_SPLIT && V.nn > split_min) V.half = (V.nn + 1) / 2;
    // split arrays end in kSplitPad spare entries (the vector loads of the
    // split sweep may read a few entries past the last node)
    const long long alloc_nn = V.nn + (V.half ? kSplitPad : 0);
    if (l > 0 || P->fp32) {
        if ((st = dalloc(P, &V.u, alloc_nn * esz))) return st;
    }
    if (l > 0 || P->fp32) {
        if ((st = dalloc(P, &V.rhs, alloc_nn * esz))) return st;
    }
    if ((st = dalloc(P, &V.r, alloc_nn * esz))) return st;
    return BCMG_OK;
}

bcmg_status setup_coarse(bcmg_problem *P) {
    LevelH &V = P->lev[P->L - 1];
    bcmg_status st;
    const int ncmax = (int)(V.ni + V.ng);
    if (ncmax > kCoarseMax) return fail(BCMG_ERR_INVALID, "coarsest level has %d unknowns (> %d)", ncmax, kCoarseMax);
    double *work = nullptr;
    int *info = nullptr;
    if ((st = dalloc_t(P, &V.ainv, (size_t)std::max(1, ncmax * ncmax))) ||
        (st = dalloc_t(P, &V.cmap, (size_t)std::max(1, ncmax))) ||
        (st = dalloc_t(P, &work, (size_t)std::max(1, 2 * ncmax * ncmax))) || (st = dalloc_t(P, &info, 2)))
        return st;
    launch_coarse_setup(P->d, V.N, V.h, V.cls, V.gidx, (int)V.ng, V.gcode, V.gtau, P->opt.bc, V.gnd, P->opt.reaction,
                        work, V.ainv, V.cmap, info, P->stream);
    int h[2];
    HIPCHK(hipMemcpyAsync(h, info, sizeof h, hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipStreamSynchronize(P->stream));
    V.nc = h[0];
    V.singular = h[1];
    return BCMG_OK;
}

bcmg_status setup_step_tables(bcmg_problem *P) {
    bcmg_status st;
    std::vector<Item> all;
    P->off_seg.assign(P->L, 0);
    P->off_gch.assign(P->L, 0);
    P->off_bch.assign(P->L, 0);
    P->n_seg.assign(P->L, 0);
    P->n_gch.assign(P->L, 0);
    P->n_bch.assign(P->L, 0);
    for (int l = 0; l < P->L; l++) {
        const LevelH &V = P->lev[l];
        P->off_seg[l] = (int)all.size();
        for (Item it : V.segs) {
            it.x = l;
            all.push_back(it);
        }
        P->n_seg[l] = (int)V.segs.size();
        P->off_gch[l] = (int)all.size();
        append_chunks(all, l, V.ng);
        P->n_gch[l] = (int)all.size() - P->off_gch[l];
        P->off_bch[l] = (int)all.size();
        append_chunks(all, l, V.nb);
        P->n_bch[l] = (int)all.size() - P->off_bch[l];
    }
    if ((st = dalloc_t(P, &P->d_stepitems, all.size() + 1))) return st;
    HIPCHK(hipMemcpyAsync(P->d_stepitems, all.data(), all.size() * sizeof(Item), hipMemcpyHostToDevice, P->stream));
    if ((st = dalloc_t(P, &P->d_step, P->L)) || (st = dalloc_t(P, &P->d_stepst, 1)) ||
        (st = dalloc_t(P, &P->d_range, 1)) || (st = dalloc_t(P, &P->d_out, 1)) || (st = dalloc_t(P, &P->d_lvl, 1)))
        return st;
    const int coarsest = P->L - 1;
    HIPCHK(hipMemcpyAsync(P->d_lvl, &coarsest, sizeof(int), hipMemcpyHostToDevice, P->stream));
    SlotState one;
    memset(&one, 0, sizeof one);
    one.active = 1;
    one.max_cycles = 1 << 30;
    HIPCHK(hipMemcpyAsync(P->d_stepst, &one, sizeof one, hipMemcpyHostToDevice, P->stream));
    const size_t np = (size_t)P->n_seg[0] + (size_t)P->n_gch[0] + 1;
    if ((st = dalloc_t(P, &P->d_partials, np))) return st;
    P->partials_cap = np;
    NormRange R{0, P->n_seg[0], 0, P->n_gch[0]};
    HIPCHK(hipMemcpyAsync(P->d_range, &R, sizeof R, hipMemcpyHostToDevice, P->stream));
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bool valid_level(const bcmg_problem *P, int l) { return P && l >= 0 && l < P->L; }

// upload step descriptors for levels [l0, l0+cnt) with the given pointers
bcmg_status upload_step_descs(bcmg_problem *P, int l0, int cnt, void *const *u, void *const *rhs, void *const *r) {
    if (!P->h_stage) HIPCHK(hipHostMalloc((void **)&P->h_stage, sizeof(Desc) * kMaxLevels));
    for (int i = 0; i < cnt; i++) P->h_stage[i] = make_desc(P, l0 + i, u[i], rhs[i], r[i], 0);
    HIPCHK(hipMemcpyAsync(P->d_step + l0, P->h_stage, sizeof(Desc) * cnt, hipMemcpyHostToDevice, P->stream));
    return BCMG_OK;
}

// Scratch of bcmg_residual_norm_noalloc: the norm's partial sums, its range
// record and its result, in a static device array (each device that runs the
// library holds one copy until the process ends).  Host code uses the address
// hipGetSymbolAddress gives on each device, never the array's name.
constexpr long long kNoAllocPartials = 1 << 19;
constexpr long long kNoAllocWords = kNoAllocPartials + 4;  // + NormRange (2 words) + result + pad
static __device__ __align__(256) double scratch[kNoAllocWords];

struct NoAllocScratch {
    std::mutex mu;
    double *ptr[64] = {};
} g_noalloc;

// Look up (once per device, with that device current) the device address of
// the scratch array.
bcmg_status noalloc_scratch_init(int dev) {
    if (dev < 0 || dev >= 64) return fail(BCMG_ERR_DEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_noalloc.mu);
    if (g_noalloc.ptr[dev]) return BCMG_OK;
    double *p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(BCMG_ERR_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_noalloc.ptr[dev] = p;
    return BCMG_OK;
}

double *noalloc_scratch(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(g_noalloc.mu);
    return g_noalloc.ptr[dev];
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char *bcmg_last_error(void) { return g_err.c_str(); }

int32_t bcmg_version(void) { return 100; }

bcmg_status bcmg_default_options(bcmg_options *o) {
    if (!o) return fail(BCMG_ERR_INVALID, "null options");
    o->nu1 = 2;
    o->nu2 = 1;
    o->coarsest_N = 4;
    o->max_cycles = 100;
    o->precision = BCMG_FP64;
    o->dtau_mode = BCMG_DTAU_OPT_EXP;
    o->dtau_const = 1.0;
    o->ext_iters = 4;
    o->restrict_mode = BCMG_RESTRICT_RENORM_FW;
    o->seg_len = kSegLen;
    o->bc = BCMG_BC_DIRICHLET;
    o->reaction = 0.0;
    o->layout = BCMG_LAYOUT_SPLIT;
    o->cycle = BCMG_CYCLE_V;
    o->smoother = BCMG_SMOOTH_RB;
    o->check_interval = 1;
    return BCMG_OK;
}

static bcmg_status check_options(int dim, int N, const bcmg_options *o) {
    if (dim < 1 || dim > 3) return fail(BCMG_ERR_INVALID, "dim must be 1, 2 or 3 (got %d)", dim);
    // the quadratic root interpolant needs 3 nodes per axis on both sides of any node: N >= 4
    if (o->coarsest_N != 4) return fail(BCMG_ERR_INVALID, "coarsest_N must be 4");
    if (N < 2 * o->coarsest_N || (N & (N - 1))) return fail(BCMG_ERR_INVALID, "N must be a power of two >= 2*coarsest_N (got %d)", N);
    const int nmax = dim == 3 ? 1024 : 4096;
    if (N > nmax) return fail(BCMG_ERR_INVALID, "N=%d exceeds the limit %d for dim %d", N, nmax, dim);
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 16 || o->nu2 > 16)
        return fail(BCMG_ERR_INVALID, "nu1, nu2 must be in 0..16 with nu1+nu2 >= 1");
    if (o->max_cycles < 1 || o->max_cycles > 1000) return fail(BCMG_ERR_INVALID, "max_cycles must be in 1..1000");
    if (o->precision != BCMG_FP64 && o->precision != BCMG_MIXED) return fail(BCMG_ERR_INVALID, "bad precision");
    if (o->dtau_mode < 0 || o->dtau_mode > 2) return fail(BCMG_ERR_INVALID, "bad dtau_mode");
    if (o->dtau_mode == BCMG_DTAU_CONST && !(o->dtau_const > 0.0 && std::isfinite(o->dtau_const)))
        return fail(BCMG_ERR_INVALID, "dtau_const must be positive");
    if (o->ext_iters < 1 || o->ext_iters > 8) return fail(BCMG_ERR_INVALID, "ext_iters must be in 1..8");
    if (o->restrict_mode != 0 && o->restrict_mode != 1) return fail(BCMG_ERR_INVALID, "bad restrict_mode");
    if (o->seg_len != 64 && o->seg_len != 128) return fail(BCMG_ERR_INVALID, "seg_len must be 64 or 128");
    if (o->bc != BCMG_BC_DIRICHLET && o->bc != BCMG_BC_NEUMANN) return fail(BCMG_ERR_INVALID, "bad bc");
    if (!(o->reaction >= 0.0 && std::isfinite(o->reaction))) return fail(BCMG_ERR_INVALID, "reaction must be >= 0");
    if (o->layout != BCMG_LAYOUT_NATURAL && o->layout != BCMG_LAYOUT_SPLIT) return fail(BCMG_ERR_INVALID, "bad layout");
    if (o->cycle != BCMG_CYCLE_V && o->cycle != BCMG_CYCLE_W) return fail(BCMG_ERR_INVALID, "bad cycle");
    if (o->smoother != BCMG_SMOOTH_RB && o->smoother != BCMG_SMOOTH_JACOBI) return fail(BCMG_ERR_INVALID, "bad smoother");
    if (o->check_interval < 1 || o->check_interval > kMaxCheckInterval)
        return fail(BCMG_ERR_INVALID, "check_interval must be in 1..%d", kMaxCheckInterval);
    return BCMG_OK;
}

bcmg_status bcmg_estimate_bytes(int32_t dim, int32_t N, int32_t precision, int64_t *bytes) {
    if (!bytes || dim < 1 || dim > 3 || N < 4) return fail(BCMG_ERR_INVALID, "bad arguments");
    double tot = 0.0;
    const double esz = precision == BCMG_MIXED ? 4.0 : 8.0;
    for (int NN = N; NN >= 2; NN /= 2) {
        double nn = std::pow(NN + 1.0, dim);
        // phi, class, u, rhs, r, band mark scratch; ghosts/band ~ surface terms
        tot += nn * (8.0 + 1.0 + 3.0 * esz) + 64.0 * std::pow(NN + 1.0, dim - 1) * 8.0;
        if (NN == N) tot += nn * 16.0;  // FP64 rhs + residual on the finest level
    }
    // arrays of up to a quarter chunk share 4 MiB arena chunks, and a chunk is
    // only left when the next array does not fit, so each chunk is at least
    // 3/4 used: held bytes <= 4/3 of the array bytes plus one open chunk
    *bytes = (int64_t)(tot * 1.1 * 4.0 / 3.0) + (int64_t)kArenaChunk;
    return BCMG_OK;
}

bcmg_status bcmg_set_allocator(bcmg_alloc_fn alloc, bcmg_free_fn free, void *ctx) {
    if ((alloc == nullptr) != (free == nullptr)) return fail(BCMG_ERR_INVALID, "give both callbacks or neither");
    mem_set_source(alloc, free, ctx);
    return BCMG_OK;
}

bcmg_status bcmg_setup(int32_t dim, int32_t N, const double *phi_dev, const bcmg_options *opt, void *stream,
                       bcmg_problem **out) {
    if (!out) return fail(BCMG_ERR_INVALID, "null output handle");
    *out = nullptr;
    if (!phi_dev) return fail(BCMG_ERR_INVALID, "null phi");
    bcmg_options o;
    if (opt)
        o = *opt;
    else
        bcmg_default_options(&o);
    bcmg_status st = check_options(dim, N, &o);
    if (st) return st;
    const TraceRange tr("bcmg_setup %dD N=%d", dim, N);
    bcmg_problem *P = new bcmg_problem();
    P->d = dim;
    P->N = N;
    P->opt = o;
    P->stream = (hipStream_t)stream;
    P->mem = mem_current();
    P->device = P->mem.device;
    MemScope mem_scope(P->mem);  // setup temporaries come from the same source
    if ((st = noalloc_scratch_init(P->device))) {
        delete P;
        return st;
    }
    PhaseTimer timer(P->stream);
    t_phase = &timer;
    struct ClearPhase {
        ~ClearPhase() { t_phase = nullptr; }
    } clear_phase;
    P->fp32 = o.precision == BCMG_MIXED;
    int L = 0;
    for (int NN = N; NN >= o.coarsest_N; NN /= 2) L++;
    if (L > kMaxLevels) {
        delete P;
        return fail(BCMG_ERR_INVALID, "too many levels");
    }
    P->L = L;
    auto bail = [&](bcmg_status s) {
        hipStreamSynchronize(P->stream);
        free_problem_memory(P);
        delete P;
        return s;
    };
    for (int l = 0; l < L; l++) {
        LevelH &V = P->lev[l];
        V.N = N >> l;
        V.n = V.N + 1;
        V.nn = 1;
        for (int k = 0; k < dim; k++) V.nn *= V.n;
        V.h = 2.0 / V.N;
        if ((st = dalloc_t(P, &V.phi, V.nn)) || (st = dalloc_t(P, &V.cls, V.nn))) return bail(st);
    }
    int *flag = nullptr;
    if ((st = dalloc_t(P, &flag, 4))) return bail(st);
    launch_check_finite(phi_dev, P->lev[0].nn, flag, P->stream);
    int hflag = 0;
    if (hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, P->stream) != hipSuccess ||
        hipStreamSynchronize(P->stream) != hipSuccess)
        return bail(fail(BCMG_ERR_DEVICE, "phi check failed: %s", hipGetErrorString(hipGetLastError())));
    if (hflag) return bail(fail(BCMG_ERR_INVALID, "phi has non-finite values"));
    if (hipMemcpyAsync(P->lev[0].phi, phi_dev, sizeof(double) * P->lev[0].nn, hipMemcpyDeviceToDevice, P->stream) !=
        hipSuccess)
        return bail(fail(BCMG_ERR_DEVICE, "copy of phi failed"));
    for (int l = 1; l < L; l++) launch_inject(dim, P->lev[l - 1].phi, P->lev[l - 1].n, P->lev[l].phi, P->lev[l].n, P->stream);
    const int nblk = compact_blocks(P->lev[0].nn);
    int *counts = nullptr, *offsets = nullptr;
    if ((st = dalloc_t(P, &counts, nblk)) || (st = dalloc_t(P, &offsets, nblk))) return bail(st);
    int *h_total = nullptr;
    if (hipHostMalloc((void **)&h_total, sizeof(int)) != hipSuccess) return bail(fail(BCMG_ERR_OOM, "pinned alloc"));
    for (int l = 0; l < L; l++) {
        if ((st = setup_level(P, l, counts, offsets, flag, h_total))) {
            hipHostFree(h_total);
            return bail(st);
        }
    }
    PHASE("levels", -1);
    for (int l = 1; l < L; l++) {
        if ((st = build_restrict_rows(P, l, h_total)) ||
            (st = build_needed_band(P, l, counts, offsets, flag, h_total))) {
            hipHostFree(h_total);
            return bail(st);
        }
    }
    hipHostFree(h_total);
    PHASE("rows", -1);
    if ((st = setup_coarse(P))) return bail(st);
    PHASE("coarse", -1);
    if ((st = dalloc_t(P, &P->rhs64, P->lev[0].nn))) return bail(st);
    if (P->fp32) {
        if ((st = dalloc_t(P, &P->r64, P->lev[0].nn))) return bail(st);
    } else {
        P->r64 = (double *)P->lev[0].r;
        P->lev[0].rhs = P->rhs64;  // the FP64 cycle reads the finest rhs directly
    }
    if ((st = setup_step_tables(P))) return bail(st);
    PHASE("tables", -1);
    hipError_t e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return bail(fail(BCMG_ERR_DEVICE, "setup: %s", hipGetErrorString(e)));
    *out = P;
    return BCMG_OK;
}

bcmg_status bcmg_batch_destroy(bcmg_batch *b);

bcmg_status bcmg_destroy(bcmg_problem *P) {
    if (!P) return BCMG_OK;
    if (P->solo) bcmg_batch_destroy(P->solo);
    // the frees are ordered after the work queued on the problem's stream;
    // the host does not wait (a serving loop retires problems while other
    // problems are being set up on that stream)
    free_problem_memory(P);
    delete P;
    return BCMG_OK;
}

bcmg_status bcmg_num_levels(const bcmg_problem *P, int32_t *levels) {
    if (!P || !levels) return fail(BCMG_ERR_INVALID, "null argument");
    *levels = P->L;
    return BCMG_OK;
}

bcmg_status bcmg_level_info(const bcmg_problem *P, int32_t l, int32_t *N, int64_t *ni, int64_t *ng, int64_t *nb,
                            int64_t *nseg) {
    if (!valid_level(P, l)) return fail(BCMG_ERR_INVALID, "bad problem or level");
    const LevelH &V = P->lev[l];
    if (N) *N = V.N;
    if (ni) *ni = V.ni;
    if (ng) *ng = V.ng;
    if (nb) *nb = V.nb;
    if (nseg) *nseg = (int64_t)V.segs.size();
    return BCMG_OK;
}

bcmg_status bcmg_problem_bytes(const bcmg_problem *P, int64_t *bytes) {
    if (!P || !bytes) return fail(BCMG_ERR_INVALID, "null argument");
    *bytes = P->bytes;
    return BCMG_OK;
}

bcmg_status bcmg_classes(const bcmg_problem *P, int32_t l, uint8_t *cls_dev) {
    if (!valid_level(P, l) || !cls_dev) return fail(BCMG_ERR_INVALID, "bad argument");
    HIPCHK(hipMemcpyAsync(cls_dev, P->lev[l].cls, (size_t)P->lev[l].nn, hipMemcpyDeviceToDevice, P->stream));
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bcmg_status bcmg_ghost_info(const bcmg_problem *P, int32_t l, int32_t *idx, int32_t *code, double *eta, double *nrm,
                            double *q, double *tau, double *dtau, int32_t *fb) {
    if (!valid_level(P, l)) return fail(BCMG_ERR_INVALID, "bad problem or level");
    const LevelH &V = P->lev[l];
    const size_t ng = (size_t)V.ng;
    if (ng == 0) return BCMG_OK;
    hipStream_t s = P->stream;
    if (idx) HIPCHK(hipMemcpyAsync(idx, V.gidx, ng * 4, hipMemcpyDeviceToDevice, s));
    if (code) HIPCHK(hipMemcpyAsync(code, V.gcode, ng * 4, hipMemcpyDeviceToDevice, s));
    if (eta) HIPCHK(hipMemcpyAsync(eta, V.geta, ng * 8, hipMemcpyDeviceToDevice, s));
    if (nrm) HIPCHK(hipMemcpyAsync(nrm, V.gn, ng * 24, hipMemcpyDeviceToDevice, s));
    if (q) HIPCHK(hipMemcpyAsync(q, V.gq, ng * 24, hipMemcpyDeviceToDevice, s));
    if (tau) HIPCHK(hipMemcpyAsync(tau, V.gtau, ng * 24, hipMemcpyDeviceToDevice, s));
    if (dtau) HIPCHK(hipMemcpyAsync(dtau, V.gdtau, ng * 8, hipMemcpyDeviceToDevice, s));
    if (fb) HIPCHK(hipMemcpyAsync(fb, V.gfb, ng * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return BCMG_OK;
}

bcmg_status bcmg_ghost_stats(const bcmg_problem *P, int32_t l, int64_t *counts, int64_t *root_fallback,
                             int64_t *row_fallback) {
    if (!valid_level(P, l)) return fail(BCMG_ERR_INVALID, "bad problem or level");
    const LevelH &V = P->lev[l];
    const size_t ng = (size_t)V.ng;
    std::vector<int32_t> code(ng), fb(ng);
    if (ng) {
        HIPCHK(hipMemcpyAsync(code.data(), V.gcode, ng * 4, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipMemcpyAsync(fb.data(), V.gfb, ng * 4, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
    }
    int64_t c[27] = {0}, nroot = 0, nrow = 0;
    for (size_t g = 0; g < ng; g++) {
        int w[3] = {1, 1, 1};
        for (int k = 0; k < P->d; k++) w[k] = code_w(code[g], k);
        std::sort(w, w + 3, [](int a, int b) { return a > b; });
        c[(3 - w[0]) * 9 + (3 - w[1]) * 3 + (3 - w[2])]++;
        nroot += fb[g] & 1;
        nrow += (fb[g] >> 1) & 1;
    }
    if (counts) std::copy(c, c + 27, counts);
    if (root_fallback) *root_fallback = nroot;
    if (row_fallback) *row_fallback = nrow;
    return BCMG_OK;
}

bcmg_status bcmg_set_data(bcmg_problem *P, const double *f, const double *gq) {
    if (!P) return fail(BCMG_ERR_INVALID, "null problem");
    if (!gq && P->lev[0].ng > 0) return fail(BCMG_ERR_INVALID, "null ghost data");
    launch_set_rhs(P->lev[0].nn, P->lev[0].cls, f, P->rhs64, P->stream);
    launch_scatter_ghosts(P->lev[0].gidx, (int)P->lev[0].ng, gq, P->rhs64, P->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bcmg_status bcmg_fill_boundary(bcmg_problem *P, const double *gbox, double *u) {
    if (!P || !u) return fail(BCMG_ERR_INVALID, "null argument");
    launch_fill_boundary(P->lev[0].nn, P->lev[0].cls, gbox, u, P->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

// ---------------------------------------------------------------- steps
static bcmg_status check_fp64_step(const bcmg_problem *P, int l) {
    if (!valid_level(P, l)) return fail(BCMG_ERR_INVALID, "bad problem or level");
    if (P->fp32) return fail(BCMG_ERR_STATE, "single-step calls need an FP64 problem");
    return BCMG_OK;
}

bcmg_status bcmg_level_smooth(bcmg_problem *P, int32_t l, double *u, const double *rhs, int32_t steps) {
    bcmg_status st = check_fp64_step(P, l);
    if (st) return st;
    if (!u || !rhs || steps < 0) return fail(BCMG_ERR_INVALID, "bad argument");
    void *pu[1] = {u}, *pr[1] = {(void *)rhs}, *px[1] = {P->lev[l].r};
    if ((st = upload_step_descs(P, l, 1, pu, pr, px))) return st;
    const Item *segs = P->d_stepitems + P->off_seg[l], *gch = P->d_stepitems + P->off_gch[l];
    for (int i = 0; i < steps; i++) {
        launch_rb_sweep(P->d, 0, P->d_step, segs, P->n_seg[l], 0, P->d_stepst, P->stream);
        launch_rb_sweep(P->d, 0, P->d_step, segs, P->n_seg[l], 1, P->d_stepst, P->stream);
        launch_ghost_relax(P->d, 0, P->d_step, gch, P->n_gch[l], P->d_stepst, P->stream, nullptr, 0,
                           P->opt.bc == BCMG_BC_NEUMANN);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bcmg_status bcmg_level_residual(bcmg_problem *P, int32_t l, const double *u, const double *rhs, double *r,
                                double *norm_host) {
    bcmg_status st = check_fp64_step(P, l);
    if (st) return st;
    if (!u || !rhs || !r) return fail(BCMG_ERR_INVALID, "null argument");
    void *pu[1] = {(void *)u}, *pr[1] = {(void *)rhs}, *px[1] = {r};
    if ((st = upload_step_descs(P, l, 1, pu, pr, px))) return st;
    const Item *segs = P->d_stepitems + P->off_seg[l], *gch = P->d_stepitems + P->off_gch[l];
    const size_t need = (size_t)P->n_seg[l] + P->n_gch[l] + 1;
    if (need > P->partials_cap) {
        if ((st = dalloc_t(P, &P->d_partials, need))) return st;
        P->partials_cap = need;
    }
    launch_residual(P->d, 0, 0, norm_host ? 1 : 0, P->d_step, segs, P->n_seg[l], gch, P->n_gch[l], P->d_stepst,
                    P->d_partials, P->stream, P->opt.bc == BCMG_BC_NEUMANN);
    if (norm_host) {
        NormRange R{0, P->n_seg[l], 0, P->n_gch[l]};
        HIPCHK(hipMemcpyAsync(P->d_range, &R, sizeof R, hipMemcpyHostToDevice, P->stream));
        launch_norm_finish(P->d_range, 1, P->d_partials, P->n_seg[l], P->d_stepst, nullptr, nullptr, 0, 2, P->d_out,
                           P->stream);
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, P->d_out, sizeof v, hipMemcpyDeviceToHost, P->stream));
        HIPCHK(hipStreamSynchronize(P->stream));
        *norm_host = std::sqrt(v);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bcmg_status bcmg_level_extend(bcmg_problem *P, int32_t l, double *v) {
    bcmg_status st = check_fp64_step(P, l);
    if (st) return st;
    if (!v) return fail(BCMG_ERR_INVALID, "null argument");
    void *pu[1] = {v}, *pr[1] = {P->lev[l].rhs}, *px[1] = {P->lev[l].r};
    if ((st = upload_step_descs(P, l, 1, pu, pr, px))) return st;
    launch_ext_gather(0, P->d_step, P->d_stepitems + P->off_bch[l], P->n_bch[l], 0, P->d_stepst, P->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bcmg_status bcmg_level_restrict(bcmg_problem *P, int32_t l, const double *rf, double *rc) {
    bcmg_status st = check_fp64_step(P, l);
    if (st) return st;
    if (l + 1 >= P->L || !rf || !rc) return fail(BCMG_ERR_INVALID, "bad argument");
    void *pu[2] = {P->lev[l].u ? P->lev[l].u : (void *)rf, P->lev[l + 1].u}, *pr[2] = {P->lev[l].rhs, rc},
         *px[2] = {(void *)rf, P->lev[l + 1].r};
    if ((st = upload_step_descs(P, l, 2, pu, pr, px))) return st;
    launch_restrict(P->d, 0, P->d_step, P->d_stepitems + P->off_seg[l + 1], P->n_seg[l + 1],
                    P->d_stepitems + P->off_gch[l + 1], P->n_gch[l + 1], P->d_stepst, P->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bcmg_status bcmg_level_prolong(bcmg_problem *P, int32_t l, double *ec, double *uf) {
    bcmg_status st = check_fp64_step(P, l);
    if (st) return st;
    if (l + 1 >= P->L || !ec || !uf) return fail(BCMG_ERR_INVALID, "bad argument");
    void *pu[2] = {uf, ec}, *pr[2] = {P->lev[l].rhs, P->lev[l + 1].rhs}, *px[2] = {P->lev[l].r, P->lev[l + 1].r};
    if ((st = upload_step_descs(P, l, 2, pu, pr, px))) return st;
    launch_ext_gather(0, P->d_step, P->d_stepitems + P->off_bch[l + 1], P->n_bch[l + 1], 0, P->d_stepst, P->stream);
    launch_prolong(P->d, 0, P->d_step, P->d_stepitems + P->off_seg[l], P->n_seg[l], P->d_stepst, P->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

bcmg_status bcmg_coarse_solve(bcmg_problem *P, double *u, const double *rhs) {
    const int l = P ? P->L - 1 : 0;
    bcmg_status st = check_fp64_step(P, l);
    if (st) return st;
    if (!u || !rhs) return fail(BCMG_ERR_INVALID, "null argument");
    void *pu[1] = {u}, *pr[1] = {(void *)rhs}, *px[1] = {P->lev[l].r};
    if ((st = upload_step_descs(P, l, 1, pu, pr, px))) return st;
    if (P->lev[l].singular) {
        const Item *segs = P->d_stepitems + P->off_seg[l], *gch = P->d_stepitems + P->off_gch[l];
        for (int i = 0; i < 50; i++) {
            launch_rb_sweep(P->d, 0, P->d_step, segs, P->n_seg[l], 0, P->d_stepst, P->stream);
            launch_rb_sweep(P->d, 0, P->d_step, segs, P->n_seg[l], 1, P->d_stepst, P->stream);
            launch_ghost_relax(P->d, 0, P->d_step, gch, P->n_gch[l], P->d_stepst, P->stream, nullptr, 0,
                           P->opt.bc == BCMG_BC_NEUMANN);
        }
    } else {
        launch_coarse(0, P->d_step, P->d_lvl, 1, P->d_stepst, P->stream);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(P->stream));
    return BCMG_OK;
}

// ---------------------------------------------------------------- batches
// device memory of a batch, ordered on its stream
static hipError_t balloc(bcmg_batch *b, void **p, size_t bytes) { return mem_alloc(b->mem, p, bytes, b->stream); }
static void bfree(bcmg_batch *b, void *p) { mem_free(b->mem, p, b->stream); }

bcmg_status bcmg_batch_create(int32_t capacity, void *stream, bcmg_batch **out) {
    if (!out || capacity < 1 || capacity > 65536) return fail(BCMG_ERR_INVALID, "bad capacity");
    *out = nullptr;
    bcmg_batch *b = new bcmg_batch();
    b->cap = capacity;
    b->user_stream = (hipStream_t)stream;
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(BCMG_ERR_DEVICE, "stream creation failed");
    }
    b->prob.assign(capacity, nullptr);
    b->u.assign(capacity, nullptr);
    b->rtol.assign(capacity, 0.0);
    b->hist_stride = 1001;
    b->mem = mem_current();
    hipError_t e = balloc(b, (void **)&b->d_state, sizeof(SlotState) * capacity);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_state, 0, sizeof(SlotState) * capacity, b->stream);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_state, sizeof(SlotState) * capacity);
    if (e == hipSuccess) e = balloc(b, (void **)&b->d_rtol2, sizeof(double) * capacity);
    if (e == hipSuccess) e = balloc(b, (void **)&b->d_hist, sizeof(double) * capacity * b->hist_stride);
    if (e == hipSuccess) e = balloc(b, (void **)&b->d_ranges, sizeof(NormRange) * capacity);
    if (e == hipSuccess) e = balloc(b, (void **)&b->d_outer, sizeof(Desc) * capacity);
    if (e == hipSuccess) e = balloc(b, (void **)&b->d_eptr, sizeof(float *) * capacity);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        bcmg_batch_destroy(b);
        return fail(BCMG_ERR_OOM, "batch allocation: %s", hipGetErrorString(e));
    }
    memset(b->h_state, 0, sizeof(SlotState) * capacity);
    b->lds_budget = kLdsBudget;
    *out = b;
    return BCMG_OK;
}

static void drop_graph(bcmg_batch *b) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_cycles = 0;
    for (int j = 0; j <= kMaxCheckInterval; j++) {
        if (b->bexec[j]) hipGraphExecDestroy(b->bexec[j]);
        if (b->bgraph[j]) hipGraphDestroy(b->bgraph[j]);
        b->bexec[j] = nullptr;
        b->bgraph[j] = nullptr;
    }
    for (auto &pr : b->tev) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
    }
    b->tev.clear();
}

bcmg_status bcmg_batch_destroy(bcmg_batch *b) {
    if (!b) return BCMG_OK;
    hipStreamSynchronize(b->stream);
    drop_graph(b);
    bfree(b, b->d_state);
    if (b->h_state) hipHostFree(b->h_state);
    bfree(b, b->d_rtol2);
    bfree(b, b->d_hist);
    bfree(b, b->d_ranges);
    bfree(b, b->d_desc);
    bfree(b, b->d_outer);
    bfree(b, b->d_eptr);
    bfree(b, b->d_items);
    bfree(b, b->d_coarse);
    bfree(b, b->d_progs);
    bfree(b, b->d_lprogs);
    bfree(b, b->d_limage);
    bfree(b, b->d_partials);
    bfree(b, b->d_norm_blk);
    bfree(b, b->d_norm_cnt);
    if (b->join) hipEventDestroy(b->join);
    if (b->stream) hipStreamDestroy(b->stream);
    delete b;
    return BCMG_OK;
}

// order the batch stream after the caller's stream
static bcmg_status batch_join(bcmg_batch *b) {
    HIPCHK(hipEventRecord(b->join, b->user_stream));
    HIPCHK(hipStreamWaitEvent(b->stream, b->join, 0));
    return BCMG_OK;
}

// Rebuild descriptor tables and work lists for the current slots.
// LDS layout of a problem's coarse levels 0..top (aligned, 0 = coarsest) for
// k_coarse_lds; returns the bytes needed.  The top level's residual stays in
// HBM (it is written and read once per cycle).
static size_t lds_plan(const bcmg_problem *P, int top, LdsProg *lp) {
    const size_t esz = P->fp32 ? 4 : 8;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 15) & ~size_t(15);
        return (int)o;
    };
    LdsLevel q[kMaxLevels];
    memset(q, 0, sizeof q);
    // the arrays fixed during a solve first (the image), then the others
    for (int a2 = 0; a2 <= top; a2++) {
        const LevelH &V = P->lev[P->L - 1 - a2];
        q[a2].nn = (int)V.nn;
        q[a2].ng = (int)V.ng;
        q[a2].nb = (int)V.nb;
        q[a2].ni = (int)V.ni;
        q[a2].nred = V.nred;
        q[a2].nbn = (int)V.nbn;
        q[a2].cls = take(V.nn);
        q[a2].gidx = take(4 * V.ng);
        q[a2].gcode = take(4 * V.ng);
        q[a2].gtau = take(24 * V.ng);
        q[a2].gdtau = take(8 * V.ng);
        q[a2].gnd = P->opt.bc == BCMG_BC_NEUMANN ? take(24 * V.ng) : -1;
        q[a2].ilist = take(4 * V.ni);
        q[a2].bneed = take(4 * V.nbn);
    }
    const size_t static_bytes = off;
    for (int a2 = 0; a2 <= top; a2++) {
        const LevelH &V = P->lev[P->L - 1 - a2];
        q[a2].u = take(V.nn * esz);
        q[a2].rhs = take(V.nn * esz);
        q[a2].r = a2 < top ? take(V.nn * esz) : -1;
        q[a2].gnew = take(8 * V.ng);
    }
    if (lp) {
        for (int a2 = 0; a2 <= top; a2++) lp->lev[a2] = q[a2];
        lp->static_words = (int)(static_bytes / 4);
    }
    return off;
}

static bcmg_status batch_rebuild(bcmg_batch *b) {
    HIPCHK(hipStreamSynchronize(b->stream));  // tables may be in use by queued work
    drop_graph(b);
    std::vector<Desc> descs;
    std::vector<Desc> outer(b->cap);
    std::vector<float *> eptr(b->cap, nullptr);
    std::vector<int> base(b->cap, -1);
    int A = 0;
    for (int s = 0; s < b->cap; s++) {
        bcmg_problem *P = b->prob[s];
        if (!P) continue;
        base[s] = (int)descs.size();
        for (int l = 0; l < P->L; l++) {
            void *u = l == 0 ? (P->fp32 ? P->lev[0].u : (void *)b->u[s]) : P->lev[l].u;
            descs.push_back(make_desc(P, l, u, P->lev[l].rhs, P->lev[l].r, s));
        }
        // outer (finest, FP64) descriptor: residual of u64 into rhs32 (mixed) or r64
        outer[s] = make_desc(P, 0, b->u[s], P->rhs64, P->fp32 ? P->lev[0].rhs : (void *)P->r64, s);
        eptr[s] = P->fp32 ? (float *)P->lev[0].u : nullptr;
        A = std::max(A, P->L);
    }
    b->A = A;
    // work lists
    std::vector<Item> items;
    struct Off {
        size_t seg, gch, bch, cseg, cbch, cgch, rseg;
        int nseg, ngch, nbch, ncseg, ncbch, ncgch, nrseg;
    };
    std::vector<Off> off(A);
    auto add_segs = [&](int desc, const LevelH &V) {
        for (Item it : V.segs) {
            it.x = desc;
            items.push_back(it);
        }
    };
    for (int a = 0; a < A; a++) {
        Off &o = off[a];
        o.seg = items.size();
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L > a) add_segs(base[s] + b->prob[s]->L - 1 - a, b->prob[s]->lev[b->prob[s]->L - 1 - a]);
        o.nseg = (int)(items.size() - o.seg);
        o.gch = items.size();
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L > a) {
                const int l = b->prob[s]->L - 1 - a;
                append_chunks(items, base[s] + l, b->prob[s]->lev[l].ng);
            }
        o.ngch = (int)(items.size() - o.gch);
        o.bch = items.size();
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L > a && a >= 1) {
                const int l = b->prob[s]->L - 1 - a;
                append_chunks(items, base[s] + l, b->prob[s]->lev[l].nb);
            }
        o.nbch = (int)(items.size() - o.bch);
        o.cseg = items.size();
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L > a && a >= 1) {
                const int l = b->prob[s]->L - 1 - a;
                add_segs(base[s] + l + 1, b->prob[s]->lev[l + 1]);
            }
        o.ncseg = (int)(items.size() - o.cseg);
        o.cbch = items.size();
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L > a && a >= 1) {
                const int l = b->prob[s]->L - 1 - a;
                append_chunks(items, base[s] + l + 1, b->prob[s]->lev[l + 1].nbn);
            }
        o.ncbch = (int)(items.size() - o.cbch);
        o.cgch = items.size();
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L > a && a >= 1) {
                const int l = b->prob[s]->L - 1 - a;
                append_chunks(items, base[s] + l + 1, b->prob[s]->lev[l + 1].ng);
            }
        o.ncgch = (int)(items.size() - o.cgch);
        o.rseg = items.size();
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L - 1 == a) add_segs(base[s], b->prob[s]->lev[0]);
        o.nrseg = (int)(items.size() - o.rseg);
    }
    // finest lists over the outer descriptors, with per-slot norm ranges
    std::vector<NormRange> ranges(b->cap, NormRange{0, 0, 0, 0});
    const size_t fseg0 = items.size();
    for (int s = 0; s < b->cap; s++) {
        if (!b->prob[s]) continue;
        ranges[s].seg_beg = (int)(items.size() - fseg0);
        add_segs(s, b->prob[s]->lev[0]);
        ranges[s].seg_end = (int)(items.size() - fseg0);
    }
    const int nfseg = (int)(items.size() - fseg0);
    const size_t fgch0 = items.size();
    for (int s = 0; s < b->cap; s++) {
        if (!b->prob[s]) continue;
        ranges[s].gch_beg = (int)(items.size() - fgch0);
        append_chunks(items, s, b->prob[s]->lev[0].ng);
        ranges[s].gch_end = (int)(items.size() - fgch0);
    }
    const int nfgch = (int)(items.size() - fgch0);
    std::vector<int> coarse;
    b->fine_inside = 0;
    b->neu = 0;
    for (int s = 0; s < b->cap; s++)
        if (b->prob[s] && b->prob[s]->opt.bc == BCMG_BC_NEUMANN) b->neu = 1;
    for (int s = 0; s < b->cap; s++)
        if (b->prob[s]) {
            coarse.push_back(base[s] + b->prob[s]->L - 1);
            if (b->prob[s]->L == A) b->fine_inside += b->prob[s]->lev[0].ni;
        }
    // aligned level a has N = 4 * 2^a on every problem: levels with at most
    // coarse_nodes nodes are cycled by one workgroup per problem
    int Ac = 0;
    for (int a2 = 0; a2 < kMaxLevels && !b->wcycle && !b->jacobi; a2++) {
        long long nn = 1;
        for (int k = 0; k < b->d; k++) nn *= (4LL << a2) + 1;
        if (nn > b->coarse_nodes) break;
        // the workgroup cycles natural-order arrays only
        bool split = false;
        for (int s = 0; s < b->cap; s++)
            if (b->prob[s] && b->prob[s]->L - 1 >= a2 && b->prob[s]->lev[b->prob[s]->L - 1 - a2].half) split = true;
        if (split) break;
        Ac = a2;
    }
    // with LDS enabled, lower the threshold until every problem's coarse
    // levels fit in the budget
    if (b->lds_budget > 0) {
        while (Ac > 0) {
            size_t need = 0;
            bool lists = true;
            for (int s = 0; s < b->cap; s++) {
                const bcmg_problem *Q = b->prob[s];
                if (!Q) continue;
                const int top = std::min(Ac, Q->L - 1);
                need = std::max(need, lds_plan(Q, top, nullptr));
                lists = lists && Q->lev[Q->L - 1 - top].ilist != nullptr;
            }
            if (need <= b->lds_budget && lists) break;
            Ac--;
        }
    }
    b->Ac = Ac;
    std::vector<CoarseProg> progs;
    for (int s = 0; s < b->cap; s++) {
        bcmg_problem *P = b->prob[s];
        if (!P) continue;
        CoarseProg cp;
        memset(&cp, 0, sizeof cp);
        cp.slot = s;
        cp.top = std::min(Ac, P->L - 1);
        cp.ext_top = cp.top < P->L - 1 ? 1 : 0;
        for (int a2 = 0; a2 <= cp.top; a2++) {
            const int l = P->L - 1 - a2;
            const LevelH &V = P->lev[l];
            CoarseLevel &cl = cp.lev[a2];
            cl.desc = base[s] + l;
            cl.seg = (int)items.size();
            add_segs(cl.desc, V);
            cl.nseg = (int)items.size() - cl.seg;
            cl.gch = (int)items.size();
            append_chunks(items, cl.desc, V.ng);
            cl.ngch = (int)items.size() - cl.gch;
            cl.bch = (int)items.size();
            append_chunks(items, cl.desc, V.nb);
            cl.nbch = (int)items.size() - cl.bch;
        }
        progs.push_back(cp);
    }
    // the same programs with their levels staged in LDS, when the LDS path is
    // on, every level has its colour-sorted INSIDE list (levels of at most
    // kListNodes nodes) and they all fit; otherwise no program or image is
    // built (the HBM workgroup needs neither)
    std::vector<LdsProg> lprogs;
    size_t lds_max = 0;
    bool lists = true;
    for (const CoarseProg &cp : progs) {
        const bcmg_problem *P = b->prob[cp.slot];
        for (int a2 = 0; a2 <= cp.top; a2++) lists = lists && P->lev[P->L - 1 - a2].ilist != nullptr;
    }
    if (b->lds_budget > 0 && lists) {
        for (const CoarseProg &cp : progs) {
            const bcmg_problem *P = b->prob[cp.slot];
            LdsProg lp;
            memset(&lp, 0, sizeof lp);
            lp.slot = cp.slot;
            lp.top = cp.top;
            lp.ext_top = cp.ext_top;
            lp.finest = cp.top == P->L - 1 ? 1 : 0;
            lds_max = std::max(lds_max, lds_plan(P, cp.top, &lp));
            for (int a2 = 0; a2 <= cp.top; a2++) lp.lev[a2].desc = cp.lev[a2].desc;
            lprogs.push_back(lp);
        }
    }
    b->lds_bytes = !lprogs.empty() && lds_max <= b->lds_budget ? std::max<size_t>(lds_max, 16) : 0;
    if (!b->lds_bytes) lprogs.clear();
    size_t image_words = 0;
    for (const LdsProg &lp : lprogs) image_words += (size_t)lp.static_words;
    // upload
    hipStream_t st = b->stream;
    if (descs.size() > b->desc_cap) {
        bfree(b, b->d_desc);
        b->desc_cap = std::max<size_t>(descs.size(), 2 * b->desc_cap);
        HIPCHK(balloc(b, (void **)&b->d_desc, sizeof(Desc) * b->desc_cap));
    }
    if (items.size() + 1 > b->items_cap) {
        bfree(b, b->d_items);
        b->items_cap = std::max<size_t>(items.size() + 1, 2 * b->items_cap);
        HIPCHK(balloc(b, (void **)&b->d_items, sizeof(Item) * b->items_cap));
    }
    bfree(b, b->d_coarse);
    HIPCHK(balloc(b, (void **)&b->d_coarse, sizeof(int) * (coarse.size() + 1)));
    bfree(b, b->d_progs);
    HIPCHK(balloc(b, (void **)&b->d_progs, sizeof(CoarseProg) * (progs.size() + 1)));
    bfree(b, b->d_lprogs);
    HIPCHK(balloc(b, (void **)&b->d_lprogs, sizeof(LdsProg) * (lprogs.size() + 1)));
    if (image_words + 1 > b->limage_cap) {
        bfree(b, b->d_limage);
        b->limage_cap = std::max(image_words + 1, 2 * b->limage_cap);
        HIPCHK(balloc(b, (void **)&b->d_limage, sizeof(uint32_t) * b->limage_cap));
    }
    {
        size_t w = 0;
        for (LdsProg &lp : lprogs) {
            lp.image = b->d_limage + w;
            w += (size_t)lp.static_words;
        }
    }
    const size_t np = (size_t)nfseg + nfgch + 1;
    if (np > b->partials_cap) {
        bfree(b, b->d_partials);
        b->partials_cap = std::max(np, 2 * b->partials_cap);
        HIPCHK(balloc(b, (void **)&b->d_partials, sizeof(double) * b->partials_cap));
    }
    {
        // one workgroup per slot sums up to kNormBlockEntries partials; a
        // slot with more gets more workgroups (all slots the same number)
        int most = 0;
        for (const NormRange &R : ranges) most = std::max(most, (R.seg_end - R.seg_beg) + (R.gch_end - R.gch_beg));
        b->norm_blocks = std::min(kNormBlocksMax, std::max(1, most / kNormBlockEntries));
        const size_t need = (size_t)b->cap * (size_t)b->norm_blocks;
        if (b->norm_blocks > 1 && need > b->norm_cap) {
            bfree(b, b->d_norm_blk);
            bfree(b, b->d_norm_cnt);
            b->d_norm_blk = nullptr;
            b->d_norm_cnt = nullptr;
            b->norm_cap = 0;
            HIPCHK(balloc(b, (void **)&b->d_norm_blk, sizeof(double) * need));
            HIPCHK(balloc(b, (void **)&b->d_norm_cnt, sizeof(int) * (size_t)b->cap));
            HIPCHK(hipMemsetAsync(b->d_norm_cnt, 0, sizeof(int) * (size_t)b->cap, b->stream));
            b->norm_cap = need;
        }
    }
    hipStream_t cs = b->stream;
    if (!descs.empty())
        HIPCHK(hipMemcpyAsync(b->d_desc, descs.data(), sizeof(Desc) * descs.size(), hipMemcpyHostToDevice, cs));
    if (!items.empty())
        HIPCHK(hipMemcpyAsync(b->d_items, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice, cs));
    if (!coarse.empty())
        HIPCHK(hipMemcpyAsync(b->d_coarse, coarse.data(), sizeof(int) * coarse.size(), hipMemcpyHostToDevice, cs));
    HIPCHK(hipMemcpyAsync(b->d_outer, outer.data(), sizeof(Desc) * b->cap, hipMemcpyHostToDevice, cs));
    b->desc_base = base;
    HIPCHK(hipMemcpyAsync(b->d_eptr, eptr.data(), sizeof(float *) * b->cap, hipMemcpyHostToDevice, cs));
    HIPCHK(hipMemcpyAsync(b->d_ranges, ranges.data(), sizeof(NormRange) * b->cap, hipMemcpyHostToDevice, cs));
    if (!progs.empty())
        HIPCHK(hipMemcpyAsync(b->d_progs, progs.data(), sizeof(CoarseProg) * progs.size(), hipMemcpyHostToDevice, cs));
    if (!lprogs.empty()) {
        HIPCHK(hipMemcpyAsync(b->d_lprogs, lprogs.data(), sizeof(LdsProg) * lprogs.size(), hipMemcpyHostToDevice, cs));
        launch_lds_images(b->d_desc, b->d_lprogs, (int)lprogs.size(), cs);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipStreamSynchronize(cs));
    b->lv.assign(A, Lists());
    for (int a = 0; a < A; a++) {
        const Off &o = off[a];
        Lists &L = b->lv[a];
        L.segs = b->d_items + o.seg;
        L.nseg = o.nseg;
        L.gch = b->d_items + o.gch;
        L.ngch = o.ngch;
        L.bch = b->d_items + o.bch;
        L.nbch = o.nbch;
        L.csegs = b->d_items + o.cseg;
        L.ncseg = o.ncseg;
        L.cbch = b->d_items + o.cbch;
        L.ncbch = o.ncbch;
        L.cgch = b->d_items + o.cgch;
        L.ncgch = o.ncgch;
        L.rsegs = b->d_items + o.rseg;
        L.nrseg = o.nrseg;
        bool any = false, all = true;
        for (int s2 = 0; s2 < b->cap; s2++) {
            const bcmg_problem *Q = b->prob[s2];
            if (!Q || Q->L <= a) continue;
            any = true;
            all = all && Q->lev[Q->L - 1 - a].half != 0;
        }
        L.split = any && all;
    }
    b->fsegs = b->d_items + fseg0;
    b->nfseg = nfseg;
    b->fgch = b->d_items + fgch0;
    b->nfgch = nfgch;
    b->ncoarse = (int)coarse.size();
    b->nprog = (int)progs.size();
    b->dirty = false;
    return BCMG_OK;
}

static void timed_sweep(bcmg_batch *b, int a, int colour, bool first = false) {
    const Lists &L = b->lv[a];
    const bool fine = g_timing.on && a == b->A - 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (fine) {
        hipEventCreate(&e0);
        hipEventCreate(&e1);
        hipEventRecord(e0, b->stream);
    }
    launch_rb_sweep(b->d, b->fp32, b->d_desc, first ? L.rsegs : L.segs, first ? L.nrseg : L.nseg, colour, b->d_state,
                    b->stream, L.split ? b->pair_segs : INT32_MAX);
    if (fine) {
        hipEventRecord(e1, b->stream);
        b->tev.push_back({e0, e1});
    }
}

// one smoothing step on aligned level a; ext: band chunks to extend into
// after the ghost step (the level's error before its prolongation)
// first: the first step of the pre-smoothing (its red half-sweep covers the
// problems whose finest level this is only)
static void smooth(bcmg_batch *b, int a, const Item *ext = nullptr, int next = 0, bool first = false) {
    const Lists &L = b->lv[a];
    if (b->jacobi) {
        launch_jacobi(b->d, b->fp32, b->d_desc, L.segs, L.nseg, b->d_state, b->stream);
    } else {
        timed_sweep(b, a, 0, first);
        timed_sweep(b, a, 1);
    }
    launch_ghost_relax(b->d, b->fp32, b->d_desc, L.gch, L.ngch, b->d_state, b->stream, ext, next, b->neu);
}

// one V(nu1, nu2) cycle over every slot, levels aligned at the coarsest grid.
// The extension of a level's error into its band (read by the prolongation
// to the next finer level) rides on the last ghost step of its post-smoothing;
// the aligned levels 0..Ac are cycled inside k_coarse_cycle, which extends
// its top level itself.
static void launch_vcycle(bcmg_batch *b) {
    const int d = b->d, f = b->fp32;
    hipStream_t s = b->stream;
    for (int a = b->A - 1; a > b->Ac; a--) {
        const Lists &L = b->lv[a];
        if (L.nseg == 0 && L.ngch == 0) continue;
        for (int i = 0; i < b->nu1; i++) smooth(b, a, nullptr, 0, i == 0);
        launch_residual(d, f, f, 0, b->d_desc, L.segs, L.nseg, L.gch, L.ngch, b->d_state, nullptr, s, b->neu, 1,
                        L.split ? 1 : 0);
        // a coarse level cycled by launches gets its first red half-sweep here
        launch_restrict(d, f, b->d_desc, L.csegs, L.ncseg, L.cgch, L.ncgch, b->d_state, s,
                        !b->jacobi && b->nu1 > 0 && a - 1 > b->Ac);
    }
    if (b->lds_bytes)
        launch_coarse_lds(d, f, b->d_desc, b->d_lprogs, b->nprog, b->lds_bytes, b->d_state, b->nu1, b->nu2, s,
                          b->neu);
    else
        launch_coarse_cycle(d, f, b->d_desc, b->d_items, b->d_progs, b->nprog, b->d_state, b->nu1, b->nu2, s,
                            b->neu);
    for (int a = b->Ac + 1; a < b->A; a++) {
        const Lists &L = b->lv[a];
        if (L.nseg == 0 && L.ngch == 0) continue;
        launch_prolong(d, f, b->d_desc, L.segs, L.nseg, b->d_state, s);
        const Lists *U = a + 1 < b->A ? &b->lv[a + 1] : nullptr;  // extension for the next prolongation
        for (int i = 0; i < b->nu2; i++) {
            const bool last = i == b->nu2 - 1;
            smooth(b, a, last && U ? U->cbch : nullptr, last && U ? U->ncbch : 0);
        }
        if (b->nu2 == 0 && U) launch_ext_gather(f, b->d_desc, U->cbch, U->ncbch, 1, b->d_state, s);
    }
}

// One W-cycle visit of aligned level a > Ac (Sec. 2.1: the two-grid step
// applied recursively, gamma = 2 on every coarse level but the one above the
// coarsest).  restricted: the level's correction starts from zero and the
// restriction into it has done its first red half-sweep (the first visit;
// the second starts from the first one's result, so its red half-sweep runs
// in full).
static void wcycle_level(bcmg_batch *b, int a, bool restricted) {
    const int d = b->d, f = b->fp32;
    hipStream_t s = b->stream;
    const Lists &L = b->lv[a];
    const bool work = L.nseg > 0 || L.ngch > 0;
    if (work) {
        for (int i = 0; i < b->nu1; i++) smooth(b, a, nullptr, 0, restricted && i == 0);
        launch_residual(d, f, f, 0, b->d_desc, L.segs, L.nseg, L.gch, L.ngch, b->d_state, nullptr, s, b->neu, 1,
                        L.split ? 1 : 0);
        launch_restrict(d, f, b->d_desc, L.csegs, L.ncseg, L.cgch, L.ncgch, b->d_state, s,
                        !b->jacobi && b->nu1 > 0 && a - 1 > b->Ac);
    }
    if (a - 1 == b->Ac) {
        if (b->lds_bytes)
            launch_coarse_lds(d, f, b->d_desc, b->d_lprogs, b->nprog, b->lds_bytes, b->d_state, b->nu1, b->nu2, s,
                              b->neu);
        else
            launch_coarse_cycle(d, f, b->d_desc, b->d_items, b->d_progs, b->nprog, b->d_state, b->nu1, b->nu2, s,
                                b->neu);
    } else {
        for (int g = 0; g < 2; g++) wcycle_level(b, a - 1, g == 0);
    }
    if (!work) return;
    launch_prolong(d, f, b->d_desc, L.segs, L.nseg, b->d_state, s);
    const Lists *U = a + 1 < b->A ? &b->lv[a + 1] : nullptr;  // extension for the next prolongation
    for (int i = 0; i < b->nu2; i++) {
        const bool last = i == b->nu2 - 1;
        smooth(b, a, last && U ? U->cbch : nullptr, last && U ? U->ncbch : 0);
    }
    if (b->nu2 == 0 && U) launch_ext_gather(f, b->d_desc, U->cbch, U->ncbch, 1, b->d_state, s);
}

// finest FP64 residual (into the FP32 right-hand side of the correction
// cycle; an FP64 batch keeps only its norm, since the next cycle recomputes
// r before the restriction reads it) plus per-slot norm and convergence
// bookkeeping
static void launch_outer_residual(bcmg_batch *b, int mode, int ncyc = 1) {
    launch_residual(b->d, 0, b->fp32, 1, b->d_outer, b->fsegs, b->nfseg, b->fgch, b->nfgch, b->d_state, b->d_partials,
                    b->stream, b->neu, b->fp32 ? 1 : 0);
    launch_norm_finish(b->d_ranges, b->cap, b->d_partials, b->nfseg, b->d_state, b->d_rtol2, b->d_hist,
                       b->hist_stride, mode, nullptr, b->stream, ncyc, b->norm_blocks, b->d_norm_blk, b->d_norm_cnt);
}

// one multigrid cycle of the batch's shape on the correction equations
static void launch_mg_cycle(bcmg_batch *b) {
    if (b->wcycle && b->A - 1 > b->Ac)
        wcycle_level(b, b->A - 1, true);
    else
        launch_vcycle(b);
}

// ncyc cycles and one convergence check after them; in mixed precision the
// ncyc FP32 cycles iterate on one correction equation before the update
static void launch_cycle(bcmg_batch *b, int ncyc = 1) {
    for (int c = 0; c < ncyc; c++) launch_mg_cycle(b);
    if (b->fp32) launch_ir_update(b->d_outer, b->fsegs, b->nfseg, b->d_state, b->d_eptr, b->stream);
    launch_outer_residual(b, 1, ncyc);
}

static bcmg_status batch_init_slot(bcmg_batch *b, int slot, double rtol) {
    bcmg_problem *P = b->prob[slot];
    SlotState s0;
    memset(&s0, 0, sizeof s0);
    s0.active = 2;  // pending: norm_finish mode 0 initialises it
    s0.max_cycles = P->opt.max_cycles;
    double r2 = rtol * rtol;
    HIPCHK(hipMemcpyAsync(b->d_state + slot, &s0, sizeof s0, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->d_rtol2 + slot, &r2, sizeof r2, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    launch_outer_residual(b, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(b->stream));
    return BCMG_OK;
}

bcmg_status bcmg_batch_add(bcmg_batch *b, bcmg_problem *P, double *u, double rtol, int32_t *slot) {
    if (!b || !P || !u) return fail(BCMG_ERR_INVALID, "null argument");
    if (!(rtol >= 0.0)) return fail(BCMG_ERR_INVALID, "bad tolerance");
    int n_used = 0;
    for (int s = 0; s < b->cap; s++) n_used += b->prob[s] != nullptr;
    if (n_used > 0) {
        if (P->d != b->d || P->fp32 != b->fp32 || P->opt.nu1 != b->nu1 || P->opt.nu2 != b->nu2 ||
            P->opt.ext_iters != b->K || (P->opt.cycle == BCMG_CYCLE_W) != (b->wcycle != 0) ||
            (P->opt.smoother == BCMG_SMOOTH_JACOBI) != (b->jacobi != 0))
            return fail(BCMG_ERR_INVALID,
                        "problem does not match the batch (dim, precision, nu1, nu2, ext_iters, cycle, smoother)");
        if (b->wcycle)
            for (int s2 = 0; s2 < b->cap; s2++)
                if (b->prob[s2] && b->prob[s2]->L != P->L)
                    return fail(BCMG_ERR_INVALID, "W-cycle problems of a batch must have the same number of levels");
    } else {
        b->d = P->d;
        b->fp32 = P->fp32;
        b->nu1 = P->opt.nu1;
        b->nu2 = P->opt.nu2;
        b->K = P->opt.ext_iters;
        b->wcycle = P->opt.cycle == BCMG_CYCLE_W;
        b->jacobi = P->opt.smoother == BCMG_SMOOTH_JACOBI;
    }
    if (b->jacobi && P->lev[P->L - 1].singular)
        return fail(BCMG_ERR_INVALID, "weighted Jacobi needs a nonsingular coarsest level");
    int s = -1;
    for (int i = 0; i < b->cap; i++)
        if (!b->prob[i]) {
            s = i;
            break;
        }
    if (s < 0) return fail(BCMG_ERR_STATE, "batch full");
    if (bcmg_status jst = batch_join(b)) return jst;
    // FP32 correction must start at 0
    if (P->fp32) HIPCHK(hipMemsetAsync(P->lev[0].u, 0, P->lev[0].nn * 4, b->stream));
    b->prob[s] = P;
    b->u[s] = u;
    b->rtol[s] = rtol;
    b->dirty = true;
    bcmg_status st = batch_rebuild(b);
    if (st) {
        b->prob[s] = nullptr;
        b->u[s] = nullptr;
        return st;
    }
    if ((st = batch_init_slot(b, s, rtol))) return st;
    if (slot) *slot = s;
    return BCMG_OK;
}

bcmg_status bcmg_batch_restart(bcmg_batch *b) {
    if (!b) return fail(BCMG_ERR_INVALID, "null batch");
    bcmg_status st = batch_join(b);
    if (st) return st;
    if (b->dirty && (st = batch_rebuild(b))) return st;
    std::vector<SlotState> s0(b->cap);
    std::vector<double> r2(b->cap, 0.0);
    for (int s = 0; s < b->cap; s++) {
        memset(&s0[s], 0, sizeof(SlotState));
        if (!b->prob[s]) continue;
        s0[s].active = 2;
        s0[s].max_cycles = b->prob[s]->opt.max_cycles;
        r2[s] = b->rtol[s] * b->rtol[s];
        if (b->prob[s]->fp32)
            HIPCHK(hipMemsetAsync(b->prob[s]->lev[0].u, 0, b->prob[s]->lev[0].nn * 4, b->stream));
    }
    HIPCHK(hipMemcpyAsync(b->d_state, s0.data(), sizeof(SlotState) * b->cap, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->d_rtol2, r2.data(), sizeof(double) * b->cap, hipMemcpyHostToDevice, b->stream));
    launch_outer_residual(b, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(b->stream));
    return BCMG_OK;
}

bcmg_status bcmg_batch_set_param(bcmg_batch *b, int32_t param, int64_t value) {
    if (!b) return fail(BCMG_ERR_INVALID, "null batch");
    if (param == BCMG_PARAM_COARSE_NODES) {
        if (value < 0 || value > 100000000) return fail(BCMG_ERR_INVALID, "coarse_nodes out of range");
        HIPCHK(hipStreamSynchronize(b->stream));
        b->coarse_nodes = value;
        b->dirty = true;
        return BCMG_OK;
    }
    if (param == BCMG_PARAM_SWEEP_PAIR_SEGS) {
        if (value < 1 || value > INT32_MAX) return fail(BCMG_ERR_INVALID, "sweep pair threshold out of range");
        HIPCHK(hipStreamSynchronize(b->stream));
        b->pair_segs = (int)value;
        drop_graph(b);
        return BCMG_OK;
    }
    if (param == BCMG_PARAM_LDS_BYTES) {
        if (value < 0 || value > (int64_t)kLdsBudget)
            return fail(BCMG_ERR_INVALID, "lds budget out of range [0, %zu]", kLdsBudget);
        HIPCHK(hipStreamSynchronize(b->stream));
        b->lds_budget = (size_t)value;
        b->dirty = true;
        return BCMG_OK;
    }
    return fail(BCMG_ERR_INVALID, "unknown parameter %d", param);
}

bcmg_status bcmg_batch_remove(bcmg_batch *b, int32_t slot) {
    if (!b || slot < 0 || slot >= b->cap || !b->prob[slot]) return fail(BCMG_ERR_INVALID, "bad slot");
    HIPCHK(hipStreamSynchronize(b->stream));
    b->prob[slot] = nullptr;
    b->u[slot] = nullptr;
    SlotState z;
    memset(&z, 0, sizeof z);
    HIPCHK(hipMemcpyAsync(b->d_state + slot, &z, sizeof z, hipMemcpyHostToDevice, b->stream));
    b->dirty = true;
    return BCMG_OK;
}

static bcmg_status batch_launch_cycles(bcmg_batch *b, int cycles) {
    if (b->dirty) {
        bcmg_status st = batch_rebuild(b);
        if (st) return st;
    }
    if (g_timing.on) {
        for (int c = 0; c < cycles; c++) launch_cycle(b);
        HIPCHK(hipGetLastError());
        return BCMG_OK;
    }
    if (!b->exec || b->graph_cycles != cycles) {
        drop_graph(b);
        HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        for (int c = 0; c < cycles; c++) launch_cycle(b);
        hipError_t e = hipStreamEndCapture(b->stream, &b->graph);
        if (e != hipSuccess) return fail(BCMG_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
        HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_cycles = cycles;
    }
    HIPCHK(hipGraphLaunch(b->exec, b->stream));
    return BCMG_OK;
}

// ncyc cycles with one check after them (bcmg_solve's blocks); one graph per
// block length, captured on first use
static bcmg_status batch_launch_block(bcmg_batch *b, int ncyc) {
    if (ncyc <= 1) return batch_launch_cycles(b, 1);
    if (b->dirty) {
        bcmg_status st = batch_rebuild(b);
        if (st) return st;
    }
    if (g_timing.on) {
        launch_cycle(b, ncyc);
        HIPCHK(hipGetLastError());
        return BCMG_OK;
    }
    if (!b->bexec[ncyc]) {
        HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        launch_cycle(b, ncyc);
        hipError_t e = hipStreamEndCapture(b->stream, &b->bgraph[ncyc]);
        if (e != hipSuccess) return fail(BCMG_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
        HIPCHK(hipGraphInstantiate(&b->bexec[ncyc], b->bgraph[ncyc], nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(b->bexec[ncyc], b->stream));
    return BCMG_OK;
}

// after a synchronisation: add the timed launches to the process-wide counters
static void drain_timing(bcmg_batch *b) {
    if (b->tev.empty()) return;
    for (auto &pr : b->tev) {
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, pr.first, pr.second);
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
        if (e != hipSuccess) continue;
        g_timing.ms += ms;
        g_timing.launches++;
    }
    b->tev.clear();
    g_timing.nodes = b->fine_inside;
}

bcmg_status bcmg_batch_step(bcmg_batch *b, int32_t cycles, int32_t *active_host) {
    if (!b || cycles < 1) return fail(BCMG_ERR_INVALID, "bad argument");
    const TraceRange tr("bcmg_batch_step %d cycles", cycles);
    bcmg_status st = batch_join(b);
    if (st) return st;
    st = batch_launch_cycles(b, cycles);
    if (st) return st;
    HIPCHK(hipMemcpyAsync(b->h_state, b->d_state, sizeof(SlotState) * b->cap, hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    drain_timing(b);
    if (active_host)
        for (int s = 0; s < b->cap; s++) active_host[s] = b->prob[s] && b->h_state[s].active ? 1 : 0;
    return BCMG_OK;
}

bcmg_status bcmg_batch_run(bcmg_batch *b, int32_t cycles_per_step, int32_t max_steps) {
    if (!b || cycles_per_step < 1) return fail(BCMG_ERR_INVALID, "bad argument");
    for (int i = 0; i < max_steps; i++) {
        bcmg_status st = bcmg_batch_step(b, cycles_per_step, nullptr);
        if (st) return st;
        bool any = false;
        for (int s = 0; s < b->cap; s++) any |= b->prob[s] && b->h_state[s].active;
        if (!any) return BCMG_OK;
    }
    return BCMG_OK;
}

bcmg_status bcmg_batch_stats(bcmg_batch *b, int32_t slot, bcmg_solve_stats *stats, double *hist) {
    if (!b || slot < 0 || slot >= b->cap) return fail(BCMG_ERR_INVALID, "bad slot");
    HIPCHK(hipMemcpyAsync(b->h_state, b->d_state, sizeof(SlotState) * b->cap, hipMemcpyDeviceToHost, b->stream));
    std::vector<double> h(b->hist_stride);
    HIPCHK(hipMemcpyAsync(h.data(), b->d_hist + (size_t)slot * b->hist_stride, sizeof(double) * b->hist_stride,
                          hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    const SlotState &S = b->h_state[slot];
    const int c = std::min(S.cycles, b->hist_stride - 1);
    if (hist) std::copy(h.begin(), h.begin() + c + 1, hist);
    if (stats) {
        stats->cycles = S.cycles;
        stats->status = S.active ? BCMG_ERR_STATE : S.status;
        stats->r0 = std::sqrt(S.r0sq);
        stats->r_final = std::sqrt(S.lastsq);
        double rho = 0.0;
        if (c >= 16) {
            bool all = true;
            for (int m = 11; m <= 16; m++) all = all && !std::isnan(h[m]);
            if (all) {
                for (int m = 11; m <= 15; m++) rho += h[m + 1] / h[m];
                rho /= 5.0;
            } else {  // unchecked cycles: the per-cycle rate between the checks around the window
                int ma = 11, mb = 16;
                while (ma > 0 && std::isnan(h[ma])) ma--;
                while (mb < c && std::isnan(h[mb])) mb++;
                if (!std::isnan(h[ma]) && !std::isnan(h[mb]) && h[ma] > 0.0)
                    rho = std::pow(h[mb] / h[ma], 1.0 / (mb - ma));
            }
        }
        stats->rho_mean = rho;
        stats->solve_ms = 0.0;
    }
    return BCMG_OK;
}

// ------------------------------------------------------------ single solve
// Slot s solves into another caller array u: only the descriptors that name
// the caller's u change (the outer one, and an FP64 problem's finest level);
// the kernels read descriptors from device memory, so the work lists and
// captured graphs stay valid.  Queued work is ordered before the copies.
static bcmg_status batch_set_u(bcmg_batch *b, int s, double *u) {
    bcmg_problem *P = b->prob[s];
    b->u[s] = u;
    if (b->dirty) return BCMG_OK;  // the next rebuild takes b->u
    const Desc o = make_desc(P, 0, u, P->rhs64, P->fp32 ? P->lev[0].rhs : (void *)P->r64, s);
    HIPCHK(hipMemcpyAsync(b->d_outer + s, &o, sizeof o, hipMemcpyHostToDevice, b->stream));
    if (!P->fp32) {
        const Desc d0 = make_desc(P, 0, u, P->lev[0].rhs, P->lev[0].r, s);
        HIPCHK(hipMemcpyAsync(b->d_desc + b->desc_base[s], &d0, sizeof d0, hipMemcpyHostToDevice, b->stream));
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    return BCMG_OK;
}

static bcmg_status solo_attach(bcmg_problem *P, double *u, double rtol) {
    bcmg_status st;
    if (!P->solo) {
        if ((st = bcmg_batch_create(1, P->stream, &P->solo))) return st;
    }
    bcmg_batch *b = P->solo;
    if ((st = batch_join(b))) return st;
    if (b->prob[0] == P) {
        if (b->u[0] != u && (st = batch_set_u(b, 0, u))) return st;
        b->rtol[0] = rtol;
        if (P->fp32) HIPCHK(hipMemsetAsync(P->lev[0].u, 0, P->lev[0].nn * 4, b->stream));
        return batch_init_slot(b, 0, rtol);
    }
    if (b->prob[0]) bcmg_batch_remove(b, 0);
    int32_t slot = 0;
    return bcmg_batch_add(b, P, u, rtol, &slot);
}

bcmg_status bcmg_solve(bcmg_problem *P, double *u, double rtol, bcmg_solve_stats *stats, double *hist) {
    if (!P || !u) return fail(BCMG_ERR_INVALID, "null argument");
    if (!(rtol >= 0.0)) return fail(BCMG_ERR_INVALID, "bad tolerance");
    const TraceRange tr("bcmg_solve");
    bcmg_status st = solo_attach(P, u, rtol);
    if (st) return st;
    bcmg_batch *b = P->solo;
    struct Events {  // destroyed on every return path
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) hipEventDestroy(e0);
            if (e1) hipEventDestroy(e1);
        }
    } ev;
    HIPCHK(hipEventCreate(&ev.e0));
    HIPCHK(hipEventCreate(&ev.e1));
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    HIPCHK(hipEventRecord(e0, b->stream));
    b->h_state[0].active = 1;
    HIPCHK(hipMemcpyAsync(b->h_state, b->d_state, sizeof(SlotState), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    if ((st = batch_join(b))) return st;
    // The host waits on the device once per k cycles, with k the number of
    // cycles the observed convergence rate still needs (at least 1, at most
    // 16 or twice check_interval).  Cycles launched after convergence find the slot inactive and
    // change nothing.  Those k cycles run in blocks of up to check_interval
    // cycles with a device-side check after each block, as long as at least
    // two predicted cycles remain after the block; the rest are checked one
    // by one.
    const int J = P->opt.check_interval;
    int k = 1, tail = 1, checked_cycles = 0;
    double checked_sq = -1.0;
    while (b->h_state[0].active) {
        const TraceRange trk("cycles %d..%d", b->h_state[0].cycles + 1, b->h_state[0].cycles + k);
        int left = k;
        while (left > tail && J > 1) {
            const int j = std::min(J, left - tail);
            if ((st = batch_launch_block(b, j))) return st;
            left -= j;
        }
        for (int i = 0; i < left; i++)
            if ((st = batch_launch_cycles(b, 1))) return st;
        HIPCHK(hipMemcpyAsync(b->h_state, b->d_state, sizeof(SlotState), hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        drain_timing(b);
        const SlotState &S = b->h_state[0];
        k = 1;
        tail = 1;
        const int dc = S.cycles - checked_cycles;
        if (S.active && checked_sq > 0.0 && dc > 0 && S.lastsq > 0.0 && S.lastsq < checked_sq && S.tolsq > 0.0) {
            const double rate = std::log(S.lastsq / checked_sq) / dc;  // log of rho^2 per cycle, < 0
            const double need = std::log(S.tolsq / S.lastsq) / rate;   // cycles still needed
            const double nc = std::min(1e6, std::floor(need));
            if (need > 1.0) k = (int)std::min((double)std::max(16, 2 * J), nc);
            k = std::max(1, std::min(k, S.max_cycles - S.cycles));
            // the cycles predicted to be the last two are checked one by one
            tail = (int)std::max(0.0, 2.0 - (nc - k));
        }
        checked_cycles = S.cycles;
        checked_sq = S.lastsq;
    }
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    bcmg_solve_stats s;
    if ((st = bcmg_batch_stats(b, 0, &s, hist))) return st;
    s.solve_ms = ms;
    if (stats) *stats = s;
    return s.status;
}

bcmg_status bcmg_vcycle(bcmg_problem *P, double *u) {
    if (!P || !u) return fail(BCMG_ERR_INVALID, "null argument");
    bcmg_status st = solo_attach(P, u, 0.0);
    if (st) return st;
    bcmg_batch *b = P->solo;
    SlotState s1;
    memset(&s1, 0, sizeof s1);
    s1.active = 1;
    s1.max_cycles = 1 << 30;
    HIPCHK(hipMemcpyAsync(b->d_state, &s1, sizeof s1, hipMemcpyHostToDevice, b->stream));
    launch_mg_cycle(b);
    if (b->fp32) launch_ir_update(b->d_outer, b->fsegs, b->nfseg, b->d_state, b->d_eptr, b->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(b->stream));
    return BCMG_OK;
}

bcmg_status bcmg_residual_norm(bcmg_problem *P, const double *u, double *norm_host) {
    if (!P || !u || !norm_host) return fail(BCMG_ERR_INVALID, "null argument");
    void *pu[1] = {(void *)u}, *pr[1] = {P->rhs64}, *px[1] = {P->r64};
    bcmg_status st;
    if ((st = upload_step_descs(P, 0, 1, pu, pr, px))) return st;
    launch_residual(P->d, 0, 0, 1, P->d_step, P->d_stepitems + P->off_seg[0], P->n_seg[0],
                    P->d_stepitems + P->off_gch[0], P->n_gch[0], P->d_stepst, P->d_partials, P->stream,
                    P->opt.bc == BCMG_BC_NEUMANN);
    NormRange R{0, P->n_seg[0], 0, P->n_gch[0]};
    HIPCHK(hipMemcpyAsync(P->d_range, &R, sizeof R, hipMemcpyHostToDevice, P->stream));
    launch_norm_finish(P->d_range, 1, P->d_partials, P->n_seg[0], P->d_stepst, nullptr, nullptr, 0, 2, P->d_out,
                       P->stream);
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, P->d_out, sizeof v, hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipStreamSynchronize(P->stream));
    (void)st;
    *norm_host = std::sqrt(v);
    return BCMG_OK;
}

bcmg_status bcmg_residual_norm_noalloc(bcmg_problem *P, const double *u, double *norm_host) {
    if (!P || !u || !norm_host) return fail(BCMG_ERR_INVALID, "null argument");
    const long long need = (long long)P->n_seg[0] + P->n_gch[0] + 1;
    if (need > kNoAllocPartials)
        return fail(BCMG_ERR_INVALID,
                    "finest level has %lld row segments and ghost chunks; bcmg_residual_norm_noalloc holds at most %lld "
                    "(use bcmg_residual_norm)",
                    need - 1, kNoAllocPartials - 1);
    double *base = noalloc_scratch(P->device);
    if (!base) return fail(BCMG_ERR_STATE, "scratch address not set up on device %d", P->device);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != P->device) return fail(BCMG_ERR_STATE, "device %d is current, the problem lives on %d", dev, P->device);
    double *partials = base;
    NormRange *range = (NormRange *)(base + kNoAllocPartials);
    double *result = base + kNoAllocPartials + 2;
    // the descriptor goes to the problem's own step table, the range record to
    // the scratch, both from host stack memory (no staging buffer)
    const Desc D = make_desc(P, 0, (void *)u, P->rhs64, P->r64, 0);
    const NormRange R{0, P->n_seg[0], 0, P->n_gch[0]};
    HIPCHK(hipMemcpyAsync(P->d_step, &D, sizeof D, hipMemcpyHostToDevice, P->stream));
    HIPCHK(hipMemcpyAsync(range, &R, sizeof R, hipMemcpyHostToDevice, P->stream));
    launch_residual(P->d, 0, 0, 1, P->d_step, P->d_stepitems + P->off_seg[0], P->n_seg[0],
                    P->d_stepitems + P->off_gch[0], P->n_gch[0], P->d_stepst, partials, P->stream,
                    P->opt.bc == BCMG_BC_NEUMANN);
    launch_norm_finish(range, 1, partials, P->n_seg[0], P->d_stepst, nullptr, nullptr, 0, 2, result, P->stream);
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, result, sizeof v, hipMemcpyDeviceToHost, P->stream));
    HIPCHK(hipStreamSynchronize(P->stream));
    HIPCHK(hipGetLastError());
    *norm_host = std::sqrt(v);
    return BCMG_OK;
}

// ------------------------------------------------------------ timing
bcmg_status bcmg_timing_enable(int32_t on) {
    g_timing.on = on != 0;
    g_timing.launches = 0;
    g_timing.ms = 0.0;
    return BCMG_OK;
}

bcmg_status bcmg_timing_read(int64_t *launches, double *total_ms, int64_t *nodes) {
    if (launches) *launches = g_timing.launches;
    if (total_ms) *total_ms = g_timing.ms;
    if (nodes) *nodes = g_timing.nodes;
    return BCMG_OK;
}

bcmg_status bcmg_timing_sweeps(bcmg_problem *P, const double *u, int32_t reps, double *ms) {
    if (!valid_level(P, 0)) return fail(BCMG_ERR_INVALID, "bad problem");
    if (!ms || reps < 1 || (!P->fp32 && !u)) return fail(BCMG_ERR_INVALID, "bad argument");
    bcmg_status st;
    const LevelH &V = P->lev[0];
    void *pu[1], *pr[1], *px[1] = {V.r};
    if (P->fp32) {  // the FP32 correction cycle's own finest arrays (overwritten)
        pu[0] = V.u;
        pr[0] = V.rhs;
    } else {  // a copy of u in the residual scratch of the finest level
        double *work = (double *)V.r;
        HIPCHK(hipMemcpyAsync(work, u, sizeof(double) * V.nn, hipMemcpyDeviceToDevice, P->stream));
        pu[0] = work;
        pr[0] = P->rhs64;
    }
    if ((st = upload_step_descs(P, 0, 1, pu, pr, px))) return st;
    const Item *segs = P->d_stepitems + P->off_seg[0];
    struct Events {  // destroyed on every return path
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) hipEventDestroy(e0);
            if (e1) hipEventDestroy(e1);
        }
    } ev;
    HIPCHK(hipEventCreate(&ev.e0));
    HIPCHK(hipEventCreate(&ev.e1));
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    const int pair = V.half ? kSweepPairSegs : INT32_MAX;  // as a batch launches it
    launch_rb_sweep(P->d, P->fp32, P->d_step, segs, P->n_seg[0], 0, P->d_stepst, P->stream, pair);  // warm
    HIPCHK(hipEventRecord(e0, P->stream));
    for (int i = 0; i < reps; i++) {
        launch_rb_sweep(P->d, P->fp32, P->d_step, segs, P->n_seg[0], 0, P->d_stepst, P->stream, pair);
        launch_rb_sweep(P->d, P->fp32, P->d_step, segs, P->n_seg[0], 1, P->d_stepst, P->stream, pair);
    }
    HIPCHK(hipEventRecord(e1, P->stream));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    *ms = t;
    return BCMG_OK;
}

}  // extern "C"
