// Internal declarations shared by the HIP translation units of libbcmg.
// Device data layout:
//   * every level keeps dense node arrays (x fastest): class (uint8), u, rhs, r;
//     with BCMG_LAYOUT_SPLIT the FP32 arrays of the large levels of a
//     mixed-precision problem (kSplitMinNodes, kSplitMinCoarseNodes) store
//     the two parities of the node index one after the other (NodeArr in
//     seg.h);
//   * the work of a launch is a list of items: row segments of <= 128 nodes
//     (one wavefront each) or chunks of <= 256 ghost / band entries (one
//     workgroup each); each item names a level descriptor, so one launch can
//     serve many problems and levels at once (batches);
//   * the normal extension of a level (K upwind Jacobi sweeps from zero) is a
//     fixed linear map from the ghost values to the band values; it is built
//     once at setup as sparse rows (CSR) and applied by one gather, and the
//     restriction of ghost rows is stored the same way over the fine ghosts;
//   * descriptors of one problem are contiguous, finest first, so the coarse
//     level of descriptor i is i+1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bcmg.h"

namespace bcmg {

enum : uint8_t { C_OUTSIDE = 0, C_INSIDE = 1, C_GHOST = 2, C_BOXDIR = 3 };

constexpr int kMaxLevels = 16;
constexpr int kSegLen = 128;    // nodes per row segment = one wavefront (two per lane)
constexpr int kChunk = 256;     // ghost / band entries per chunk = one workgroup
constexpr int kBlock = 256;     // threads per workgroup
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kRefZero = INT32_MIN;       // band reference to a node whose value is 0
constexpr int kRefFallback = INT32_MIN + 1; // band node with zero weight sum
constexpr int kCoarseMax = 125;           // unknowns of the coarsest level (5^3)
// levels with at most this many nodes are cycled by one workgroup per problem
constexpr long long kCoarseNodes = 5000;
// FP32 red-black launches over split levels with at least this many row
// segments take four of them per wavefront (BCMG_PARAM_SWEEP_PAIR_SEGS)
constexpr int kSweepPairSegs = 1;
// the finest residual's norm: partials per workgroup, and at most this many
// workgroups per slot
constexpr int kNormBlockEntries = 4096;
constexpr int kNormBlocksMax = 32;
// largest check_interval (cycles per convergence check of bcmg_solve)
constexpr int kMaxCheckInterval = 16;
// the finest FP32 arrays of a mixed-precision problem with more nodes than
// this are stored split by node parity under BCMG_LAYOUT_SPLIT
constexpr long long kSplitMinNodes = 1 << 17;
// the same for a coarser level: its restriction and prolongation reach the
// coarse values through the split index, which costs about what the vector
// sweep saves until the level is large (measured: a 257^3 level gains, the
// 129^3 and 65^3 levels, whose sweeps take a few microseconds, lose)
constexpr long long kSplitMinCoarseNodes = 1 << 22;
// spare entries at the end of a split array
constexpr long long kSplitPad = 16;
// levels with at most this many nodes keep a colour-sorted list of their
// INSIDE nodes (used when they are cycled in LDS)
constexpr long long kListNodes = 1 << 15;
// dynamic LDS a coarse workgroup may use to hold its levels (else they stay
// in HBM); gfx950 gives a workgroup up to 160 KiB
constexpr size_t kLdsBudget = 150 * 1024;

// Work item over a row segment: desc, first node, x0 | len << 16 (| kSegAllInside), j | k << 16.
// Ghost / band chunk: desc, first entry, count, unused.
using Item = int4;
// flag of a segment item whose nodes are all INSIDE (the sweep then needs no classes)
constexpr int kSegAllInside = 1 << 24;

struct alignas(16) Desc {
    int d, n, N, level;
    long long nn;
    long long sy, sz;         // strides of y and z (0 beyond d)
    double h, h2;
    const uint8_t *cls;
    int ng, nb;
    const int *gidx;          // ghost node indices, ascending
    const int *gcode;         // widths / signs (see bcmg_ghost_info)
    const double *gtau;       // [3*ng]
    const double *gdtau;      // [ng]
    const int *bidx;          // band node indices, ascending
    const int *bneed;         // band entries the prolongation reads (levels >= 1), ascending
    int nbn;                  //   their count
    const int *eptr;          // [nb+1] extension rows: v(band b) = sum ecoef * u(ghost eidx)
    const int *eidx;          //   ghost-list indices, ascending within a row
    const double *ecoef;
    const int *rptr;          // [ng+1] restricted value of this level's ghost g (levels >= 1):
    const int *ridx;          //   sum rcoef * r_fine(ridx), ridx = fine node indices
    const double *rcoef;
    const int *ilist;         // INSIDE nodes, even i+j+k first (small levels only, else null)
    int ni, nred;             //   their count and the count of the first colour
    void *u, *rhs, *r;        // level arrays, element type = cycle precision
    long long half_u, half_r; // storage order of u and rhs / of r: 0 natural (x fastest), else split by the
                              //   parity of the node index, even first, half = (nn + 1) / 2 (see NodeArr)
    double *gnew;             // [ng] new ghost values of a Jacobi ghost step
    // coarsest level: dense inverse over INSIDE then GHOST unknowns
    int nc, singular;
    const double *ainv;       // [nc*nc]
    const int *cmap;          // [nc] node index of each unknown
    int slot;                 // problem slot (state / flags index)
    int restrict_mode;
    const double *gnd;        // [3*ng] Neumann rows: coefficient of d/dt_k (t_k local, growing along -s_k);
                              //   null: Dirichlet rows
    double reaction;          // c of the interior row c u - Laplace u
};

// Per-slot solve state kept on the device.
struct alignas(16) SlotState {
    int active;     // 1 while the slot iterates
    int cycles;     // cycles done
    int status;     // bcmg_status of the solve
    int max_cycles;
    double r0sq;    // ||r^0||^2
    double tolsq;   // (rel_tol * ||r^0||)^2
    double refsq;   // max(||r^0||^2, ||r^1||^2): divergence reference
    double lastsq;  // latest ||r||^2
};

// Work of one level inside the per-problem coarse workgroup: ranges in the
// batch's item array (segments, ghost chunks, band chunks) and its descriptor.
struct CoarseLevel {
    int seg, nseg, gch, ngch, bch, nbch, desc, pad;
};

// The aligned levels 0..top of one problem (0 = coarsest) run by k_coarse_cycle.
struct alignas(16) CoarseProg {
    int slot, top;
    int ext_top;  // 1 if the problem has a finer level above top: extend top's error for its prolongation
    int pad;
    CoarseLevel lev[kMaxLevels];
};

// A level of the per-problem coarse workgroup held in LDS: sizes, and the
// byte offsets of its node arrays and ghost records in the workgroup's
// dynamic LDS block (its extension and restriction rows, read once per
// cycle, stay in HBM).
struct LdsLevel {
    int desc;                              // global descriptor of the level
    int nn, ng, nb, ni, nred, nbn;         // nodes, ghosts, band nodes, INSIDE nodes (first colour), needed band
    int cls, u, rhs, r;                    // node arrays (r < 0: the residual stays in HBM)
    int ilist;                             // INSIDE nodes by colour
    int bneed;                             // needed band entries
    int gidx, gcode, gtau, gdtau, gnew;    // ghost records
    int gnd;                               // Neumann derivative coefficients (< 0: Dirichlet rows)
};

// The aligned levels 0..top of one problem cycled in LDS by k_coarse_lds.
// The arrays that do not change during a solve (classes, ghost records,
// INSIDE lists, needed band entries) of all its levels come first in the
// LDS block, and image holds a copy of that part (static_words 4-byte
// words), built when the batch's programs are built.
struct alignas(16) LdsProg {
    int slot, top, ext_top;
    int finest;  // 1 if top is the problem's finest level (u is the caller's: only unknowns are written back)
    int static_words, pad;
    const uint32_t *image;
    LdsLevel lev[kMaxLevels];
};

// Per-slot ranges of the partial sums written by a finest-level residual.
struct alignas(16) NormRange {
    int seg_beg, seg_end;     // wavefront partials
    int gch_beg, gch_end;     // ghost-chunk partials (offset by the segment count)
};

inline __host__ __device__ int code_w(int code, int k) { return (code >> (2 * k)) & 3; }
inline __host__ __device__ int code_s(int code, int k) { return ((code >> (6 + k)) & 1) ? -1 : 1; }

}  // namespace bcmg
