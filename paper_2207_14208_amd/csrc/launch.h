// Host-side launchers of the device kernels (defined in cycle.hip / setup.hip).
#pragma once

#include "bcmg_internal.h"

namespace bcmg {

// ---- cycle kernels (cycle.hip); fp32 selects the element type of u/rhs/r ----
// FP32 launches over 2D/3D split levels with at least pair_min segments take four segments per
// wavefront and four nodes per lane (callers pass their threshold for split levels, INT32_MAX elsewhere)
void launch_rb_sweep(int d, int fp32, const Desc *descs, const Item *items, int nseg, int colour,
                     const SlotState *st, hipStream_t s, int pair_min = INT32_MAX);
// weighted Jacobi on the INSIDE rows: new values into r from the old field,
// then copied into u (two launches)
void launch_jacobi(int d, int fp32, const Desc *descs, const Item *items, int nseg, const SlotState *st,
                   hipStream_t s);
// Jacobi ghost step (new values into gnew, then applied); with bch, the
// applying launch also extends the new field into the band chunks bch.
// neu: some problem of the launch has Neumann ghost rows (selects the kernels
// that carry them; the others keep the Dirichlet row's registers)
void launch_ghost_relax(int d, int fp32, const Desc *descs, const Item *gch, int ngch, const SlotState *st,
                        hipStream_t s, const Item *bch = nullptr, int nbch = 0, int neu = 0);
// tu32/tr32: element types of (u, rhs) and r; norm: write partial sums of r^2;
// store 0: skip the stores of r (only the partial sums are wanted);
// split: every descriptor's level is stored split by node parity (an FP32,
// 2D or 3D level: vector loads and stores)
void launch_residual(int d, int tu32, int tr32, int norm, const Desc *descs, const Item *segs, int nseg,
                     const Item *gch, int ngch, const SlotState *st, double *partials, hipStream_t s, int neu = 0,
                     int store = 1, int split = 0);
// mode 1: the check after ncyc cycles (ncyc - 1 of them unchecked)
// nblk > 1 (with blk: nslots * nblk doubles, cnt: nslots ints, zero): nblk
// workgroups per slot
void launch_norm_finish(const NormRange *ranges, int nslots, const double *partials, int nseg_total, SlotState *st,
                        const double *rtol2, double *hist, int hist_stride, int mode, double *out, hipStream_t s,
                        int ncyc = 1, int nblk = 1, double *blk = nullptr, int *cnt = nullptr);
// extension of u into the band chunks bch (ghost values read from u)
// via_need: the chunks run over the needed band entries (bneed) instead of all of them
void launch_ext_gather(int fp32, const Desc *descs, const Item *bch, int nbch, int via_need, const SlotState *st,
                       hipStream_t s);
// restriction into the coarse segments csegs (INSIDE rows) and coarse ghost chunks cgch;
// red: the coarse INSIDE rows also take the first red half-sweep of their
// pre-smoothing (from the zero initial guess)
void launch_restrict(int d, int fp32, const Desc *descs, const Item *csegs, int nseg, const Item *cgch, int ncgch,
                     const SlotState *st, hipStream_t s, int red = 0);
void launch_prolong(int d, int fp32, const Desc *descs, const Item *fsegs, int nseg, const SlotState *st,
                    hipStream_t s);
void launch_coarse(int fp32, const Desc *descs, const int *list, int n, const SlotState *st, hipStream_t s);
// one workgroup per program: the V-cycle on the program's coarse levels
void launch_coarse_cycle(int d, int fp32, const Desc *descs, const Item *items, const CoarseProg *progs, int nprog,
                         const SlotState *st, int nu1, int nu2, hipStream_t s, int neu = 0);
// the same on the levels staged in LDS (lds_bytes of dynamic LDS per workgroup)
void launch_coarse_lds(int d, int fp32, const Desc *descs, const LdsProg *progs, int nprog, size_t lds_bytes,
                       const SlotState *st, int nu1, int nu2, hipStream_t s, int neu = 0);
// fill the programs' images (their levels' arrays fixed during a solve, at their LDS offsets)
void launch_lds_images(const Desc *descs, const LdsProg *progs, int nprog, hipStream_t s);
void launch_ir_update(const Desc *descs, const Item *segs, int nseg, const SlotState *st, float *const *eptr,
                      hipStream_t s);

// ---- setup kernels (setup.hip) ----
void launch_check_finite(const double *a, long long n, int *flag, hipStream_t s);
void launch_inject(int d, const double *phi_f, int nf, double *phi_c, int nc, hipStream_t s);
void launch_classify(int d, int n, const double *phi, uint8_t *cls, hipStream_t s);
// ordered compaction of the node indices p < nn with pred(p):
//   kind 0: cls[p] == value;  kind 1: mark[p] != 0 (mark passed as cls)
// counts/offsets: scratch of compact_blocks(nn) ints each; total written to *total_dev
int compact_blocks(long long nn);
// (fails only if its scan's temporary cannot be allocated; nothing is written then)
hipError_t launch_compact(const uint8_t *cls, long long nn, uint8_t value, int *counts, int *offsets, int *out,
                          int *total_dev, hipStream_t s);
void launch_ghost_geometry(int d, int N, int level, double h, const double *phi, const uint8_t *cls, const int *gidx,
                           int ng, int dtau_mode, double dtau_const, int bc, int *gcode, double *gtau, double *gdtau,
                           double *geta, double *gn, double *gq, int *gfb, double *gnd, hipStream_t s);
void launch_band_mark(int d, int N, const uint8_t *cls, const int *gidx, int ng, int K, uint8_t *mark,
                      hipStream_t s);
void launch_band_records(int d, int N, double h, const double *phi, const uint8_t *cls, const int *bidx, int nb,
                         int *bref, double *bw, hipStream_t s);
void launch_erow(int d, int N, const uint8_t *cls, const int *gidx, int ng, const int *bidx, int nb, const int *bref,
                 const double *bw, int j, const int *pptr, const int *pidx, const double *pcf, const int *optr,
                 int *counts, int *oidx, double *ocf, hipStream_t s);
void launch_rrow(int d, int Nc, const int *gidx_c, int ngc, int Nf, const uint8_t *cls_f, const int *gidx_f, int ngf,
                 const int *bidx_f, int nbf, const int *eptr_f, const int *eidx_f, const double *ecf_f,
                 int restrict_mode, const int *optr, int *counts, int *oidx, double *ocf, hipStream_t s);
hipError_t launch_scan(const int *counts, int n, int *ptr, hipStream_t s);
void launch_need_mark(int d, int Nf, const uint8_t *cls_f, const uint8_t *cls_c, uint8_t *mark_c, long long nnf,
                      hipStream_t s);
void launch_need_flags(const int *bidx, int nb, const uint8_t *mark, uint8_t *flag, hipStream_t s);
// per row: INSIDE/GHOST extent [xmin, xmax], and the INSIDE run [ia, ib] (ib = -1 unless the row's
// INSIDE nodes are consecutive)
void launch_row_extent(int d, int n, const uint8_t *cls, int *xmin, int *xmax, int *ia, int *ib, hipStream_t s);
void launch_coarse_setup(int d, int N, double h, const uint8_t *cls, const int *gidx, int ng, const int *gcode,
                         const double *gtau, int bc, const double *gnd, double reaction, double *work, double *ainv,
                         int *cmap, int *info, hipStream_t s);
void launch_set_rhs(long long nn, const uint8_t *cls, const double *f, double *rhs, hipStream_t s);
void launch_scatter_ghosts(const int *gidx, int ng, const double *gq, double *rhs, hipStream_t s);
void launch_fill_boundary(long long nn, const uint8_t *cls, const double *gbox, double *u, hipStream_t s);

}  // namespace bcmg
