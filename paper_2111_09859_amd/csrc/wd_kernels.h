// wd_kernels.h -- launchers of the gfx950 kernels (host side).
#pragma once

#include "wd_common.h"

namespace wd {

enum PassKind {
    PASS_CART = 0,    // Cartesian directional pass (derivatives + partials)
    PASS_D1 = 1,      // general pass 1: F_l = D_l phi
    PASS_D2 = 2,      // general pass 2: D_l U_m (and D_l n_m)
    PASS_FILTER = 3,  // filter along l
    PASS_FINAL = 4,   // pointwise stage finish (general, no Laplacian)
    PASS_RESID = 5,   // pointwise pseudo-step change
    PASS_FACE = 6,    // extrapolated face; l = face, stage = target buffer
    PASS_INIT = 7,    // initial field; stage = unused
    PASS_LAD = 8,     // LAD diffusivity along l; stage = phase (0 sensor,
                      // 1 smoothing)
    PASS_D12 = 9,     // pass 2 along direction 0 that also forms F_0
    PASS_UWADV = 10,  // pointwise upwind advective term (Eikonal grids)
    PASS_SCART = 11,  // segmented Cartesian pass (one wave per tile)
    PASS_SFILTER = 12,
    PASS_SLAD = 13,
    PASS_SCART_LAST = 14,   // segmented Cartesian pass that finishes the stage
    PASS_CFIN = 15,         // pointwise stage finish of a segmented Cartesian grid
    PASS_XSTAGE = 16,       // one-pass stage of an explicit-scheme Cartesian grid
    PASS_XLAD = 17,         // LAD field of a Cartesian grid in two passes (np 1 sensor, 2 smoothing)
                            // (l = the scheme's radius)
};

// Segmented passes (segment length M = 16, 24 or 32): workgroups of one
// wave, `lds` bytes of dynamic LDS.
void launch_seg(int kind, int fp64, int M, const GridDev *grids, const Item *items, int nitems,
                int l, int stage, int nwg, size_t lds, hipStream_t s);
// workgroups of a segmented kernel one compute unit holds by its registers
int seg_blocks_per_cu_regs(int kind, int fp64, int M);

// One launch of a pass over `nitems` work items with at most `nwg`
// workgroups (a persistent loop covers the rest).  Line passes run the
// variant whose tiles hold up to kThreads*np points (np = 1, 2, 4, 8).
void launch_pass(int kind, int fp64, int np, const GridDev *grids, const Item *items,
                 int nitems, int l, int stage, int nwg, hipStream_t s);

// line-pass launchers, one per value type and points per thread
#define WD_LINE_LAUNCHER(name)                                                    \
    void name(int kind, const GridDev *grids, const Item *items, int nitems, int l, \
              int stage, int nwg, hipStream_t s);                                   \
    int name##_occ(int kind);
WD_LINE_LAUNCHER(line_launch_f32_1)
WD_LINE_LAUNCHER(line_launch_f32_2)
WD_LINE_LAUNCHER(line_launch_f32_4)
WD_LINE_LAUNCHER(line_launch_f32_8)
WD_LINE_LAUNCHER(line_launch_f64_1)
WD_LINE_LAUNCHER(line_launch_f64_2)
WD_LINE_LAUNCHER(line_launch_f64_4)
WD_LINE_LAUNCHER(line_launch_f64_8)
#undef WD_LINE_LAUNCHER
// workgroups of a line pass's kernel that one compute unit holds at once
// workgroups of the one-pass explicit stage (scheme radius r, general or
// fast tiles) that one compute unit holds at once
int xstage_blocks_per_cu(int fp64, int r, int fast);
// workgroups of the two LAD passes (np 1 sensor, 2 smoothing) that one
// compute unit holds at once
int xlad_blocks_per_cu(int fp64, int np);
int line_blocks_per_cu(int kind, int fp64, int np);
// level-set burnback (uniform grids)
constexpr int kMaxLevels = 8;   // iso-values per length call
constexpr int kLsChunk = 4096;  // most points per work item of a level-set stage
// chunk: points per work item, kThreads .. kLsChunk
void launch_ls_stage(int fp64, const GridDev *g, const Item *it, int nitems, int stage,
                     double fdt, int chunk, int nwg, hipStream_t s);
// 2D/3D grids (grids[0], n0 x n1 x n2, n2 = 1 in 2D): lanes along x,
// kLsRows rows per thread, one z plane per launch-grid layer; -1 (nothing
// launched) when the launch grid would not fit
constexpr int kLsLanes = 256;
constexpr int kLsRows = 4;
int launch_ls_stage_rows(int fp64, const GridDev *g, int n0, int n1, int n2, int stage,
                         double fdt, hipStream_t s);
// both directions' faces of a 2D grid (grids[0], n0, n1 >= 4) in one launch
void launch_ls_face2d(int fp64, const GridDev *g, int n0, int n1, int stage, hipStream_t s);
void launch_ls_face(int fp64, const GridDev *g, const Item *it, int nitems, int l, int stage,
                    int nwg, hipStream_t s);
void launch_ls_signed(int fp64, long long n, const unsigned char *solid, const void *ds,
                      const void *dg, void *out, hipStream_t s);
// partials [nb][kMaxLevels] (FP64, device)
void launch_ls_length(int fp64, const void *phi, int nx, int ny, double hx, double hy,
                      const double *levels, int nlev, double *part, int nb, hipStream_t s);
// The device's copy of the library's static scratch array (calls that
// allocate nothing): its device address, looked up once per device with that
// device current; WD_OK or WD_ERR_HIP.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
int noalloc_scratch(int device, void **ptr);
void launch_finalize(const GridDev *grids, int ngrids, hipStream_t s);
void launch_mirror(const GridDev *grids, int ngrids, hipStream_t s);
// field-major metrics [c][q] into the point-major array [q][c] (dd = ndim^2)
void launch_met_points(int fp64, const void *src, void *dst, long long N, int dd, hipStream_t s);
void launch_convert(int src_fp64, int dst_fp64, const void *src, void *dst,
                    long long n, hipStream_t s);
void launch_invert(const double *J, void *out, int out_fp64, int d,
                   long long N, hipStream_t s);
// conservative metric form (3D): coordinate products, then the metrics from
// their derivatives (layouts as in wd_compute_metrics_form)
void launch_gcl_products(const double *x, const double *J, double *Q, long long N, hipStream_t s);
void launch_gcl_combine(const double *J, const double *D, void *out, int out_fp64, long long N,
                        hipStream_t s);
void launch_poisson_dist(const GridDev *g, int fp64, long long N,
                         const double *phip, void *out, hipStream_t s);

}  // namespace wd
