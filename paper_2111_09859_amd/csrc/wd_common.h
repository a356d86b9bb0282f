// wd_common.h -- structures shared by the host planner and the gfx950
// kernels of the wall-distance library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace wd {

constexpr int kThreads = 512;             // threads per workgroup (8 waves)
constexpr int kPPT = 8;                   // max points per thread in a tile
constexpr int kTileMax = kThreads * kPPT; // max points held by one tile
constexpr int kMaxLev = 14;               // max PCR levels of a line system
constexpr int kXTX = 64, kXTY = 16;    // one-pass explicit stage: x-y tile
constexpr int kChunk = 1024;              // points per pointwise work item
constexpr int kMaxLine = kTileMax;        // longest grid line supported

// A tridiagonal line system whose matrix does not depend on the data
// (compact first derivative or filter correction).  The host reduces it by
// parallel cyclic reduction once, in FP64, and stores per level and per
// position the two multipliers that fold the neighbours at distance
// s = 2^level into the right-hand side.  After `nlev` levels every row is
// decoupled to within rounding and x_i = d_i * scale_i.
struct LineOpDev {
    int n;
    int periodic;
    int nlev;                 // 0: no solve (explicit scheme), scale == 1
    int uniform;              // 1: every row has the same multipliers
                              //    (periodic lines): use lr / usc below
    int smod[kMaxLev];        // neighbour distance of each level (mod n)
    const void *tab;          // T2 [nlev][n]: (left, right) multipliers
    const void *scale;        // T [n]
    double lr[kMaxLev][2];    // uniform multipliers per level
    double usc;               // uniform final scale
};

// A data-independent tridiagonal line system split into S segments (the
// segmentation of SegGeo: M rows each, one of them possibly shorter).
// Each segment is solved on its own by Thomas' algorithm with host-factored
// rows, then corrected by its two coupling vectors (spikes) times the true
// values at the neighbouring segments' ends, which the host-inverted
// reduced system gives as linear combinations of all segments' local end
// values.  tab (T): five row arrays of n + S entries, position j at
// j + (segment of j): ell, ib, cb (local LU: y_j = r_j - ell_j y_{j-1},
// x_j = ib_j y_j - cb_j x_{j+1}), vv, ww (spikes on the previous segment's
// last and the next segment's first value); then per segment, 4S + 1
// apart, red[s][4][S]: the rows giving the previous segment's last value
// and the next segment's first value from (local first values, local last
// values).
__host__ __device__ inline int seg_table_len(int n, int S)
{
    return 5 * (n + S) + S * (4 * S + 1);
}

struct SegOpDev {
    int n, S;
    int periodic;
    int solve;                // 0: explicit scheme (no system)
    const void *tab;
};

// Segmentation and LDS geometry of the segmented passes along one
// direction: a tile holds W whole lines, lane w S + s owns segment s of
// line w.  Segments hold M positions except segment ks, which starts at bk
// and holds r (ks = S, bk = n when all are full); a short segment is never
// the last one, and is the first one only when it holds >= 5 positions.
// The line buffer keeps line w at w P, position j at j + (segment of j).
struct SegGeo {
    int S, W, M;
    int ks, bk, r;
    int P, xsize;
};

enum GridMode { MODE_CART = 0, MODE_GENERAL = 1 };
enum { XBC_NONE = 0, XBC_NEUMANN = 1, XBC_OUTFLOW = 2 };

// Per-grid state kept on the device.
struct GridState {
    int done;                 // set once the grid has stopped
    int iter;                 // pseudo iterations completed
    int status;               // wd status code
    int best_iter;            // iteration of the smallest max change
    double best;              // smallest max change so far
    double last;              // last max change
};

// Everything a kernel needs about one grid of a batch.
struct GridDev {
    int ndim, mode;
    int n[3];
    long long N;
    long long stride[3];
    int periodic[3];
    int wall_lo[3], wall_hi[3];
    int xbc[6];               // XBC_* per face (dir*2 + side)
    int uniform;
    double invh[3];
    double jump[3];           // coordinate seam jump (metric helper only)
    const void *met;          // FIELDS metrics (T), point-major: the ndim*ndim
                              // values of a point together, [q][l*ndim + m]
    const void *met_src;      // the caller's field-major metrics [l*ndim + m][q],
                              // copied into met by the initial pass
    const unsigned char *mask;

    // method
    int eq, lad, curv, scheme, rk, need_lap, filter, fused_resid;
    int fuse_faces;           // extrapolated faces all normal to the last
                              // direction: applied inside its passes
    int fnext;                // the finishing pass also forms the next
                              // stage's F of the last direction
    int stages;
    int uw;                   // first-order upwind advective term (Eqs. UW1-UW5)
    double eps, C, nu0, eps0, sigma, tol;
    double kp, kp2;           // largest modified wavenumbers: advective, diffusive
    int max_iter, stall;
    int warm;                 // initial field given by the caller
    int warm_probe;           // > 0: the runaway check after this iteration
    double fcoef[6];          // filter correction factor for N = 1..5
    double da, db, dc;        // interior derivative coefficients
    int dradius, compact;

    // buffers (T unless stated)
    void *phi, *ps, *acc, *dt;
    void *F[3];
    void *P[3];               // partial sums carried between passes
    void *uw2;                // upwind baseline: |U|^2 of the stage (its
                              // advective term is carried in P[1])
    double *rpart;            // [nparts][4] FP64 partials: max change, sum of
                              // squared changes, max -phi, max |phi|
    double *hist;             // [hist_cap][2]
    int hist_cap;
    int nparts;
    GridState *state;         // in the grid's own region
    GridState *mirror;        // copy in the batch's contiguous state array

    int seg;                  // 1: the segmented passes serve this grid
    int seg_split;            // 1: its last direction carries the sums on and
                              // a pointwise pass finishes the stage
    int xstage;               // 1: explicit scheme, each stage one pointwise
                              // pass (stage values alternate ps / P[0])
    int xkz, xkz2;            // z planes per item (chunk of the march) of its
                              // fast and of its general tiles
    int xlad;                 // 1: the LAD field in two passes over x-y tiles
    int xlkz;                 // their z planes per item
    SegGeo sgeo[3];
    SegOpDev sdop[3];         // segmented first-derivative operator
    SegOpDev sfop[3];         // segmented filter-correction operator
    LineOpDev dop[3];         // first-derivative operator per direction
    LineOpDev fop[3];         // filter-correction operator per direction
    int tw[3];                // tile width (lines per tile) per direction
    int ntiles[3];
    int nchunks;              // pointwise work items
};

// One-pass explicit stage tiles (kXTX x kXTY points of an x-y plane).
// Origin of tile t along a direction of n points, tiles of w points: the
// last tile is moved back to end at point n - 1 (it then covers points of
// the tile before it and finishes only its own ones), so that the closure
// rows of either end read points inside the tile and its halo.
__host__ __device__ inline int xtile_origin(int t, int w, int n)
{
    const int e = n - w > 0 ? n - w : 0;
    return t * w < e ? t * w : e;
}

// Whether x-y tile (x0, y0) of a grid is full and every U position it
// forms along x and y takes the interior row: such tiles go to the fast
// variant, the rest to the general one.
__host__ __device__ inline bool xtile_fast(int x0, int y0, int n0, int n1, bool px, bool py, int R)
{
    return n0 >= kXTX && n1 >= kXTY && (px || (x0 >= 2 * R && x0 + kXTX + 2 * R <= n0)) &&
           (py || (y0 >= 2 * R && y0 + kXTY + 2 * R <= n1));
}

struct Item {
    int grid;
    int tile;
};

}  // namespace wd
