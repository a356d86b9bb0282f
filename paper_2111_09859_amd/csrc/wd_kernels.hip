// wd_kernels.hip -- gfx950 kernels of the wall-distance pseudo-time march.
//
// Every pass works on "line tiles": a workgroup loads whole grid lines of
// one direction into LDS (rows for direction 0; a band of consecutive
// x-columns for directions 1 and 2, so global loads stay coalesced along x),
// evaluates the explicit right-hand side of a derivative or filter stencil
// there, and solves the line's tridiagonal system (compact schemes,
// Sec. 3.2; implicit filter, Sec. 3.4) by parallel cyclic reduction with
// host-precomputed multipliers, so every lane keeps working on its own
// points with one barrier per level instead of a serial Thomas sweep.
// Partial sums (|grad phi|^2, Laplacian, curvature, LAD sensor) are carried
// between the directional passes in HBM and the last pass of each RK stage
// finishes the pseudo-time update point by point (Sec. 3.3).
//
// All kernels take a table of grids and a list of (grid, tile) work items,
// so one launch advances any number of independent grids; a persistent
// workgroup loop walks the items, giving each XCD a contiguous range.
#include "wd_common.h"
#include "wd_kernels.h"

#include <cmath>

namespace wd {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

enum { EQ_EIK = 0, EQ_HJ = 1, EQ_POIS = 2 };
enum { SCH_E2 = 0, SCH_E4 = 1, SCH_E6 = 2, SCH_C4 = 3, SCH_C6 = 4 };

// ---------------------------------------------------------------------
// work distribution
__device__ inline int item_begin(int nitems, int &step, int &end)
{
    const int b = blockIdx.x, nb = gridDim.x;
    if (nb >= nitems || nb < 8 || (nb & 7)) {
        step = nb;
        end = nitems;
        return b;
    }
    // contiguous item range per XCD (workgroups go round-robin to XCDs)
    const int xcd = b & 7, slot = b >> 3, wpx = nb >> 3;
    const int ipx = (nitems + 7) >> 3;
    const int lo = xcd * ipx;
    end = min(nitems, lo + ipx);
    step = wpx;
    return lo + slot;
}

// ---------------------------------------------------------------------
// tile geometry
struct Tile {
    long long base;  // offset of (line 0, position 0)
    long long gw;    // offset between lines of the tile
    long long gj;    // offset along a line
    int wa;          // lines in the tile
    int n;           // line length
    int lj;          // LDS distance along a line
    int P;           // points in the tile
    int i0s;         // first x index (directions 1, 2)
    long long rest;  // first line (dir 0) / i2 (dir 1) / i1 (dir 2)
};

__device__ inline Tile decode_tile(const GridDev &g, int l, int t)
{
    Tile r;
    r.n = g.n[l];
    const int W = g.tw[l];
    if (l == 0) {
        const long long lines = g.N / g.n[0];
        const long long first = (long long)t * W;
        r.wa = (int)min((long long)W, lines - first);
        r.base = first * g.n[0];
        r.gw = g.n[0];
        r.gj = 1;
        r.lj = 1;
        r.i0s = 0;
        r.rest = first;
    } else {
        const int n0 = g.n[0];
        const int tpp = (n0 + W - 1) / W;
        const int c = t % tpp;
        const long long rest = t / tpp;
        r.i0s = c * W;
        r.wa = min(W, n0 - r.i0s);
        r.base = (l == 1) ? r.i0s + rest * (long long)n0 * g.n[1]
                          : r.i0s + rest * (long long)n0;
        r.gw = 1;
        r.gj = g.stride[l];
        r.lj = r.wa;
        r.rest = rest;
    }
    r.P = r.wa * r.n;
    return r;
}

struct Pts {
    int J[kPPT];    // position along the line
    int Q[kPPT];    // global offset within the grid
};

__device__ inline void tile_points(const Tile &tl, int l, Pts &pt)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        const int p = tid + k * kThreads;
        int j, w;
        if (l == 0) {
            w = p / tl.n;
            j = p - w * tl.n;
        } else {
            j = p / tl.wa;
            w = p - j * tl.wa;
        }
        pt.J[k] = j;
        pt.Q[k] = (int)(tl.base + w * tl.gw + j * tl.gj);
    }
}

__device__ inline bool pvalid(const Tile &tl, int k)
{
    return (int)threadIdx.x + k * kThreads < tl.P;
}

// grid indices of point k of this thread in a tile
__device__ inline void tile_index(const GridDev &g, const Tile &tl, int l,
                                  int k, int j, int *idx)
{
    const int p = (int)threadIdx.x + k * kThreads;
    const int w = l == 0 ? p / tl.n : p - j * tl.wa;
    if (l == 0) {
        const long long line = tl.rest + w;
        idx[0] = j;
        idx[1] = (int)(line % g.n[1]);
        idx[2] = (int)(line / g.n[1]);
    } else if (l == 1) {
        idx[0] = tl.i0s + w;
        idx[1] = j;
        idx[2] = (int)tl.rest;
    } else {
        idx[0] = tl.i0s + w;
        idx[1] = (int)tl.rest;
        idx[2] = j;
    }
}

__device__ inline bool wall_point(const GridDev &g, const int *idx)
{
    bool z = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < g.ndim) {
            z |= (idx[d] == 0 && g.wall_lo[d]);
            z |= (idx[d] == g.n[d] - 1 && g.wall_hi[d]);
        }
    }
    return z;
}

__device__ inline void index_of(const GridDev &g, long long q, int *idx)
{
    idx[0] = (int)(q % g.n[0]);
    const long long r = q / g.n[0];
    idx[1] = (int)(r % g.n[1]);
    idx[2] = (int)(r / g.n[1]);
}

// metric d xi_l / d x_m at point q
template <typename T>
__device__ inline T metric(const GridDev &g, int l, int m, int q)
{
    if (g.uniform)
        return l == m ? (T)g.invh[l] : (T)0;
    return static_cast<const T *>(g.met)[(long long)(l * g.ndim + m) * g.N + q];
}

// ---------------------------------------------------------------------
// Right-hand sides.  X holds the tile in LDS; p is the point's LDS index,
// j its position on a line of length n whose LDS stride is lj.

// value at position j+o on a periodic line, with the coordinate seam jump
template <typename T>
__device__ inline T pval(const T *X, int p, int j, int o, int n, int lj, T jump)
{
    int jj = j + o;
    T add = (T)0;
    if (jj >= n) { jj -= n; add = jump; }
    else if (jj < 0) { jj += n; add = -jump; }
    return X[p + (jj - j) * lj] + add;
}

// first-derivative right-hand side (index space), scheme of Sec. 3.2
template <typename T>
__device__ T deriv_rhs(const GridDev &g, const T *X, int p, int j, int n,
                       int lj, int periodic, T jump)
{
    const T a = (T)g.da, b = (T)g.db, c = (T)g.dc;
    const int r = g.dradius;
    if (periodic) {
        T s = a * (pval(X, p, j, 1, n, lj, jump) - pval(X, p, j, -1, n, lj, jump)) * (T)0.5;
        if (r >= 2)
            s += b * (pval(X, p, j, 2, n, lj, jump) - pval(X, p, j, -2, n, lj, jump)) * (T)0.25;
        if (r >= 3)
            s += c * (pval(X, p, j, 3, n, lj, jump) - pval(X, p, j, -3, n, lj, jump)) / (T)6;
        return s;
    }
    const int p0 = p - j * lj;
    if (g.compact) {
        if (j == 0) {
            return (T)(-17.0 / 6.0) * X[p0] + (T)1.5 * X[p0 + lj]
                   + (T)1.5 * X[p0 + 2 * lj] - X[p0 + 3 * lj] / (T)6;
        }
        if (j == n - 1) {
            const int e = p0 + (n - 1) * lj;
            return -((T)(-17.0 / 6.0) * X[e] + (T)1.5 * X[e - lj]
                     + (T)1.5 * X[e - 2 * lj] - X[e - 3 * lj] / (T)6);
        }
        if (g.scheme == SCH_C6 && (j == 1 || j == n - 2))
            return (T)0.75 * (X[p + lj] - X[p - lj]);
    } else if (j < r || j > n - 1 - r) {
        // one-sided / biased closures, mirrored with a sign flip
        const bool hi = j > n - 1 - r;
        const int k = hi ? n - 1 - j : j;
        const int e = hi ? p0 + (n - 1) * lj : p0;
        const int sgn = hi ? -1 : 1;
        T f[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) f[i] = (i <= 2 || g.scheme != SCH_E2) ? X[e + sgn * i * lj] : (T)0;
        T v;
        if (g.scheme == SCH_E2)
            v = ((T)-3 * f[0] + (T)4 * f[1] - f[2]) * (T)0.5;
        else if (k == 0)
            v = ((T)-25 * f[0] + (T)48 * f[1] - (T)36 * f[2] + (T)16 * f[3] - (T)3 * f[4]) / (T)12;
        else if (k == 1)
            v = ((T)-3 * f[0] - (T)10 * f[1] + (T)18 * f[2] - (T)6 * f[3] + f[4]) / (T)12;
        else
            v = (f[0] - (T)8 * f[1] + (T)8 * f[3] - f[4]) / (T)12;
        return hi ? -v : v;
    }
    T s = a * (X[p + lj] - X[p - lj]) * (T)0.5;
    if (r >= 2) s += b * (X[p + 2 * lj] - X[p - 2 * lj]) * (T)0.25;
    if (r >= 3) s += c * (X[p + 3 * lj] - X[p - 3 * lj]) / (T)6;
    return s;
}

// filter correction right-hand side: c_N * delta^{2N} f, with N = 5 inside
// and N = distance to a non-periodic boundary near it (0 on the boundary)
template <typename T>
__device__ T filter_rhs(const GridDev &g, const T *X, int p, int j, int n,
                        int lj, int periodic)
{
    int N = 5;
    if (!periodic) {
        const int d = min(j, n - 1 - j);
        if (d == 0) return (T)0;
        N = min(d, 5);
    }
    T s;
    if (N == 5) {
        // tenth central difference, symmetric pairs
        T v[11];
#pragma unroll
        for (int o = -5; o <= 5; ++o)
            v[o + 5] = periodic ? pval(X, p, j, o, n, lj, (T)0) : X[p + o * lj];
        s = (v[0] + v[10]) - (T)10 * (v[1] + v[9]) + (T)45 * (v[2] + v[8])
            - (T)120 * (v[3] + v[7]) + (T)210 * (v[4] + v[6]) - (T)252 * v[5];
    } else {
        // sum_k (-1)^k C(2N, k) f_{j-N+k}, binomials built as we go
        s = (T)0;
        int c = 1;
        for (int k = 0; k <= 2 * N; ++k) {
            s += (T)((k & 1) ? -c : c) * X[p + (k - N) * lj];
            c = c * (2 * N - k) / (k + 1);
        }
    }
    return (T)g.fcoef[N] * s;
}

// five-point fourth difference, copied inward of the two boundary points
template <typename T>
__device__ T fourth_diff(const T *X, int p, int j, int n, int lj, int periodic)
{
    if (periodic) {
        return pval(X, p, j, -2, n, lj, (T)0) - (T)4 * pval(X, p, j, -1, n, lj, (T)0)
               + (T)6 * X[p] - (T)4 * pval(X, p, j, 1, n, lj, (T)0)
               + pval(X, p, j, 2, n, lj, (T)0);
    }
    const int c = min(max(j, 2), n - 3);
    const int pc = p + (c - j) * lj;
    return X[pc - 2 * lj] - (T)4 * X[pc - lj] + (T)6 * X[pc] - (T)4 * X[pc + lj]
           + X[pc + 2 * lj];
}

// ---------------------------------------------------------------------
// Parallel cyclic reduction with precomputed multipliers, for g <= G
// right-hand sides of the same line system at once (field f uses LDS
// segment f of A and B, each tl.P long).  On entry v[f] holds this thread's
// right-hand sides, on exit the solutions.  One barrier per level serves
// all fields; periodic lines use per-level scalar multipliers, other lines
// read the next level's multipliers while the current one is applied.  The
// caller must have finished every read of A and B.
template <typename T, int G>
__device__ void pcr_multi(T (&v)[G][kPPT], int g, const Pts &pt, const Tile &tl,
                          const LineOpDev &op, T *A, T *B, bool in_lds = false)
{
    using T2 = typename V2<T>::t;
    const int nlev = op.nlev;
    const int tid = threadIdx.x;
    const int n = tl.n, lj = tl.lj, P = tl.P;
    if (in_lds) {
        // right-hand sides were written to A by the caller (after a barrier)
#pragma unroll
        for (int f = 0; f < G; ++f) {
            if (f >= g) break;
#pragma unroll
            for (int k = 0; k < kPPT; ++k)
                if (pvalid(tl, k)) v[f][k] = A[f * P + tid + k * kThreads];
        }
    }
    if (nlev == 0) {
        if (in_lds) __syncthreads();
        return;
    }
    if (!in_lds) {
#pragma unroll
        for (int f = 0; f < G; ++f) {
            if (f >= g) break;
#pragma unroll
            for (int k = 0; k < kPPT; ++k)
                if (pvalid(tl, k)) A[f * P + tid + k * kThreads] = v[f][k];
        }
        __syncthreads();
    }
    T *cur = A, *nxt = B;
    const T2 *tab = static_cast<const T2 *>(op.tab);
    const bool uni = op.uniform;
    T2 cn[kPPT];
    if (!uni) {
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) cn[k] = tab[pt.J[k]];
    }
    for (int lev = 0; lev < nlev; ++lev) {
        const int s = op.smod[lev];
        const bool more = lev + 1 < nlev;
        T2 cu;
        cu.x = (T)op.lr[lev][0];
        cu.y = (T)op.lr[lev][1];
        const T2 *nrow = tab + (long long)(lev + 1) * n;
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            if (!pvalid(tl, k)) continue;
            const int j = pt.J[k];
            T2 c = cu;
            if (!uni) {
                c = cn[k];
                if (more) cn[k] = nrow[j];   // next level, in flight meanwhile
            }
            const int p = tid + k * kThreads;
            int jm = j - s, jp = j + s;
            if (op.periodic) {
                jm += jm < 0 ? n : 0;
                jp -= jp >= n ? n : 0;
            } else {
                jm = max(jm, 0);
                jp = min(jp, n - 1);
            }
            const int om = p + (jm - j) * lj, opp = p + (jp - j) * lj;
#pragma unroll
            for (int f = 0; f < G; ++f) {
                if (f >= g) break;
                v[f][k] = v[f][k] + c.x * cur[f * P + om] + c.y * cur[f * P + opp];
                if (more) nxt[f * P + p] = v[f][k];
            }
        }
        if (more) {
            __syncthreads();
            T *t = cur; cur = nxt; nxt = t;
        }
    }
    const T *sc = static_cast<const T *>(op.scale);
#pragma unroll
    for (int k = 0; k < kPPT; ++k) {
        if (!pvalid(tl, k)) continue;
        const T m = uni ? (T)op.usc : sc[pt.J[k]];
#pragma unroll
        for (int f = 0; f < G; ++f)
            if (f < g) v[f][k] *= m;
    }
    __syncthreads();
}

template <typename T>
__device__ inline void pcr_solve(T (&v)[kPPT], const Pts &pt, const Tile &tl,
                                 const LineOpDev &op, T *A, T *B)
{
    pcr_multi<T, 1>(reinterpret_cast<T(&)[1][kPPT]>(v), 1, pt, tl, op, A, B);
}

// Extrapolated faces normal to direction l, applied inside a line tile
// whose new values sit in LDS X: points j = 0 / n-1 of each line take
// (4 f_1 - f_2)/3 (Neumann) or 2 f_1 - f_2 (outflow) from their inward
// neighbours, unless they are wall or solid points.
template <typename T>
__device__ inline T face_value(const GridDev &g, int l, const T *X, int p, int j, int n,
                               int lj, T v, bool zero)
{
    int code = XBC_NONE, in = 0;
    if (j == 0) {
        code = g.xbc[2 * l];
        in = lj;
    } else if (j == n - 1) {
        code = g.xbc[2 * l + 1];
        in = -lj;
    }
    if (code == XBC_NONE || zero) return v;
    const T a = X[p + in], b = X[p + 2 * in];
    return code == XBC_NEUMANN ? ((T)4 * a - b) / (T)3 : (T)2 * a - b;
}

// ---------------------------------------------------------------------
// Pseudo-time update of one point (Sec. 3.3): residual of the chosen
// equation, local time step at stage 0, RK stage combination, walls/solids;
// returns the new stage value (the caller stores it).
template <typename T>
__device__ T finish_point(const GridDev &g, int stage, int q, bool zero,
                          T phis, T g2, T lap, T kap, T lads, T S1, T S2)
{
    T *dtp = static_cast<T *>(g.dt);
    const T gm = sqrt(g2);
    T gam = (T)0, nu = (T)0, R;
    if (g.eq == EQ_HJ) {
        gam = (T)g.eps * phis;
        if (g.lad && lads < gam) gam = lads;   // smoothed C|S| of this iteration
        gam = gam > (T)0 ? gam : (T)0;
        if (g.curv) {
            nu = (T)g.nu0 * ((T)1 - gm) * ((T)1 - gm);
            const T gk = gm * kap;
            R = (T)1 + (gam + nu) * (lap - (gk > (T)0 ? gk : (T)0)) - g2;
        } else {
            R = (T)1 + gam * lap - g2;
        }
    } else if (g.eq == EQ_EIK) {
        R = (T)1 - g2;
    } else {
        R = (T)1 + lap;
    }
    T dt;
    if (stage == 0) {
        const T kp = (T)g.kp;
        const T gmx = gm > (T)1 ? gm : (T)1;
        T den;
        if (g.eq == EQ_EIK)
            den = (T)2 * kp * S1 * gmx;
        else if (g.eq == EQ_POIS)
            den = kp * kp * S2;
        else
            den = (T)2 * kp * S1 * gmx + kp * kp * (gam + nu) * S2;
        dt = (T)g.sigma / den;
        dtp[q] = dt;
    } else {
        dt = dtp[q];
    }
    const T pn = stage == 0 ? phis : static_cast<const T *>(g.phi)[q];
    T out;
    if (g.rk == 1) {
        T *acc = static_cast<T *>(g.acc);
        if (stage == 0) {
            acc[q] = pn + dt / (T)6 * R;
            out = pn + dt / (T)2 * R;
        } else if (stage == 1) {
            acc[q] += dt / (T)3 * R;
            out = pn + dt / (T)2 * R;
        } else if (stage == 2) {
            acc[q] += dt / (T)3 * R;
            out = pn + dt * R;
        } else {
            out = acc[q] + dt / (T)6 * R;
        }
    } else {
        if (stage == 0)
            out = pn + dt * R;
        else if (stage == 1)
            out = (T)0.75 * pn + (T)0.25 * (phis + dt * R);
        else
            out = pn / (T)3 + (T)2 / (T)3 * (phis + dt * R);
    }
    return zero ? (T)0 : out;
}

template <typename T>
__device__ inline void metric_sums(const GridDev &g, int q, T &S1, T &S2)
{
    S1 = (T)0;
    S2 = (T)0;
    for (int l = 0; l < g.ndim; ++l) {
        T s2 = (T)0;
        for (int m = 0; m < g.ndim; ++m) {
            const T e = metric<T>(g, l, m, q);
            s2 += e * e;
        }
        S1 += sqrt(s2);
        S2 += s2;
    }
}

// Store a tile's new stage values (last pass of an RK stage), applying
// the extrapolated faces of this direction inside the tile when the grid
// keeps all of them here.
template <typename T>
__device__ void store_stage(const GridDev &g, const Tile &tl, const Pts &pt, int l,
                            T (&v)[kPPT], const bool (&zero)[kPPT], T *X)
{
    T *ps = static_cast<T *>(g.ps);
    if (g.fuse_faces) {
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) X[threadIdx.x + k * kThreads] = v[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k))
                v[k] = face_value(g, l, X, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj,
                                  v[k], zero[k]);
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < kPPT; ++k)
        if (pvalid(tl, k)) ps[pt.Q[k]] = v[k];
}

// ---------------------------------------------------------------------
// Cartesian pass along direction l (uniform spacing, no curvature): the
// line already holds everything the direction contributes -- U_l = D_l phi,
// D_l U_l, and the LAD sensor -- so one pass per direction suffices; the
// last direction finishes the stage.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cart(const GridDev *__restrict__ grids, const Item *__restrict__ items,
       int nitems, int l, int stage)
{
    __shared__ T A[kTileMax];
    __shared__ T B[kTileMax];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts pt;
        tile_points(tl, l, pt);
        const T *src = static_cast<const T *>(stage == 0 ? g.phi : g.ps);
        const int per = g.periodic[l];
        T v0[kPPT], r[kPPT];
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) {
                v0[k] = src[pt.Q[k]];
                A[threadIdx.x + k * kThreads] = v0[k];
            }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k))
                r[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per, (T)0);
        __syncthreads();
        pcr_solve(r, pt, tl, g.dop[l], A, B);
        const T ih = (T)g.invh[l];
        T g2c[kPPT], lapc[kPPT];
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            r[k] *= ih;              // U_l
            g2c[k] = r[k] * r[k];
            lapc[k] = (T)0;
        }
        if (g.need_lap) {
#pragma unroll
            for (int k = 0; k < kPPT; ++k)
                if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = r[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kPPT; ++k)
                if (pvalid(tl, k))
                    lapc[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k],
                                        tl.n, tl.lj, per, (T)0);
            __syncthreads();
            pcr_solve(lapc, pt, tl, g.dop[l], A, B);
#pragma unroll
            for (int k = 0; k < kPPT; ++k) lapc[k] *= ih;
        }
        T *P0 = static_cast<T *>(g.P[0]);
        T *P1 = static_cast<T *>(g.P[1]);
        T *P2 = static_cast<T *>(g.P[2]);
        const bool last = l == g.ndim - 1;
        if (!last) {
#pragma unroll
            for (int k = 0; k < kPPT; ++k) {
                if (!pvalid(tl, k)) continue;
                const int q = pt.Q[k];
                P0[q] = l == 0 ? g2c[k] : P0[q] + g2c[k];
                if (g.need_lap) P1[q] = l == 0 ? lapc[k] : P1[q] + lapc[k];
            }
        } else {
            T S1 = (T)0, S2 = (T)0;
            for (int d = 0; d < g.ndim; ++d) {
                S1 += (T)g.invh[d];
                S2 += (T)g.invh[d] * (T)g.invh[d];
            }
            bool zero[kPPT];
#pragma unroll
            for (int k = 0; k < kPPT; ++k) {
                zero[k] = true;
                if (!pvalid(tl, k)) continue;
                const int q = pt.Q[k];
                int idx[3];
                tile_index(g, tl, l, k, pt.J[k], idx);
                zero[k] = wall_point(g, idx) || (g.mask && g.mask[q]);
                const T g2 = P0[q] + g2c[k];
                const T lap = g.need_lap ? P1[q] + lapc[k] : (T)0;
                const T lads = g.lad ? P2[q] : (T)0;
                v0[k] = finish_point<T>(g, stage, q, zero[k], v0[k], g2, lap, (T)0, lads, S1, S2);
            }
            store_stage(g, tl, pt, l, v0, zero, A);
        }
    }
}

// General pass 1 along direction l: F_l = D_l phi.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_d1(const GridDev *__restrict__ grids, const Item *__restrict__ items,
     int nitems, int l, int stage)
{
    __shared__ T A[kTileMax];
    __shared__ T B[kTileMax];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts pt;
        tile_points(tl, l, pt);
        const T *src = static_cast<const T *>(stage == 0 ? g.phi : g.ps);
        const int per = g.periodic[l];
        T r[kPPT];
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = src[pt.Q[k]];
        __syncthreads();
        const T jump = (T)g.jump[l];
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k))
                r[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per, jump);
        __syncthreads();
        pcr_solve(r, pt, tl, g.dop[l], A, B);
        T *F = static_cast<T *>(g.F[l]);
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) F[pt.Q[k]] = r[k];
    }
}

// contravariant pieces at a point from the stored F_l and the metrics
template <typename T>
__device__ inline void grad_at(const GridDev &g, int q, T *U, T &g2)
{
    g2 = (T)0;
    U[2] = (T)0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        if (m >= g.ndim) break;
        T u = (T)0;
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (l >= g.ndim) break;
            u += metric<T>(g, l, m, q) * static_cast<const T *>(g.F[l])[q];
        }
        U[m] = u;
        g2 += u * u;
    }
}

// General pass 2 along direction l: D_l of U_m (and of n_m for the
// curvature), weighted by xi_{l,m}: the chain-rule Laplacian of Eq.
// Ham_Jac_trans and kappa = div n.  The last direction finishes the stage.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_d2(const GridDev *__restrict__ grids, const Item *__restrict__ items,
     int nitems, int l, int stage)
{
    __shared__ T A[kTileMax];
    __shared__ T B[kTileMax];
    constexpr int GM = sizeof(T) == 4 ? 4 : 2;   // fields per reduction sweep
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts pt;
        tile_points(tl, l, pt);
        const int per = g.periodic[l];
        const int d = g.ndim;
        const int P = tl.P;
        // fields differentiated along l: U_m (and n_m), weighted by xi_{l,m};
        // field f is coded in bits 3f..3f+2 of `code` (component m, n-flag)
        int code = 0, nf = 0;
        for (int f = 0; f < (g.curv ? 2 * d : d); ++f) {
            const int m = f % d;
            if (g.uniform && m != l) continue;
            code |= (m | ((f >= d) << 2)) << (3 * nf);
            ++nf;
        }
        const int G = min(GM, max(1, kTileMax / P));
        T lapc[kPPT], kapc[kPPT];
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            lapc[k] = (T)0;
            kapc[k] = (T)0;
        }
        for (int f0 = 0; f0 < nf; f0 += G) {
            const int gcount = min(G, nf - f0);
            // field values of this group into B, point by point
#pragma unroll 1
            for (int k = 0; k < kPPT; ++k) {
                if (!pvalid(tl, k)) break;
                const int q = pt.Q[k];
                T U[3], g2;
                grad_at<T>(g, q, U, g2);
                const T inv = (T)1 / (sqrt(g2) + (T)g.eps0);
                for (int f = 0; f < gcount; ++f) {
                    const int c = code >> (3 * (f0 + f));
                    const int m = c & 3;
                    const T u = m == 0 ? U[0] : (m == 1 ? U[1] : U[2]);
                    B[f * P + threadIdx.x + k * kThreads] = (c & 4) ? u * inv : u;
                }
            }
            __syncthreads();
            // right-hand sides from B into A
            for (int f = 0; f < gcount; ++f)
#pragma unroll 1
                for (int k = 0; k < kPPT; ++k) {
                    if (!pvalid(tl, k)) break;
                    const int p = threadIdx.x + k * kThreads;
                    A[f * P + p] = deriv_rhs(g, B + f * P, p, pt.J[k], tl.n, tl.lj, per, (T)0);
                }
            __syncthreads();
            T v[GM][kPPT];
            pcr_multi<T, GM>(v, gcount, pt, tl, g.dop[l], A, B, true);
#pragma unroll
            for (int f = 0; f < GM; ++f) {
                if (f >= gcount) break;
                const int c = code >> (3 * (f0 + f));
                const int m = c & 3;
                const bool isn = (c & 4) != 0;
#pragma unroll
                for (int k = 0; k < kPPT; ++k) {
                    if (!pvalid(tl, k)) continue;
                    const T wgt = metric<T>(g, l, m, pt.Q[k]);
                    if (isn) kapc[k] += wgt * v[f][k];
                    else lapc[k] += wgt * v[f][k];
                }
            }
        }
        T *P0 = static_cast<T *>(g.P[0]);
        T *P1 = static_cast<T *>(g.P[1]);
        T *P2 = static_cast<T *>(g.P[2]);
        const bool last = l == d - 1;
        if (!last) {
#pragma unroll
            for (int k = 0; k < kPPT; ++k) {
                if (!pvalid(tl, k)) continue;
                const int q = pt.Q[k];
                P0[q] = l == 0 ? lapc[k] : P0[q] + lapc[k];
                if (g.curv) P1[q] = l == 0 ? kapc[k] : P1[q] + kapc[k];
            }
            continue;
        }
        // park the partial sums in LDS (own points only) and finish the
        // stage point by point, keeping the unrolled state small
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) {
                A[threadIdx.x + k * kThreads] = lapc[k];
                B[threadIdx.x + k * kThreads] = kapc[k];
            }
        T *ps = static_cast<T *>(g.ps);
        const T *src = static_cast<const T *>(stage == 0 ? g.phi : g.ps);
#pragma unroll 1
        for (int k = 0; k < kPPT; ++k) {
            if (!pvalid(tl, k)) break;
            const int p = threadIdx.x + k * kThreads;
            const int q = pt.Q[k];
            const int j = pt.J[k];
            const T lap = l == 0 ? A[p] : P0[q] + A[p];
            const T kap = g.curv ? (l == 0 ? B[p] : P1[q] + B[p]) : (T)0;
            const T lads = g.lad ? P2[q] : (T)0;
            int idx[3];
            tile_index(g, tl, l, k, j, idx);
            const bool zero = wall_point(g, idx) || (g.mask && g.mask[q]);
            T U[3], g2;
            grad_at<T>(g, q, U, g2);
            T S1, S2;
            metric_sums<T>(g, q, S1, S2);
            const T nv = finish_point<T>(g, stage, q, zero, src[q], g2, lap, kap, lads, S1, S2);
            B[p] = zero ? (T)1 : (T)0;   // wall flag for the face step
            A[p] = nv;
            if (!g.fuse_faces) ps[q] = nv;
        }
        if (g.fuse_faces) {
            __syncthreads();
#pragma unroll 1
            for (int k = 0; k < kPPT; ++k) {
                if (!pvalid(tl, k)) break;
                const int p = threadIdx.x + k * kThreads;
                ps[pt.Q[k]] = face_value(g, l, A, p, pt.J[k], tl.n, tl.lj, A[p], B[p] != (T)0);
            }
        }
        __syncthreads();
    }
}

// LAD diffusivity of Eq. Gamma_form2, once per pseudo iteration from
// phi^n.  mode 0 (one pass per direction): S += |grad xi_l| d4_l phi, and
// after the last direction S <- C |S|.  mode 1 (one pass per direction):
// smoothing of S along l with the nine-point truncated Gaussian filter of
// Kawai & Lele (ends clamped on non-periodic lines).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_lad(const GridDev *__restrict__ grids, const Item *__restrict__ items,
      int nitems, int l, int mode)
{
    __shared__ T A[kTileMax];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts pt;
        tile_points(tl, l, pt);
        const int per = g.periodic[l];
        T *S = static_cast<T *>(g.P[2]);
        const T *src = mode == 0 ? static_cast<const T *>(g.phi) : S;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = src[pt.Q[k]];
        __syncthreads();
        const bool last = l == g.ndim - 1;
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            if (!pvalid(tl, k)) continue;
            const int p = threadIdx.x + k * kThreads;
            const int q = pt.Q[k];
            const int j = pt.J[k];
            if (mode == 0) {
                T s2 = (T)0;
                for (int m = 0; m < g.ndim; ++m) {
                    const T e = metric<T>(g, l, m, q);
                    s2 += e * e;
                }
                T v = sqrt(s2) * fourth_diff(A, p, j, tl.n, tl.lj, per);
                if (l != 0) v += S[q];
                S[q] = last ? (T)g.C * fabs(v) : v;
            } else {
                const T b[5] = {(T)(3565.0 / 10368.0), (T)(3091.0 / 12960.0),
                                (T)(1997.0 / 25920.0), (T)(149.0 / 12960.0),
                                (T)(107.0 / 103680.0)};
                T acc = (T)0;
#pragma unroll
                for (int o = -4; o <= 4; ++o) {
                    int jj = j + o;
                    if (per) jj += jj < 0 ? tl.n : (jj >= tl.n ? -tl.n : 0);
                    else jj = min(max(jj, 0), tl.n - 1);
                    acc += b[o < 0 ? -o : o] * A[p + (jj - j) * tl.lj];
                }
                S[q] = acc;
            }
        }
    }
}

// Pointwise stage finish for general grids without a second derivative
// level (Eikonal).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_final(const GridDev *__restrict__ grids, const Item *__restrict__ items,
        int nitems, int stage)
{
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done) continue;
        const long long q0 = (long long)item.tile * kChunk;
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long qq = q0 + i;
            if (qq >= g.N) break;
            const int q = (int)qq;
            T U[3], g2;
            grad_at<T>(g, q, U, g2);
            int idx[3];
            index_of(g, q, idx);
            const bool zero = wall_point(g, idx) || (g.mask && g.mask[q]);
            const T phis = static_cast<const T *>(stage == 0 ? g.phi : g.ps)[q];
            T S1, S2;
            metric_sums<T>(g, q, S1, S2);
            static_cast<T *>(g.ps)[q] =
                finish_point<T>(g, stage, q, zero, phis, g2, (T)0, (T)0, (T)0, S1, S2);
        }
    }
}

// ---------------------------------------------------------------------
// residual block reduction: NaN-propagating max and a plain sum
__device__ inline double nanmax(double a, double b)
{
    return (a > b || a != a) ? a : b;
}

__device__ void block_reduce(double &mx, double &sm, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, o));
        sm += __shfl_xor(sm, o);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[2 * wv] = mx;
        sh[2 * wv + 1] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) {
            mx = nanmax(mx, sh[2 * w]);
            sm += sh[2 * w + 1];
        }
    }
}

// Filter pass along direction l (Sec. 3.4), in correction form:
//   (filter matrix) (fh - f) = c_N delta^{2N} f.
// The last direction re-imposes walls/solids and, when the grid has no
// extrapolated faces, also takes the pseudo-step change (Eq. Con-criter)
// and stores the new iterate.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_filter(const GridDev *__restrict__ grids, const Item *__restrict__ items,
         int nitems, int l)
{
    __shared__ T A[kTileMax];
    __shared__ T B[kTileMax];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts pt;
        tile_points(tl, l, pt);
        T *ps = static_cast<T *>(g.ps);
        const int per = g.periodic[l];
        T v0[kPPT], r[kPPT];
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k)) {
                v0[k] = ps[pt.Q[k]];
                A[threadIdx.x + k * kThreads] = v0[k];
            }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPPT; ++k)
            if (pvalid(tl, k))
                r[k] = filter_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per);
        __syncthreads();
        pcr_solve(r, pt, tl, g.fop[l], A, B);
        const bool last = l == g.ndim - 1;
        if (!last) {
#pragma unroll
            for (int k = 0; k < kPPT; ++k)
                if (pvalid(tl, k)) ps[pt.Q[k]] = v0[k] + r[k];
            continue;
        }
        T *phi = static_cast<T *>(g.phi);
        double mx = 0.0, sm = 0.0;
        bool zr[kPPT];
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            zr[k] = true;
            if (!pvalid(tl, k)) continue;
            int idx[3];
            tile_index(g, tl, l, k, pt.J[k], idx);
            zr[k] = wall_point(g, idx) || (g.mask && g.mask[pt.Q[k]]);
            v0[k] = zr[k] ? (T)0 : v0[k] + r[k];
        }
        if (g.fuse_faces) {
#pragma unroll
            for (int k = 0; k < kPPT; ++k)
                if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = v0[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kPPT; ++k)
                if (pvalid(tl, k))
                    v0[k] = face_value(g, l, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj,
                                       v0[k], zr[k]);
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < kPPT; ++k) {
            if (!pvalid(tl, k)) continue;
            const int q = pt.Q[k];
            const T nv = v0[k];
            if (g.fused_resid) {
                const double e = fabs((double)nv - (double)phi[q]);
                mx = nanmax(mx, e);
                sm += e * e;
                phi[q] = nv;
            } else {
                ps[q] = nv;
            }
        }
        if (g.fused_resid) {
            block_reduce(mx, sm, reinterpret_cast<double *>(B));
            if (threadIdx.x == 0) {
                g.rpart[2 * item.tile] = mx;
                g.rpart[2 * item.tile + 1] = sm;
            }
            __syncthreads();
        }
    }
}

// Pseudo-step change and copy of the new iterate (grids whose change is
// not taken by the filter pass).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_resid(const GridDev *__restrict__ grids, const Item *__restrict__ items,
        int nitems)
{
    __shared__ double sh[2 * kThreads / 64];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done) continue;
        T *phi = static_cast<T *>(g.phi);
        const T *ps = static_cast<const T *>(g.ps);
        const long long q0 = (long long)item.tile * kChunk;
        double mx = 0.0, sm = 0.0;
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long q = q0 + i;
            if (q >= g.N) break;
            const T nv = ps[q];
            const double e = fabs((double)nv - (double)phi[q]);
            mx = nanmax(mx, e);
            sm += e * e;
            phi[q] = nv;
        }
        block_reduce(mx, sm, sh);
        if (threadIdx.x == 0) {
            g.rpart[2 * item.tile] = mx;
            g.rpart[2 * item.tile + 1] = sm;
        }
        __syncthreads();
    }
}

// Extrapolated faces (Neumann, outflow): items are (grid, chunk of face
// points); `face` = 2*dir + side; `target` 0 -> phi, 1 -> ps.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_face(const GridDev *__restrict__ grids, const Item *__restrict__ items,
       int nitems, int face, int target)
{
    const int l = face >> 1, side = face & 1;
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (g.state->done && target == 1) continue;
        const int code = g.xbc[face];
        if (code == XBC_NONE) continue;
        T *f = static_cast<T *>(target ? g.ps : g.phi);
        const long long nface = g.N / g.n[l];
        const long long k0 = (long long)item.tile * kChunk;
        const int ib = side ? g.n[l] - 1 : 0;
        const long long in = side ? -g.stride[l] : g.stride[l];
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long k = k0 + i;
            if (k >= nface) break;
            int idx[3];
            const int n0 = g.n[0];
            if (l == 0) {
                idx[0] = ib;
                idx[1] = (int)(k % g.n[1]);
                idx[2] = (int)(k / g.n[1]);
            } else if (l == 1) {
                idx[0] = (int)(k % n0);
                idx[1] = ib;
                idx[2] = (int)(k / n0);
            } else {
                idx[0] = (int)(k % n0);
                idx[1] = (int)(k / n0);
                idx[2] = ib;
            }
            const long long q = idx[0] + (long long)n0 * (idx[1] + (long long)g.n[1] * idx[2]);
            if (wall_point(g, idx) || (g.mask && g.mask[q])) continue;
            const T a = f[q + in], b = f[q + 2 * in];
            f[q] = code == XBC_NEUMANN ? ((T)4 * a - b) / (T)3 : (T)2 * a - b;
        }
    }
}

// Initial field (Sec. 3.5): zero (cold) or the given guess, walls/solids
// set to zero; resets the grid's stopping state.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_init(const GridDev *__restrict__ grids, const Item *__restrict__ items,
       int nitems, int unused)
{
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        T *phi = static_cast<T *>(g.phi);
        if (item.tile == 0 && threadIdx.x == 0) {
            GridState st;
            st.done = 0;
            st.iter = 0;
            st.status = 1;
            st.best_iter = 0;
            st.best = INFINITY;
            st.last = INFINITY;
            *g.state = st;
            *g.mirror = st;
        }
        const long long q0 = (long long)item.tile * kChunk;
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long q = q0 + i;
            if (q >= g.N) break;
            int idx[3];
            index_of(g, q, idx);
            const bool zero = !g.warm || wall_point(g, idx) || (g.mask && g.mask[q]);
            if (zero) phi[q] = (T)0;
        }
    }
}

// Per-grid stopping logic (Eq. Con-criter) on the FP64 partials.
__global__ void __launch_bounds__(kThreads)
k_finalize(const GridDev *__restrict__ grids, int ngrids)
{
    __shared__ double sh[2 * kThreads / 64];
    const GridDev &g = grids[blockIdx.x];
    if (g.state->done) return;
    double mx = 0.0, sm = 0.0;
    for (int i = threadIdx.x; i < g.nparts; i += kThreads) {
        mx = nanmax(mx, g.rpart[2 * i]);
        sm += g.rpart[2 * i + 1];
    }
    block_reduce(mx, sm, sh);
    if (threadIdx.x != 0) return;
    GridState st = *g.state;
    const int it = st.iter;
    const double l2 = sqrt(sm / (double)g.N);
    if (it < g.hist_cap) {
        g.hist[2 * it] = mx;
        g.hist[2 * it + 1] = l2;
    }
    const int nit = it + 1;
    st.iter = nit;
    st.last = mx;
    if (!(fabs(mx) <= 1.0e300) || !(fabs(l2) <= 1.0e300)) {
        st.status = -3;
        st.done = 1;
    } else if (mx <= g.tol) {
        st.status = 0;
        st.done = 1;
    } else {
        if (mx < st.best) {
            st.best = mx;
            st.best_iter = nit;
        }
        if (g.stall > 0 && nit - st.best_iter >= g.stall) {
            st.status = 2;
            st.done = 1;
        } else if (nit >= g.max_iter) {
            st.status = 1;
            st.done = 1;
        }
    }
    *g.state = st;
    *g.mirror = st;   // the host reads the contiguous mirrors after each round
}

// copy every grid's state into the batch mirrors (after a re-plan)
__global__ void k_mirror(const GridDev *__restrict__ grids, int ngrids)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ngrids) *grids[i].mirror = *grids[i].state;
}

// ---------------------------------------------------------------------
// FP64 helpers: precision conversion, metric inversion, Poisson distance.
template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ src, D *__restrict__ dst, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = (D)src[i];
}

// J[(m*d + l)*N + q] = d x_m / d xi_l  ->  out[(l*d + m)*N + q] = d xi_l / d x_m
template <typename T>
__global__ void k_invert(const double *__restrict__ J, T *__restrict__ out, int d,
                         long long N)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N;
         q += (long long)gridDim.x * blockDim.x) {
        double a[3][3];
        for (int m = 0; m < d; ++m)
            for (int l = 0; l < d; ++l) a[m][l] = J[(m * d + l) * N + q];
        double inv[3][3];
        if (d == 2) {
            const double det = a[0][0] * a[1][1] - a[0][1] * a[1][0];
            inv[0][0] = a[1][1] / det;
            inv[0][1] = -a[0][1] / det;
            inv[1][0] = -a[1][0] / det;
            inv[1][1] = a[0][0] / det;
        } else {
            // adjugate / determinant
            const double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
            const double c01 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
            const double c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
            const double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
            inv[0][0] = c00 / det;
            inv[1][0] = c01 / det;
            inv[2][0] = c02 / det;
            inv[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) / det;
            inv[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) / det;
            inv[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) / det;
            inv[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) / det;
            inv[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) / det;
            inv[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) / det;
        }
        for (int l = 0; l < d; ++l)
            for (int m = 0; m < d; ++m) out[(l * d + m) * N + q] = (T)inv[l][m];
    }
}

// distance = 2 phi' / (|grad phi'| + sqrt(|grad phi'|^2 + 2 phi')), the
// cancellation-free form of Eq. Poiss2 with the minus sign, in FP64 from
// g.F[l] (FP64, index space) and the metrics of grid g (T).
template <typename T>
__global__ void k_poisson_dist(const GridDev *__restrict__ gp, const double *__restrict__ phip,
                               T *__restrict__ out)
{
    const GridDev &g = *gp;
    for (long long qq = blockIdx.x * (long long)blockDim.x + threadIdx.x; qq < g.N;
         qq += (long long)gridDim.x * blockDim.x) {
        const int q = (int)qq;
        double s = 0.0;
        for (int m = 0; m < g.ndim; ++m) {
            double u = 0.0;
            for (int l = 0; l < g.ndim; ++l)
                u += (double)metric<T>(g, l, m, q) * static_cast<const double *>(g.F[l])[q];
            s += u * u;
        }
        const double gm = sqrt(s);
        double inner = s + 2.0 * phip[q];
        inner = inner > 0.0 ? inner : 0.0;
        const double den = gm + sqrt(inner);
        out[q] = (T)(den > 0.0 ? 2.0 * phip[q] / den : 0.0);
    }
}

// ---------------------------------------------------------------------
// launchers
template <typename T>
static void line_launch(int kind, const GridDev *g, const Item *it, int nitems,
                        int l, int stage, int nwg, hipStream_t s)
{
    dim3 grid(nwg), block(kThreads);
    switch (kind) {
    case PASS_CART: hipLaunchKernelGGL(k_cart<T>, grid, block, 0, s, g, it, nitems, l, stage); break;
    case PASS_D1: hipLaunchKernelGGL(k_d1<T>, grid, block, 0, s, g, it, nitems, l, stage); break;
    case PASS_D2: hipLaunchKernelGGL(k_d2<T>, grid, block, 0, s, g, it, nitems, l, stage); break;
    case PASS_FILTER: hipLaunchKernelGGL(k_filter<T>, grid, block, 0, s, g, it, nitems, l); break;
    case PASS_FINAL: hipLaunchKernelGGL(k_final<T>, grid, block, 0, s, g, it, nitems, stage); break;
    case PASS_RESID: hipLaunchKernelGGL(k_resid<T>, grid, block, 0, s, g, it, nitems); break;
    case PASS_FACE: hipLaunchKernelGGL(k_face<T>, grid, block, 0, s, g, it, nitems, l, stage); break;
    case PASS_INIT: hipLaunchKernelGGL(k_init<T>, grid, block, 0, s, g, it, nitems, stage); break;
    case PASS_LAD: hipLaunchKernelGGL(k_lad<T>, grid, block, 0, s, g, it, nitems, l, stage); break;
    default: break;
    }
}

void launch_pass(int kind, int fp64, const GridDev *g, const Item *it, int nitems,
                 int l, int stage, int nwg, hipStream_t s)
{
    if (nitems <= 0) return;
    if (nwg > nitems) nwg = nitems;
    if (fp64) line_launch<double>(kind, g, it, nitems, l, stage, nwg, s);
    else line_launch<float>(kind, g, it, nitems, l, stage, nwg, s);
}

void launch_mirror(const GridDev *g, int ngrids, hipStream_t s)
{
    if (ngrids <= 0) return;
    hipLaunchKernelGGL(k_mirror, dim3((ngrids + 255) / 256), dim3(256), 0, s, g, ngrids);
}

void launch_finalize(const GridDev *g, int ngrids, hipStream_t s)
{
    if (ngrids <= 0) return;
    hipLaunchKernelGGL(k_finalize, dim3(ngrids), dim3(kThreads), 0, s, g, ngrids);
}

static int blocks_for(long long n)
{
    long long b = (n + kThreads - 1) / kThreads;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

void launch_convert(int src_fp64, int dst_fp64, const void *src, void *dst,
                    long long n, hipStream_t s)
{
    dim3 grid(blocks_for(n)), block(kThreads);
    if (src_fp64 && dst_fp64)
        hipLaunchKernelGGL((k_convert<double, double>), grid, block, 0, s, (const double *)src, (double *)dst, n);
    else if (src_fp64)
        hipLaunchKernelGGL((k_convert<double, float>), grid, block, 0, s, (const double *)src, (float *)dst, n);
    else if (dst_fp64)
        hipLaunchKernelGGL((k_convert<float, double>), grid, block, 0, s, (const float *)src, (double *)dst, n);
    else
        hipLaunchKernelGGL((k_convert<float, float>), grid, block, 0, s, (const float *)src, (float *)dst, n);
}

void launch_invert(const double *J, void *out, int out_fp64, int d, long long N,
                   hipStream_t s)
{
    dim3 grid(blocks_for(N)), block(kThreads);
    if (out_fp64)
        hipLaunchKernelGGL(k_invert<double>, grid, block, 0, s, J, (double *)out, d, N);
    else
        hipLaunchKernelGGL(k_invert<float>, grid, block, 0, s, J, (float *)out, d, N);
}

void launch_poisson_dist(const GridDev *g, int fp64, long long N, const double *phip,
                         void *out, hipStream_t s)
{
    dim3 grid(blocks_for(N)), block(kThreads);
    if (fp64)
        hipLaunchKernelGGL(k_poisson_dist<double>, grid, block, 0, s, g, phip, (double *)out);
    else
        hipLaunchKernelGGL(k_poisson_dist<float>, grid, block, 0, s, g, phip, (float *)out);
}

}  // namespace wd
