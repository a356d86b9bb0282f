// wd_line.h -- device code of the wall-distance pseudo-time march for
// gfx950: tile geometry, stencils, the line solver and the line-tile
// passes, templated on the value type T and on NP, the number of tile
// points each of the kThreads threads of a workgroup holds.
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
// A tile holds at most kThreads*NP points.  Small tiles (NP * sizeof(T)
// <= 8 bytes) load every per-point operand and every level's line-solve
// multipliers when the tile starts, so a pass waits on memory about once;
// larger tiles keep the register footprint down and load operands where
// they are used.
//
// All kernels take a table of grids and a list of (grid, tile) work items,
// so one launch advances any number of independent grids; a persistent
// workgroup loop walks the items, giving each XCD a contiguous range.
#pragma once

#include "wd_common.h"

#include <cmath>

namespace wd {

// The buffers a GridDev points at are device global memory, but the
// pointers reach the kernels as plain (generic) values read from a table,
// for which the compiler emits FLAT memory instructions.  On this GPU those
// also count against the LDS wait counter, so every wait for an LDS result
// (each barrier of a line solve) would wait for all outstanding global loads
// and stores as well.  Passing the pointers through the global address
// space makes it emit global loads and stores, which LDS waits ignore.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
#else
template <typename T>
using gptr = T *;   // the host pass only parses device code
#endif

template <typename T>
__device__ __forceinline__ gptr<T> gmem(T *p)
{
    return (gptr<T>)p;
}

// gcast<E>(p): the buffer p as a global pointer to E
template <typename E, typename V>
__device__ __forceinline__ gptr<E> gcast(V *p)
{
    return (gptr<E>)p;
}

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

// element i of a global array of (left, right) pairs, as one 2-wide load
template <typename T>
__device__ __forceinline__ typename V2<T>::t ld2(gptr<const typename V2<T>::t> tab, long long i)
{
    typedef T vec2 __attribute__((ext_vector_type(2)));
    const vec2 v = reinterpret_cast<gptr<const vec2>>(tab)[i];
    typename V2<T>::t r;
    r.x = v.x;
    r.y = v.y;
    return r;
}

enum { EQ_EIK = 0, EQ_HJ = 1, EQ_POIS = 2 };
enum { SCH_E2 = 0, SCH_E4 = 1, SCH_E6 = 2, SCH_C4 = 3, SCH_C6 = 4 };

// ---------------------------------------------------------------------
// work distribution
// Workgroups are dealt round-robin to the eight XCDs (workgroup b runs on
// XCD b mod 8), each with its own L2.  Every XCD gets one contiguous range
// of the items, so neighbouring tiles -- which share cache lines when a
// tile holds only a few x-columns -- are fetched into one L2, and its
// workgroups stride through that range.
__device__ inline int item_begin(int nitems, int &step, int &end)
{
    const int b = blockIdx.x, nb = gridDim.x;
    if (nb < 8) {
        step = nb;
        end = nitems;
        return b;
    }
    const int xcd = b & 7, slot = b >> 3;
    const int wpx = (nb - xcd + 7) >> 3;      // workgroups on this XCD
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
    float rn, rwa;   // 1/n, 1/wa for the in-tile quotients
};

// floor(a / b) for 0 <= a, b < 2^13 from a reciprocal rb = 1/b (float):
// (a + 1/2) / b sits at least 1/(2b) from an integer, far more than the
// rounding of the two float operations.
__device__ inline int qdiv(int a, float rb)
{
    return (int)(((float)a + 0.5f) * rb);
}

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
    r.rn = 1.0f / (float)r.n;
    r.rwa = 1.0f / (float)r.wa;
    return r;
}

template <int NP>
struct Pts {
    int J[NP];    // position along the line
    int Q[NP];    // global offset within the grid
};

template <int NP>
__device__ inline void tile_points(const Tile &tl, int l, Pts<NP> &pt)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int p = tid + k * kThreads;
        int j, w;
        if (l == 0) {
            w = qdiv(p, tl.rn);
            j = p - w * tl.n;
        } else {
            j = qdiv(p, tl.rwa);
            w = p - j * tl.wa;
        }
        pt.J[k] = j;
        pt.Q[k] = (int)tl.base + w * (int)tl.gw + j * (int)tl.gj;
    }
}

// position along the line and grid offset of point k of this thread
// (recomputed, for loops that are not unrolled)
__device__ inline void point_jq(const Tile &tl, int l, int k, int &j, int &q)
{
    const int p = (int)threadIdx.x + k * kThreads;
    int w;
    if (l == 0) {
        w = qdiv(p, tl.rn);
        j = p - w * tl.n;
    } else {
        j = qdiv(p, tl.rwa);
        w = p - j * tl.wa;
    }
    q = (int)tl.base + w * (int)tl.gw + j * (int)tl.gj;
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
    const int w = l == 0 ? qdiv(p, tl.rn) : p - j * tl.wa;
    if (l == 0) {
        const int line = (int)tl.rest + w;
        idx[0] = j;
        if (g.ndim == 2) {
            idx[1] = line;
            idx[2] = 0;
        } else {
            // line < 2^31: the double quotient is exact to well within 1/(2 n1)
            const int i2 = (int)(((double)line + 0.5) / (double)g.n[1]);
            idx[1] = line - i2 * g.n[1];
            idx[2] = i2;
        }
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

// wall or solid point k of this thread (phi held at zero there)
__device__ inline bool zero_at(const GridDev &g, const Tile &tl, int l, int k, int j, int q)
{
    int idx[3];
    tile_index(g, tl, l, k, j, idx);
    return wall_point(g, idx) || (g.mask && gmem(g.mask)[q]);
}

template <int NP>
__device__ inline bool zero_point(const GridDev &g, const Tile &tl, int l,
                                  const Pts<NP> &pt, int k)
{
    return zero_at(g, tl, l, k, pt.J[k], pt.Q[k]);
}

// grid indices of point q (grids hold fewer than 2^31 points, so 32-bit
// unsigned division, far shorter than the 64-bit sequence, is exact)
__device__ inline void index_of(const GridDev &g, long long q, int *idx)
{
    const unsigned u = (unsigned)q, n0 = (unsigned)g.n[0], n1 = (unsigned)g.n[1];
    const unsigned r = u / n0;
    idx[0] = (int)(u - r * n0);
    const unsigned r2 = r / n1;
    idx[1] = (int)(r - r2 * n1);
    idx[2] = (int)r2;
}

// metric d xi_l / d x_m at point q
template <typename T>
__device__ inline T metric(const GridDev &g, int l, int m, int q)
{
    if (g.uniform)
        return l == m ? (T)g.invh[l] : (T)0;
    const int d = g.ndim;
    return gcast<const T>(g.met)[(long long)q * (d * d) + l * d + m];
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
            s += c * (pval(X, p, j, 3, n, lj, jump) - pval(X, p, j, -3, n, lj, jump)) * (T)(1.0 / 6.0);
        return s;
    }
    const int p0 = p - j * lj;
    if (g.compact) {
        if (j == 0) {
            return (T)(-17.0 / 6.0) * X[p0] + (T)1.5 * X[p0 + lj]
                   + (T)1.5 * X[p0 + 2 * lj] - X[p0 + 3 * lj] * (T)(1.0 / 6.0);
        }
        if (j == n - 1) {
            const int e = p0 + (n - 1) * lj;
            return -((T)(-17.0 / 6.0) * X[e] + (T)1.5 * X[e - lj]
                     + (T)1.5 * X[e - 2 * lj] - X[e - 3 * lj] * (T)(1.0 / 6.0));
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
            v = ((T)-25 * f[0] + (T)48 * f[1] - (T)36 * f[2] + (T)16 * f[3] - (T)3 * f[4]) * (T)(1.0 / 12.0);
        else if (k == 1)
            v = ((T)-3 * f[0] - (T)10 * f[1] + (T)18 * f[2] - (T)6 * f[3] + f[4]) * (T)(1.0 / 12.0);
        else
            v = (f[0] - (T)8 * f[1] + (T)8 * f[3] - f[4]) * (T)(1.0 / 12.0);
        return hi ? -v : v;
    }
    T s = a * (X[p + lj] - X[p - lj]) * (T)0.5;
    if (r >= 2) s += b * (X[p + 2 * lj] - X[p - 2 * lj]) * (T)0.25;
    if (r >= 3) s += c * (X[p + 3 * lj] - X[p - 3 * lj]) * (T)(1.0 / 6.0);
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

// nine-point truncated Gaussian of Kawai & Lele along a line held in LDS
// (ends clamped on non-periodic lines)
template <typename T>
__device__ T gauss9(const T *X, int p, int j, int n, int lj, int periodic)
{
    const T b[5] = {(T)(3565.0 / 10368.0), (T)(3091.0 / 12960.0),
                    (T)(1997.0 / 25920.0), (T)(149.0 / 12960.0),
                    (T)(107.0 / 103680.0)};
    T acc = (T)0;
#pragma unroll
    for (int o = -4; o <= 4; ++o) {
        int jj = j + o;
        if (periodic) jj += jj < 0 ? n : (jj >= n ? -n : 0);
        else jj = min(max(jj, 0), n - 1);
        acc += b[o < 0 ? -o : o] * X[p + (jj - j) * lj];
    }
    return acc;
}

// ---------------------------------------------------------------------
// Parallel cyclic reduction with precomputed multipliers.
//
// Pcr holds this thread's multipliers of one line operator when the
// thread has one point: the pair of every level and the final scale,
// loaded when the tile starts, so the reduction never waits on memory.
// With more points only the level in use is held (the next one is loaded
// while the current one is applied).  Periodic (circulant) lines use
// per-level scalars and need none.
template <typename T, int NP, bool ALL = (NP == 1)>
struct Pcr {
    using T2 = typename V2<T>::t;
    static constexpr bool kAll = true;
    T2 c[NP][kMaxLev];
    T sc[NP];
};

template <typename T, int NP>
struct Pcr<T, NP, false> {
    static constexpr bool kAll = false;
};

template <typename T, int NP>
__device__ inline void pcr_load(Pcr<T, NP> &pc, const Pts<NP> &pt, const Tile &tl,
                                const LineOpDev &op)
{
    using T2 = typename V2<T>::t;
    if constexpr (Pcr<T, NP>::kAll) {
        if (op.nlev == 0 || op.uniform) return;
        gptr<const T2> tab = gcast<const T2>(op.tab);
        gptr<const T> sc = gcast<const T>(op.scale);
        const int n = tl.n, nlev = op.nlev;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (!pvalid(tl, k)) continue;
            const int j = pt.J[k];
            pc.sc[k] = sc[j];
#pragma unroll
            for (int lev = 0; lev < kMaxLev; ++lev)
                if (lev < nlev) pc.c[k][lev] = ld2<T>(tab, (long long)lev * n + j);
        }
    }
}

// Solve for g <= G right-hand sides of the same line system at once (field
// f uses LDS segment f of A and B, each tl.P long).  On entry v[f] holds
// this thread's right-hand sides (or, with in_lds, they sit in A after a
// barrier), on exit the solutions.  One barrier per level serves all
// fields.  The caller must have finished every read of A and B.
template <typename T, int NP, int G>
__device__ void pcr_multi(T (&v)[G][NP], int g, const Pts<NP> &pt, const Tile &tl,
                          const LineOpDev &op, Pcr<T, NP> &pc, T *A, T *B,
                          bool in_lds = false)
{
    using T2 = typename V2<T>::t;
    constexpr bool kAll = Pcr<T, NP>::kAll;
    const int nlev = op.nlev;
    const int tid = threadIdx.x;
    const int n = tl.n, lj = tl.lj, P = tl.P;
    if (in_lds) {
#pragma unroll
        for (int f = 0; f < G; ++f) {
            if (f >= g) break;
#pragma unroll
            for (int k = 0; k < NP; ++k)
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
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) A[f * P + tid + k * kThreads] = v[f][k];
        }
        __syncthreads();
    }
    T *cur = A, *nxt = B;
    gptr<const T2> tab = gcast<const T2>(op.tab);
    const bool uni = op.uniform;
    T2 cn[kAll ? 1 : NP];   // level in use (larger tiles)
    if (!kAll && !uni) {
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k)) cn[k] = ld2<T>(tab, pt.J[k]);
    }
    auto level = [&](int lev) {
        const int s = op.smod[lev];
        const bool more = lev + 1 < nlev;
        T2 cu;
        cu.x = (T)op.lr[lev][0];
        cu.y = (T)op.lr[lev][1];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (!pvalid(tl, k)) continue;
            const int j = pt.J[k];
            T2 c = cu;
            if (!uni) {
                if constexpr (kAll) {
                    c = pc.c[k][lev];
                } else {
                    c = cn[k];
                    if (more) cn[k] = ld2<T>(tab, (long long)(lev + 1) * n + j);
                }
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
    };
    if constexpr (kAll) {
#pragma unroll
        for (int lev = 0; lev < kMaxLev; ++lev)
            if (lev < nlev) level(lev);
    } else {
        for (int lev = 0; lev < nlev; ++lev) level(lev);
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        if (!pvalid(tl, k)) continue;
        T m;
        if (uni) m = (T)op.usc;
        else if constexpr (kAll) m = pc.sc[k];
        else m = gcast<const T>(op.scale)[pt.J[k]];
#pragma unroll
        for (int f = 0; f < G; ++f)
            if (f < g) v[f][k] *= m;
    }
    __syncthreads();
}

template <typename T, int NP>
__device__ inline void pcr_solve(T (&v)[NP], const Pts<NP> &pt, const Tile &tl,
                                 const LineOpDev &op, Pcr<T, NP> &pc, T *A, T *B)
{
    pcr_multi<T, NP, 1>(reinterpret_cast<T(&)[1][NP]>(v), 1, pt, tl, op, pc, A, B);
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
    return code == XBC_NEUMANN ? ((T)4 * a - b) * (T)(1.0 / 3.0) : (T)2 * a - b;
}

// ---------------------------------------------------------------------
// Pseudo-time update of one point (Sec. 3.3).

// operands of the stage finish that come from memory
template <typename T>
struct FinIn {
    T pn;     // phi^n
    T dt;     // local step (stages > 0)
    T acc;    // RK4 accumulator: the increment so far (stage 0: the
              // remainder the previous iteration's rounding dropped)
};

template <typename T>
__device__ inline FinIn<T> fin_load(const GridDev &g, int stage, int q, T phis)
{
    FinIn<T> r;
    r.pn = stage == 0 ? phis : gcast<const T>(g.phi)[q];
    r.dt = stage == 0 ? (T)0 : gcast<const T>(g.dt)[q];
    r.acc = g.rk == 1 ? gcast<const T>(g.acc)[q] : (T)0;
    return r;
}

// Residual of the chosen equation, local time step at stage 0, RK stage
// combination, walls/solids; returns the new stage value and gives the
// local step to store (stage 0) and the accumulator to store (RK4); the
// caller stores all three.  g2 = |U|^2, adv = U.grad(phi) (= g2 for the
// central schemes; the upwind product for the baseline).  G holds the
// method's fields (eq, lad, curv, rk, eps, nu0, kp, kp2, sigma): the grid
// record itself or a copy of them.
template <typename T, typename G>
__device__ __forceinline__ T finish_core(const G &g, int stage, bool zero, T phis, T g2,
                                         T adv, T lap, T kap, T lads, T S1, T S2,
                                         const FinIn<T> &in, T &dt_out, T &acc_out)
{
    const T gm = sqrt(g2);
    T gam = (T)0, nu = (T)0, R;
    if (g.eq == EQ_HJ) {
        gam = (T)g.eps * phis;
        if (g.lad && lads < gam) gam = lads;   // smoothed C|S| of this iteration
        gam = gam > (T)0 ? gam : (T)0;
        if (g.curv) {
            nu = (T)g.nu0 * ((T)1 - gm) * ((T)1 - gm);
            const T gk = gm * kap;
            R = (T)1 + (gam + nu) * (lap - (gk > (T)0 ? gk : (T)0)) - adv;
        } else {
            R = (T)1 + gam * lap - adv;
        }
    } else if (g.eq == EQ_EIK) {
        R = (T)1 - adv;
    } else {
        R = (T)1 + lap;
    }
    T dt;
    if (stage == 0) {
        const T kp = (T)g.kp, kp2 = (T)g.kp2;
        const T gmx = gm > (T)1 ? gm : (T)1;
        T den;
        if (g.eq == EQ_EIK)
            den = (T)2 * kp * S1 * gmx;
        else if (g.eq == EQ_POIS)
            den = kp2 * kp2 * S2;
        else
            den = (T)2 * kp * S1 * gmx + kp2 * kp2 * (gam + nu) * S2;
        dt = (T)g.sigma / den;
        dt_out = dt;
    } else {
        dt = in.dt;
    }
    const T pn = in.pn;
    T out;
    if (g.rk == 1) {
        // RK4 with the accumulator holding the iteration's increment
        // dt (R1/6 + R2/3 + R3/3 + R4/6), added to phi^n once.  The part of
        // it that this one rounding drops (exactly inc - (out - pn) when
        // |inc| <= |pn|) is kept in the accumulator and starts the next
        // iteration's increment, so a near-converged field does not stall
        // where increments fall below half an ulp of phi (which biases the
        // FP32 fixed point by about ulp(phi) / (2 dt) per point).
        if (stage == 0) {
            acc_out = in.acc + dt * (T)(1.0 / 6.0) * R;
            out = pn + dt * (T)0.5 * R;
        } else if (stage == 1) {
            acc_out = in.acc + dt * (T)(1.0 / 3.0) * R;
            out = pn + dt * (T)0.5 * R;
        } else if (stage == 2) {
            acc_out = in.acc + dt * (T)(1.0 / 3.0) * R;
            out = pn + dt * R;
        } else {
            const T inc = in.acc + dt * (T)(1.0 / 6.0) * R;
            out = pn + inc;
            const T kept = out - pn;
            acc_out = zero ? (T)0 : inc - kept;
        }
    } else {
        if (stage == 0)
            out = pn + dt * R;
        else if (stage == 1)
            out = (T)0.75 * pn + (T)0.25 * (phis + dt * R);
        else
            out = pn * (T)(1.0 / 3.0) + (T)(2.0 / 3.0) * (phis + dt * R);
    }
    return zero ? (T)0 : out;
}

// finish_core with the local step (stage 0) and the RK4 accumulator stored
// at point q; returns the new stage value (the caller stores it).
template <typename T>
__device__ __forceinline__ T finish_point(const GridDev &g, int stage, int q, bool zero, T phis,
                                          T g2, T adv, T lap, T kap, T lads, T S1, T S2,
                                          const FinIn<T> &in)
{
    T dt = (T)0, acc = (T)0;
    const T out = finish_core<T>(g, stage, zero, phis, g2, adv, lap, kap, lads, S1, S2, in, dt, acc);
    if (stage == 0) gcast<T>(g.dt)[q] = dt;
    if (g.rk == 1) gcast<T>(g.acc)[q] = acc;
    return out;
}

// Per-point metric values are kept as m[3*l + c] = d xi_l / d x_c (fixed
// stride, so every index is a compile-time constant after unrolling).

// S1 = sum_l |grad xi_l|, S2 = sum_l |grad xi_l|^2 (d = 2 or 3)
template <typename T>
__device__ inline void metric_sums(int d, const T *m, T &S1, T &S2)
{
    S1 = (T)0;
    S2 = (T)0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l < d) {
            T s2 = (T)0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c < d) {
                    const T e = m[3 * l + c];
                    s2 += e * e;
                }
            }
            S1 += sqrt(s2);
            S2 += s2;
        }
    }
}

// the d*d metric values of point q
template <typename T>
__device__ inline void metric_load(const GridDev &g, int q, T *m)
{
    // values first, stores after the branches join (every slot is written
    // at a fixed index, so the array stays in registers)
    const bool uni = g.uniform != 0;
    T t[9];
    if (g.ndim == 2) {
        T a0, a1, a2, a3;
        if (uni) {
            a0 = (T)g.invh[0];
            a1 = (T)0;
            a2 = (T)0;
            a3 = (T)g.invh[1];
        } else {
            // a point's metrics are contiguous: the loads merge
            gptr<const T> a = gcast<const T>(g.met) + (long long)q * 4;
            a0 = a[0];
            a1 = a[1];
            a2 = a[2];
            a3 = a[3];
        }
        t[0] = a0; t[1] = a1; t[2] = (T)0;
        t[3] = a2; t[4] = a3; t[5] = (T)0;
        t[6] = (T)0; t[7] = (T)0; t[8] = (T)0;
    } else {
        if (uni) {
#pragma unroll
            for (int e = 0; e < 9; ++e) t[e] = (e % 4 == 0) ? (T)g.invh[e / 4] : (T)0;
        } else {
            gptr<const T> a = gcast<const T>(g.met) + (long long)q * 9;
#pragma unroll
            for (int e = 0; e < 9; ++e) t[e] = a[e];
        }
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = t[e];
}

// contravariant pieces U_m = sum_l xi_{l,m} F_l and g2 = |U|^2
template <typename T>
__device__ inline void grad_from(int d, const T *m, const T *F, T *U, T &g2)
{
    g2 = (T)0;
    U[2] = (T)0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (c < d) {
            T u = (T)0;
#pragma unroll
            for (int l = 0; l < 3; ++l)
                if (l < d) u += m[3 * l + c] * F[l];
            U[c] = u;
            g2 += u * u;
        }
    }
}

// Advective term of the upwind baseline at point q (Sec. 3.2.1): along
// each direction the one-sided differences B = phi_i - phi_{i-1},
// F = phi_{i+1} - phi_i of the stage value (periodic lines wrap; at a
// non-periodic end the missing one equals the other); the switch of Eqs.
// UW4-UW5, with n_{i-1} weighing B and n_{i+1} weighing F (B on a rising
// line, F on a falling one, 0 at a minimum, the steeper side on a ridge),
// gives the derivative of Eq. UW3; U_m = sum_l xi_{l,m} phi_l,
// Uh_l = sum_m xi_{l,m} U_m and Eq. UW1 gives
// adv = sum_l [(Uh_l + |Uh_l|) B + (Uh_l - |Uh_l|) F] / 2; g2 = |U|^2.
// m holds the point's metrics as m[3 l + c].
template <typename T>
__device__ void uw_term(const GridDev &g, const T *src, int q, const int *idx, const T *m,
                        T &adv, T &g2)
{
    const int d = g.ndim;
    const T p0 = src[q];
    T Bv[3], Fv[3], D[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        Bv[l] = Fv[l] = D[l] = (T)0;
        if (l >= d) continue;
        const int n = g.n[l], i = idx[l], s = (int)g.stride[l];
        const bool per = g.periodic[l] != 0;
        const bool hm = i > 0 || per, hp = i < n - 1 || per;
        T b = (T)0, f = (T)0;
        if (hm) b = p0 - src[i > 0 ? q - s : q + (n - 1) * s];
        if (hp) f = src[i < n - 1 ? q + s : q - (n - 1) * s] - p0;
        if (!hm) b = f;
        if (!hp) f = b;
        const T sfb = (f + b) >= (T)0 ? (T)1 : (T)-1;
        const T sb = b >= (T)0 ? (T)1 : (T)-1, sf = f >= (T)0 ? (T)1 : (T)-1;
        const T wm = (T)0.25 * ((T)1 + sfb) * ((T)1 + sb);
        const T wp = (T)0.25 * ((T)1 - sfb) * ((T)1 - sf);
        Bv[l] = b;
        Fv[l] = f;
        D[l] = wm * b + wp * f;
    }
    T U[3] = {(T)0, (T)0, (T)0};
    g2 = (T)0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (c >= d) continue;
#pragma unroll
        for (int l = 0; l < 3; ++l)
            if (l < d) U[c] += m[3 * l + c] * D[l];
        g2 += U[c] * U[c];
    }
    adv = (T)0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l >= d) continue;
        T uh = (T)0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (c < d) uh += m[3 * l + c] * U[c];
        adv += (T)0.5 * (uh + fabs(uh)) * Bv[l] + (T)0.5 * (uh - fabs(uh)) * Fv[l];
    }
}

// |grad xi_l| at point q (the LAD sensor's metric factor)
template <typename T>
__device__ inline T grad_xi(const GridDev &g, int l, int q)
{
    T s2 = (T)0;
#pragma unroll
    for (int m = 0; m < 3; ++m)
        if (m < g.ndim) {
            const T e = metric<T>(g, l, m, q);
            s2 += e * e;
        }
    return sqrt(s2);
}

// a[i] for a runtime i in 0..2 without indexing a register array
template <typename T>
__device__ inline T sel3(const T *a, int i)
{
    return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}

// ---------------------------------------------------------------------
// Cartesian pass along direction l (uniform spacing, no curvature): the
// line already holds everything the direction contributes -- U_l = D_l phi,
// D_l U_l -- so one pass per direction suffices; the last direction
// finishes the stage (with the extrapolated faces normal to it, when the
// grid keeps them here).
template <typename T, int NP>
__global__ void __launch_bounds__(kThreads)
k_cart(const GridDev *__restrict__ grids, const Item *__restrict__ items,
       int nitems, int l, int stage)
{
    constexpr int SZ = kThreads * NP;
    constexpr bool kPre = NP * sizeof(T) <= 8;
    __shared__ T A[SZ];
    __shared__ T B[SZ];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts<NP> pt;
        tile_points<NP>(tl, l, pt);
        gptr<const T> src = gcast<const T>(stage == 0 ? g.phi : g.ps);
        const int per = g.periodic[l];
        const bool last = l == g.ndim - 1;
        gptr<T> P0 = gcast<T>(g.P[0]);
        gptr<T> P1 = gcast<T>(g.P[1]);
        gptr<const T> P2 = gcast<const T>(g.P[2]);
        Pcr<T, NP> pc;
        pcr_load(pc, pt, tl, g.dop[l]);
        T v0[NP], r[NP];
        // carried partial sums and finish operands (small tiles: now)
        T pg2[NP], plap[NP], plad[NP];
        FinIn<T> fin[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (!pvalid(tl, k)) continue;
            const int q = pt.Q[k];
            v0[k] = src[q];
            A[threadIdx.x + k * kThreads] = v0[k];
            if constexpr (kPre) {
                pg2[k] = l > 0 ? P0[q] : (T)0;
                plap[k] = (l > 0 && g.need_lap) ? P1[q] : (T)0;
                plad[k] = (last && g.lad) ? P2[q] : (T)0;
                if (last) fin[k] = fin_load<T>(g, stage, q, v0[k]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k))
                r[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per, (T)0);
        __syncthreads();
        pcr_solve<T, NP>(r, pt, tl, g.dop[l], pc, A, B);
        const T ih = (T)g.invh[l];
        T g2c[NP], lapc[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            r[k] *= ih;              // U_l
            g2c[k] = r[k] * r[k];
            lapc[k] = (T)0;
        }
        if (g.need_lap) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = r[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k))
                    lapc[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k],
                                        tl.n, tl.lj, per, (T)0);
            __syncthreads();
            pcr_solve<T, NP>(lapc, pt, tl, g.dop[l], pc, A, B);
#pragma unroll
            for (int k = 0; k < NP; ++k) lapc[k] *= ih;
        }
        if constexpr (!kPre) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const int q = pt.Q[k];
                pg2[k] = l > 0 ? P0[q] : (T)0;
                plap[k] = (l > 0 && g.need_lap) ? P1[q] : (T)0;
            }
        }
        if (!last) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const int q = pt.Q[k];
                P0[q] = l == 0 ? g2c[k] : pg2[k] + g2c[k];
                if (g.need_lap) P1[q] = l == 0 ? lapc[k] : plap[k] + lapc[k];
            }
            continue;
        }
        T S1 = (T)0, S2 = (T)0;
        for (int d = 0; d < g.ndim; ++d) {
            S1 += (T)g.invh[d];
            S2 += (T)g.invh[d] * (T)g.invh[d];
        }
        gptr<T> ps = gcast<T>(g.ps);
        bool zero[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            zero[k] = true;
            if (!pvalid(tl, k)) continue;
            const int q = pt.Q[k];
            if constexpr (!kPre) {
                plad[k] = g.lad ? P2[q] : (T)0;
                fin[k] = fin_load<T>(g, stage, q, v0[k]);
            }
            zero[k] = zero_point(g, tl, l, pt, k);
            const T g2 = pg2[k] + g2c[k];
            const T lap = g.need_lap ? plap[k] + lapc[k] : (T)0;
            v0[k] = finish_point<T>(g, stage, q, zero[k], v0[k], g2, g2, lap, (T)0, plad[k], S1, S2,
                                    fin[k]);
        }
        if (g.fuse_faces) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = v0[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k))
                    v0[k] = face_value(g, l, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj,
                                       v0[k], zero[k]);
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k)) ps[pt.Q[k]] = v0[k];
    }
}

// General pass 1 along direction l: F_l = D_l phi.  At stage 0 of an LAD
// grid it also adds this direction's part of the LAD sensor of phi^n
// (Eq. Gamma_form2), |grad xi_l| d4_l phi, to the sensor field; the first
// such direction (l = 1) starts the sum.
template <typename T, int NP>
__global__ void __launch_bounds__(kThreads)
k_d1(const GridDev *__restrict__ grids, const Item *__restrict__ items,
     int nitems, int l, int stage)
{
    constexpr int SZ = kThreads * NP;
    __shared__ T A[SZ];
    __shared__ T B[SZ];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts<NP> pt;
        tile_points<NP>(tl, l, pt);
        Pcr<T, NP> pc;
        pcr_load(pc, pt, tl, g.dop[l]);
        gptr<const T> src = gcast<const T>(stage == 0 ? g.phi : g.ps);
        const int per = g.periodic[l];
        T r[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = src[pt.Q[k]];
        __syncthreads();
        const T jump = (T)g.jump[l];
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k))
                r[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per, jump);
        if (stage == 0 && g.lad) {
            gptr<T> S = gcast<T>(g.P[2]);
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const int q = pt.Q[k];
                const T t = grad_xi<T>(g, l, q) *
                            fourth_diff(A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per);
                S[q] = l == 1 ? t : S[q] + t;
            }
        }
        __syncthreads();
        pcr_solve<T, NP>(r, pt, tl, g.dop[l], pc, A, B);
        gptr<T> F = gcast<T>(g.F[l]);
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k)) F[pt.Q[k]] = r[k];
    }
}

// General pass 2 along direction l: D_l of U_m (and of n_m for the
// curvature), weighted by xi_{l,m}: the chain-rule Laplacian of Eq.
// Ham_Jac_trans and kappa = div n.  Direction 0 runs first and, with
// FUSED, also computes F_0 = D_0 phi in the same tile (its line is already
// there) before forming U; the last direction finishes the stage.
// At stage 0 of an LAD grid these passes also complete the LAD diffusivity
// of phi^n: direction 0 adds its sensor part, takes C |S| and smooths it
// along 0; every later direction smooths it along itself (the nine-point
// truncated Gaussian, directions in order), the last one before using it.
template <typename T, int NP, bool FUSED>
__global__ void __launch_bounds__(kThreads)
k_d2(const GridDev *__restrict__ grids, const Item *__restrict__ items,
     int nitems, int l, int stage)
{
    // fields per reduction sweep: as many as LDS holds for the tile sizes
    // of this variant (tiles of NP >= 2 hold more than kThreads*NP/2 points)
    constexpr int GM = NP >= 8 ? 1 : (sizeof(T) == 4 ? (NP >= 4 ? 3 : 4) : 2);
    constexpr int SZ = kThreads * NP * GM < kTileMax ? kThreads * NP * GM : kTileMax;
    constexpr bool kPre = NP * sizeof(T) <= 8;
    constexpr int UR = kPre ? NP : 1;            // unroll of per-point loops
    __shared__ T A[SZ];
    __shared__ T B[SZ];
    __shared__ T Cf[(FUSED && !kPre) ? kThreads * NP : 1];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts<NP> pt;
        tile_points<NP>(tl, l, pt);
        const int per = g.periodic[l];
        const int d = g.ndim;
        const int P = tl.P;
        const bool last = l == d - 1;
        gptr<const T> src = gcast<const T>(stage == 0 ? g.phi : g.ps);
        gptr<T> P0 = gcast<T>(g.P[0]);
        gptr<T> P1 = gcast<T>(g.P[1]);
        gptr<const T> P2 = gcast<const T>(g.P[2]);
        Pcr<T, NP> pc;
        pcr_load(pc, pt, tl, g.dop[l]);
        // j, q of point k: from the unrolled table, or recomputed in loops
        // that stay rolled (no dynamic indexing of register arrays)
        auto JQ = [&](int k, int &j, int &q) {
            if constexpr (kPre) {
                j = pt.J[k];
                q = pt.Q[k];
            } else {
                point_jq(tl, l, k, j, q);
            }
        };
        // per-point operands; small tiles load them all now
        T sv[kPre ? NP : 1];
        T Fv[kPre ? NP : 1][3];
        T Mv[kPre ? NP : 1][9];
        T pl[NP], pk[NP], plad[NP];
        bool zr[NP];
        FinIn<T> fin[kPre ? NP : 1];
        const bool ladst = stage == 0 && g.lad;   // this pass updates the LAD field
        gptr<T> Sl = gcast<T>(g.P[2]);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            zr[k] = true;
            if (!pvalid(tl, k)) continue;
            const int q = pt.Q[k];
            if ((FUSED || last) && kPre) sv[k] = src[q];
            if constexpr (kPre) {
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    if (m < d && !(FUSED && m == l)) Fv[k][m] = gcast<const T>(g.F[m])[q];
                metric_load<T>(g, q, Mv[k]);
                pl[k] = l > 0 ? P0[q] : (T)0;
                pk[k] = (l > 0 && g.curv) ? P1[q] : (T)0;
                if (last || ladst) plad[k] = g.lad ? P2[q] : (T)0;
                if (last) {
                    zr[k] = zero_point(g, tl, l, pt, k);
                    fin[k] = fin_load<T>(g, stage, q, sv[k]);
                }
            }
        }
        if (FUSED && g.uw) {
            // upwind advective term of the stage value (Eqs. UW1-UW5): its
            // stencil reaches across tiles, so it is formed here, in a pass
            // that does not write the stage value, for the last pass's finish
            gptr<T> adv = gcast<T>(g.P[1]);
            gptr<T> u2 = gcast<T>(g.uw2);
#pragma unroll UR
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                int j, q;
                JQ(k, j, q);
                int idx[3];
                tile_index(g, tl, l, k, j, idx);
                T m9[9], a, g2;
                if constexpr (kPre) {
#pragma unroll
                    for (int c = 0; c < 9; ++c) m9[c] = Mv[k][c];
                } else {
                    metric_load<T>(g, q, m9);
                }
                uw_term<T>(g, src, q, idx, m9, a, g2);
                adv[q] = a;
                u2[q] = g2;
            }
        }
        if (ladst && !FUSED) {
            // smooth the LAD field along l (tile lines) before it is used
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) {
                    if constexpr (kPre) A[threadIdx.x + k * kThreads] = plad[k];
                    else A[threadIdx.x + k * kThreads] = P2[pt.Q[k]];
                }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const T sm = gauss9(A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per);
                Sl[pt.Q[k]] = sm;
                plad[k] = sm;
            }
            // A is next written after the barrier that follows the field phase
        }
        if constexpr (FUSED) {
            // F_l = D_l phi on the tile's lines
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) {
                    if constexpr (kPre) A[threadIdx.x + k * kThreads] = sv[k];
                    else A[threadIdx.x + k * kThreads] = src[pt.Q[k]];
                }
            __syncthreads();
            const T jump = (T)g.jump[l];
            T fl[NP], lv[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k))
                    fl[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj,
                                      per, jump);
            if (ladst) {
                // sensor part of direction 0 added to the others, then C |S|
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    if (!pvalid(tl, k)) continue;
                    const int q = pt.Q[k];
                    const T t = grad_xi<T>(g, l, q) *
                                fourth_diff(A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per);
                    T rest;
                    if constexpr (kPre) rest = plad[k];
                    else rest = P2[q];
                    lv[k] = (T)g.C * fabs(d > 1 ? t + rest : t);
                }
            }
            __syncthreads();
            pcr_solve<T, NP>(fl, pt, tl, g.dop[l], pc, A, B);
            if (ladst) {
                // smoothing along 0 (A and B are free after the solve)
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = lv[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k))
                        Sl[pt.Q[k]] = gauss9(A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per);
                // A is next written after the barrier that follows the field phase
            }
            gptr<T> Fl = gcast<T>(g.F[l]);
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                Fl[pt.Q[k]] = fl[k];
                if constexpr (kPre) {
#pragma unroll
                    for (int m = 0; m < 3; ++m)
                        if (m == l) Fv[k][m] = fl[k];
                } else {
                    Cf[threadIdx.x + k * kThreads] = fl[k];   // read back by this thread only
                }
            }
        }
        // fields differentiated along l: U_m (and n_m), weighted by xi_{l,m};
        // field f is coded in bits 3f..3f+2 of `code` (component m, n-flag)
        int code = 0, nf = 0;
        for (int f = 0; f < (g.curv ? 2 * d : d); ++f) {
            const int m = f % d;
            if (g.uniform && m != l) continue;
            code |= (m | ((f >= d) << 2)) << (3 * nf);
            ++nf;
        }
        const int G = min(GM, max(1, SZ / P));
        T lapc[NP], kapc[NP], g2s[kPre ? NP : 1];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            lapc[k] = (T)0;
            kapc[k] = (T)0;
        }
        for (int f0 = 0; f0 < nf; f0 += G) {
            const int gcount = min(G, nf - f0);
            // field values of this group into B, point by point
#pragma unroll UR
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const int p = threadIdx.x + k * kThreads;
                T U[3], g2;
                if constexpr (kPre) {
                    grad_from<T>(d, Mv[k], Fv[k], U, g2);
                } else {
                    int j, q;
                    JQ(k, j, q);
                    T m9[9], F3[3];
                    metric_load<T>(g, q, m9);
#pragma unroll
                    for (int m = 0; m < 3; ++m)
                        if (m < d) F3[m] = (FUSED && m == l) ? Cf[p]
                                                             : gcast<const T>(g.F[m])[q];
                    grad_from<T>(d, m9, F3, U, g2);
                }
                if constexpr (kPre) g2s[k] = g2;
                const T inv = (T)1 / (sqrt(g2) + (T)g.eps0);
                for (int f = 0; f < gcount; ++f) {
                    const int c = code >> (3 * (f0 + f));
                    const int m = c & 3;
                    const T u = m == 0 ? U[0] : (m == 1 ? U[1] : U[2]);
                    B[f * P + p] = (c & 4) ? u * inv : u;
                }
            }
            __syncthreads();
            // right-hand sides from B into A
            for (int f = 0; f < gcount; ++f)
#pragma unroll 1
                for (int k = 0; k < NP; ++k) {
                    if (!pvalid(tl, k)) break;
                    const int p = threadIdx.x + k * kThreads;
                    int j, q;
                    point_jq(tl, l, k, j, q);
                    A[f * P + p] = deriv_rhs(g, B + f * P, p, j, tl.n, tl.lj, per, (T)0);
                }
            __syncthreads();
            T v[GM][NP];
            pcr_multi<T, NP, GM>(v, gcount, pt, tl, g.dop[l], pc, A, B, true);
#pragma unroll
            for (int f = 0; f < GM; ++f) {
                if (f >= gcount) break;
                const int c = code >> (3 * (f0 + f));
                const int m = c & 3;
                const bool isn = (c & 4) != 0;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    if (!pvalid(tl, k)) continue;
                    T wgt;
                    if constexpr (kPre) {
                        T row[3];
#pragma unroll
                        for (int c2 = 0; c2 < 3; ++c2)
                            row[c2] = l == 0 ? Mv[k][c2] : (l == 1 ? Mv[k][3 + c2] : Mv[k][6 + c2]);
                        wgt = sel3(row, m);
                    } else {
                        wgt = metric<T>(g, l, m, pt.Q[k]);
                    }
                    if (isn) kapc[k] += wgt * v[f][k];
                    else lapc[k] += wgt * v[f][k];
                }
            }
        }
        if (!last) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const int q = pt.Q[k];
                if constexpr (!kPre) {
                    pl[k] = l > 0 ? P0[q] : (T)0;
                    pk[k] = (l > 0 && g.curv) ? P1[q] : (T)0;
                }
                P0[q] = l == 0 ? lapc[k] : pl[k] + lapc[k];
                if (g.curv) P1[q] = l == 0 ? kapc[k] : pk[k] + kapc[k];
            }
            continue;
        }
        gptr<T> ps = gcast<T>(g.ps);
        // the next stage's F_l = D_l of the new stage value, from the
        // tile's whole lines (the next stage's pass along l skips the grid)
        const bool fnext = g.fnext && stage < g.stages - 1;
        const T jump = (T)g.jump[l];
        if constexpr (kPre) {
            T nv[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const T lap = pl[k] + lapc[k];
                const T kap = g.curv ? pk[k] + kapc[k] : (T)0;
                T S1, S2;
                metric_sums<T>(d, Mv[k], S1, S2);
                T g2 = g2s[k], adv = g2s[k];
                if (g.uw) {   // formed by the fused pass along 0
                    adv = gcast<const T>(g.P[1])[pt.Q[k]];
                    g2 = gcast<const T>(g.uw2)[pt.Q[k]];
                }
                nv[k] = finish_point<T>(g, stage, pt.Q[k], zr[k], sv[k], g2, adv, lap, kap,
                                        plad[k], S1, S2, fin[k]);
            }
            if (g.fuse_faces) {
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = nv[k];
                __syncthreads();
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k))
                        nv[k] = face_value(g, l, A, threadIdx.x + k * kThreads, pt.J[k], tl.n,
                                           tl.lj, nv[k], zr[k]);
            }
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) ps[pt.Q[k]] = nv[k];
            if (fnext) {
                __syncthreads();   // the face step's reads of A are done
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = nv[k];
                __syncthreads();
                T fl[NP];
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k))
                        fl[k] = deriv_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj,
                                          per, jump);
                __syncthreads();
                pcr_solve<T, NP>(fl, pt, tl, g.dop[l], pc, A, B);
                gptr<T> Fl = gcast<T>(g.F[l]);
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k)) Fl[pt.Q[k]] = fl[k];
            }
        } else {
            // park the partial sums in LDS (own points only) and finish the
            // stage point by point, keeping the unrolled state small
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) {
                    A[threadIdx.x + k * kThreads] = lapc[k];
                    B[threadIdx.x + k * kThreads] = kapc[k];
                }
#pragma unroll 1
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) break;
                const int p = threadIdx.x + k * kThreads;
                int j, q;
                JQ(k, j, q);
                const T lap = l == 0 ? A[p] : P0[q] + A[p];
                const T kap = g.curv ? (l == 0 ? B[p] : P1[q] + B[p]) : (T)0;
                const T lads = g.lad ? P2[q] : (T)0;
                const bool zero = zero_at(g, tl, l, k, j, q);
                T m9[9], F3[3], U[3], g2;
                metric_load<T>(g, q, m9);
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    if (m < d) F3[m] = gcast<const T>(g.F[m])[q];
                grad_from<T>(d, m9, F3, U, g2);
                T adv = g2;
                if (g.uw) {   // formed by the fused pass along 0
                    adv = gcast<const T>(g.P[1])[q];
                    g2 = gcast<const T>(g.uw2)[q];
                }
                T S1, S2;
                metric_sums<T>(d, m9, S1, S2);
                const T phis = src[q];
                const FinIn<T> fi = fin_load<T>(g, stage, q, phis);
                const T nv = finish_point<T>(g, stage, q, zero, phis, g2, adv, lap, kap, lads, S1,
                                             S2, fi);
                B[p] = zero ? (T)1 : (T)0;   // wall flag for the face step
                A[p] = nv;
                if (!g.fuse_faces) ps[q] = nv;
            }
            if (g.fuse_faces) {
                __syncthreads();
#pragma unroll 1
                for (int k = 0; k < NP; ++k) {
                    if (!pvalid(tl, k)) break;
                    const int p = threadIdx.x + k * kThreads;
                    int j, q;
                    JQ(k, j, q);
                    const T fv = face_value(g, l, A, p, j, tl.n, tl.lj, A[p], B[p] != (T)0);
                    ps[q] = fv;
                    B[p] = fv;   // own slot: read just above by this thread only
                }
            }
            if (fnext) {
                // the new stage values sit in A (or, after the face step, in B)
                const T *X = g.fuse_faces ? B : A;
                __syncthreads();
                T fl[NP];
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k))
                        fl[k] = deriv_rhs(g, X, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj,
                                          per, jump);
                __syncthreads();
                pcr_solve<T, NP>(fl, pt, tl, g.dop[l], pc, A, B);
                gptr<T> Fl = gcast<T>(g.F[l]);
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k)) Fl[pt.Q[k]] = fl[k];
            }
        }
        __syncthreads();
    }
}

// LAD diffusivity of Eq. Gamma_form2, once per pseudo iteration from
// phi^n.  phase 0, direction l: S += |grad xi_l| d4_l phi; on the grid's
// last direction S <- C |S|, then smoothed along that same direction in
// the tile.  phase 1, direction l < last: smoothing of S along l.  The
// smoothing is the nine-point truncated Gaussian of Kawai & Lele (ends
// clamped on non-periodic lines); its directional sweeps commute.
template <typename T, int NP>
__global__ void __launch_bounds__(kThreads)
k_lad(const GridDev *__restrict__ grids, const Item *__restrict__ items,
      int nitems, int l, int phase)
{
    __shared__ T A[kThreads * NP];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts<NP> pt;
        tile_points<NP>(tl, l, pt);
        const int per = g.periodic[l];
        gptr<T> S = gcast<T>(g.P[2]);
        gptr<const T> src = phase == 0 ? gcast<const T>(g.phi) : S;
        const bool last = l == g.ndim - 1;
        T sp[NP], w[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (!pvalid(tl, k)) continue;
            const int q = pt.Q[k];
            A[threadIdx.x + k * kThreads] = src[q];
            if (phase == 0) {
                sp[k] = l != 0 ? S[q] : (T)0;
                T s2 = (T)0;
                for (int m = 0; m < g.ndim; ++m) {
                    const T e = metric<T>(g, l, m, q);
                    s2 += e * e;
                }
                w[k] = sqrt(s2);
            }
        }
        __syncthreads();
        if (phase == 0) {
            T v[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (!pvalid(tl, k)) continue;
                const int p = threadIdx.x + k * kThreads;
                v[k] = w[k] * fourth_diff(A, p, pt.J[k], tl.n, tl.lj, per);
                if (l != 0) v[k] += sp[k];
            }
            if (!last) {
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    if (pvalid(tl, k)) S[pt.Q[k]] = v[k];
                __syncthreads();
                continue;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = (T)g.C * fabs(v[k]);
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k))
                S[pt.Q[k]] = gauss9(A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------
// residual block reduction: NaN-propagating max and a plain sum
__device__ inline double nanmax(double a, double b)
{
    return (a > b || a != a) ? a : b;
}

// The FP64 partials of one tile or chunk, reduced over the workgroup into
// thread 0: largest change mx, sum of squared changes sm, and of the new
// field the largest -phi (ng) and the largest |phi| (mg).  sh holds
// 4 * kThreads / 64 doubles.
__device__ inline void block_reduce(double &mx, double &sm, double &ng, double &mg, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) {
        mx = nanmax(mx, __shfl_xor(mx, o));
        sm += __shfl_xor(sm, o);
        ng = nanmax(ng, __shfl_xor(ng, o));
        mg = nanmax(mg, __shfl_xor(mg, o));
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[4 * wv] = mx;
        sh[4 * wv + 1] = sm;
        sh[4 * wv + 2] = ng;
        sh[4 * wv + 3] = mg;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) {
            mx = nanmax(mx, sh[4 * w]);
            sm += sh[4 * w + 1];
            ng = nanmax(ng, sh[4 * w + 2]);
            mg = nanmax(mg, sh[4 * w + 3]);
        }
    }
}

// a tile's or chunk's partials into rpart (thread 0)
__device__ inline void put_rpart(const GridDev &g, int part, double mx, double sm, double ng,
                                 double mg)
{
    gptr<double> r = gmem(g.rpart) + 4 * (long long)part;
    r[0] = mx;
    r[1] = sm;
    r[2] = ng;
    r[3] = mg;
}

// Filter pass along direction l (Sec. 3.4), in correction form:
//   (filter matrix) (fh - f) = c_N delta^{2N} f.
// The last direction re-imposes walls/solids and, when the grid has no
// extrapolated faces outside this pass, also takes the pseudo-step change
// (Eq. Con-criter) and stores the new iterate.
template <typename T, int NP>
__global__ void __launch_bounds__(kThreads)
k_filter(const GridDev *__restrict__ grids, const Item *__restrict__ items,
         int nitems, int l)
{
    constexpr int SZ = kThreads * NP;
    constexpr bool kPre = NP * sizeof(T) <= 8;
    __shared__ T A[SZ];
    __shared__ __align__(16) T B[SZ];   // also the FP64 reduction scratch
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const Tile tl = decode_tile(g, l, item.tile);
        Pts<NP> pt;
        tile_points<NP>(tl, l, pt);
        Pcr<T, NP> pc;
        pcr_load(pc, pt, tl, g.fop[l]);
        gptr<T> ps = gcast<T>(g.ps);
        gptr<T> phi = gcast<T>(g.phi);
        const int per = g.periodic[l];
        const bool last = l == g.ndim - 1;
        const bool resid = last && g.fused_resid;
        T v0[NP], r[NP], pold[NP];
        bool zr[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            zr[k] = true;
            if (!pvalid(tl, k)) continue;
            v0[k] = ps[pt.Q[k]];
            A[threadIdx.x + k * kThreads] = v0[k];
            if constexpr (kPre) {
                if (resid) pold[k] = phi[pt.Q[k]];
                if (last) zr[k] = zero_point(g, tl, l, pt, k);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NP; ++k)
            if (pvalid(tl, k))
                r[k] = filter_rhs(g, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj, per);
        __syncthreads();
        pcr_solve<T, NP>(r, pt, tl, g.fop[l], pc, A, B);
        if (!last) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) ps[pt.Q[k]] = v0[k] + r[k];
            continue;
        }
        double mx = 0.0, sm = 0.0, ng = 0.0, mg = 0.0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (!pvalid(tl, k)) continue;
            if constexpr (!kPre) zr[k] = zero_point(g, tl, l, pt, k);
            v0[k] = zr[k] ? (T)0 : v0[k] + r[k];
        }
        if (g.fuse_faces) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k)) A[threadIdx.x + k * kThreads] = v0[k];
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (pvalid(tl, k))
                    v0[k] = face_value(g, l, A, threadIdx.x + k * kThreads, pt.J[k], tl.n, tl.lj,
                                       v0[k], zr[k]);
            __syncthreads();
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (!pvalid(tl, k)) continue;
            const int q = pt.Q[k];
            const T nv = v0[k];
            if (resid) {
                if constexpr (!kPre) pold[k] = phi[q];
                const double e = fabs((double)nv - (double)pold[k]);
                mx = nanmax(mx, e);
                sm += e * e;
                ng = nanmax(ng, -(double)nv);
                mg = nanmax(mg, fabs((double)nv));
                phi[q] = nv;
            } else {
                ps[q] = nv;
            }
        }
        if (resid) {
            block_reduce(mx, sm, ng, mg, reinterpret_cast<double *>(B));
            if (threadIdx.x == 0) put_rpart(g, item.tile, mx, sm, ng, mg);
            __syncthreads();
        }
    }
}

}  // namespace wd
