// wd_seg.h -- segmented line passes for uniform Cartesian grids (gfx950).
//
// The compact derivative (Sec. 3.2) and the implicit filter (Sec. 3.4)
// need one tridiagonal solve per grid line; the LAD sensor and its
// smoothing (Eq. Gamma_form2) need short stencils along the line.  Here a
// workgroup is ONE wave and its tile is W whole lines of one direction.
// Every line is cut into S segments of M positions (M a compile-time 16,
// 24 or 32; one segment may be shorter); lane (w, s) owns segment s of
// line w and keeps it in registers:
//
//   window    the segment and kSegH neighbours on each side, read from the
//             tile's line buffer in LDS (the only data LDS holds)
//   forward   y_i = r_i - ell_i y_{i-1}      (r from the stencil on the window)
//   backward  x_i = ib_i y_i - cb_i x_{i+1}  (local solve of the segment)
//   reduce    the true values at the neighbouring segments' ends are fixed
//             linear combinations (host-inverted reduced system) of every
//             segment's local end values, gathered by cross-lane shuffles
//   correct   x_i -= vv_i * last_{s-1} + ww_i * first_{s+1}
//
// Every loop over a segment is unrolled at compile time, so the sweeps are
// register FMA chains whose table reads (LDS) the compiler issues early;
// no barrier sits inside a solve.  Each lane also reads and writes the
// grid fields of its own segment directly (the lanes of a step cover runs
// of W x-columns along directions 1 and 2), up to M loads in flight, and
// the extrapolated faces at a line's ends are fixed inside the end
// segments' registers.
#pragma once

#include "wd_line.h"

namespace wd {

constexpr int kSegH = 5;          // window positions beyond each segment end
constexpr int kSegThreads = 64;   // one wave per workgroup

// floor(a / b) from rb = 1/b (float) for 0 <= a < 2^22: (a + 1/2)/b lies
// at least 1/(2b) from an integer, the two roundings move it by less.
__device__ inline int sdiv(int a, float rb)
{
    return (int)(((float)a + 0.5f) * rb);
}

// segment of line position j
template <int M>
__device__ inline int seg_of(const SegGeo &sg, int j)
{
    if (j < sg.bk) return j / M;
    if (j < sg.bk + sg.r) return sg.ks;
    return sg.ks + 1 + (j - sg.bk - sg.r) / M;
}

// LDS slot of line w, position j: lines sg.P apart, position j shifted by
// its segment index so the lanes of a step spread over the banks
template <int M>
__device__ inline int seg_slot(const SegGeo &sg, int w, int j)
{
    return w * sg.P + j + seg_of<M>(sg, j);
}

// this lane's segment
struct SegLane {
    int w, s;        // line in the tile (0 for idle lanes), segment
    int b, len;      // first line position, positions in the segment
    bool act;        // a lane of the W x S grid
};

template <int M>
__device__ inline void seg_lane(const SegGeo &sg, SegLane &L)
{
    const int lane = threadIdx.x;
    L.act = lane < sg.W * sg.S;
    const int w = lane / sg.S, s = lane - w * sg.S;
    L.w = L.act ? w : 0;
    L.s = L.act ? s : 0;
    if (L.s < sg.ks) {
        L.b = L.s * M;
        L.len = M;
    } else if (L.s == sg.ks) {
        L.b = sg.bk;
        L.len = sg.r;
    } else {
        L.b = sg.bk + sg.r + (L.s - sg.ks - 1) * M;
        L.len = M;
    }
}

template <typename T>
__device__ inline void seg_tables(const SegOpDev &op, T *tb)
{
    if (!op.solve) return;
    const int ntab = seg_table_len(op.n, op.S);
    gptr<const T> src = gcast<const T>(op.tab);
    for (int k = threadIdx.x; k < ntab; k += kSegThreads) tb[k] = src[k];
}

// write this lane's segment values to the line buffer
template <typename T, int M>
__device__ inline void seg_put(const SegGeo &sg, const SegLane &L, T *X, const T (&x)[M])
{
    if (!L.act) return;
    if (L.len == M) {
        const int base = seg_slot<M>(sg, L.w, L.b);
#pragma unroll
        for (int i = 0; i < M; ++i) X[base + i] = x[i];
        return;
    }
#pragma unroll
    for (int i = 0; i < M; ++i)
        if (i < L.len) X[seg_slot<M>(sg, L.w, L.b + i)] = x[i];
}

// the window of a lane: v[k] = line position b - kSegH + k (wrapped on
// periodic lines, clamped at the ends of others, where the one-sided rows
// do not use it).  When every segment is full (ks == S) the slots follow
// from the lane's base with compile-time offsets.
template <typename T, int M>
__device__ inline void seg_window(const SegGeo &sg, const SegLane &L, int n, int per,
                                  const T *X, T (&v)[M + 2 * kSegH])
{
    constexpr int H = kSegH;
    if (sg.ks == sg.S) {
        const int base = L.w * sg.P + L.s * (M + 1) - H;
        const bool first = L.s == 0, lastseg = L.s == sg.S - 1;
#pragma unroll
        for (int k = 0; k < M + 2 * H; ++k) {
            const int d = k < H ? -1 : (k < M + H ? 0 : 1);
            int sl = base + k + d;
            if (k < H && first)        // position k - H < 0
                sl = per ? L.w * sg.P + n + sg.S - 1 + k - H : L.w * sg.P;
            if (k >= M + H && lastseg)  // position n + k - M - H
                sl = per ? L.w * sg.P + k - M - H : L.w * sg.P + n - 1 + sg.S - 1;
            v[k] = X[sl];
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < M + 2 * H; ++k) {
        int p = L.b - H + k;
        if (p < 0) p = per ? p + n : 0;
        else if (p >= n) p = per ? p - n : n - 1;
        v[k] = X[seg_slot<M>(sg, L.w, p)];
    }
}

// ---------------------------------------------------------------------
// Right-hand sides on the window, position i of the segment (line
// position b + i).  lo: the segment starts the line (non-periodic), so
// positions i < 5 are the line's first rows; hi: it ends the line, full,
// so positions M-5.. are its last rows.  Index-space stencils.

// first derivative (Sec. 3.2) at every position of the segment: the
// interior stencil, then the one-sided rows where the segment holds the
// line's first (lo) or last (hi) positions.  x[i] for i >= len is zero.
template <typename T, int M>
__device__ inline void seg_deriv_all(const GridDev &g, const T (&v)[M + 2 * kSegH], int len,
                                     bool lo, bool hi, T (&x)[M])
{
    constexpr int H = kSegH;
    const int r = g.dradius;
    const T a = (T)(0.5 * g.da), b = (T)(0.25 * g.db), c = (T)(g.dc / 6.0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
        T s = a * (v[H + i + 1] - v[H + i - 1]);
        if (r >= 2) s += b * (v[H + i + 2] - v[H + i - 2]);
        if (r >= 3) s += c * (v[H + i + 3] - v[H + i - 3]);
        x[i] = i < len ? s : (T)0;
    }
    if (!lo && !hi) return;
    // one-sided rows, at index distance k from the line end (sign: +1 at
    // the first end, -1 at the last, mirrored)
    auto row = [&](const T *f, int k) -> T {
        if (g.compact) {
            if (k == 0)
                return (T)(-17.0 / 6.0) * f[0] + (T)1.5 * f[1] + (T)1.5 * f[2] -
                       f[3] * (T)(1.0 / 6.0);
            return (T)0.75 * (f[2] - f[0]);   // C6 row next to the end (k == 1)
        }
        if (g.scheme == SCH_E2) return ((T)-3 * f[0] + (T)4 * f[1] - f[2]) * (T)0.5;
        if (k == 0)
            return ((T)-25 * f[0] + (T)48 * f[1] - (T)36 * f[2] + (T)16 * f[3] - (T)3 * f[4]) *
                   (T)(1.0 / 12.0);
        if (k == 1)
            return ((T)-3 * f[0] - (T)10 * f[1] + (T)18 * f[2] - (T)6 * f[3] + f[4]) *
                   (T)(1.0 / 12.0);
        return (f[0] - (T)8 * f[1] + (T)8 * f[3] - f[4]) * (T)(1.0 / 12.0);
    };
    // rows 0..nr-1 from each end take the one-sided forms
    const int nr = g.compact ? (g.scheme == SCH_C6 ? 2 : 1) : r;
    if (lo) {
        T f[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) f[t] = v[H + t];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < nr) x[k] = row(f, k);
    }
    if (hi) {
        T f[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) f[t] = v[H + M - 1 - t];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < nr) x[M - 1 - k] = -row(f, k);
    }
}

// c_N delta^{2N} f at window centre c (compile-time N and c)
template <typename T, int M>
__device__ inline T seg_delta(const GridDev &g, const T (&v)[M + 2 * kSegH], int c, int N)
{
    T s = (T)0;
    int bc = 1;
#pragma unroll
    for (int k = 0; k <= 10; ++k) {
        if (k > 2 * N) break;
        s += (T)((k & 1) ? -bc : bc) * v[c - N + k];
        bc = bc * (2 * N - k) / (k + 1);
    }
    return (T)g.fcoef[N] * s;
}

// filter correction c_N delta^{2N} f (Sec. 3.4) at every position: N = 5
// inside, N = the distance to the line end near it, 0 on the end point
template <typename T, int M>
__device__ inline void seg_frhs_all(const GridDev &g, const T (&v)[M + 2 * kSegH], int len,
                                    bool lo, bool hi, T (&x)[M])
{
    constexpr int H = kSegH;
    const T f5 = (T)g.fcoef[5];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int c = H + i;
        const T s = (v[c - 5] + v[c + 5]) - (T)10 * (v[c - 4] + v[c + 4]) +
                    (T)45 * (v[c - 3] + v[c + 3]) - (T)120 * (v[c - 2] + v[c + 2]) +
                    (T)210 * (v[c - 1] + v[c + 1]) - (T)252 * v[c];
        x[i] = i < len ? f5 * s : (T)0;
    }
    if (lo) {
        x[0] = (T)0;
#pragma unroll
        for (int i = 1; i < 5; ++i) x[i] = seg_delta<T, M>(g, v, H + i, i);
    }
    if (hi) {
        x[M - 1] = (T)0;
#pragma unroll
        for (int k = 1; k < 5; ++k) x[M - 1 - k] = seg_delta<T, M>(g, v, H + M - 1 - k, k);
    }
}

// five-point fourth difference, copied inward of the two end points
template <typename T, int M>
__device__ inline T seg_fourth(const T (&v)[M + 2 * kSegH], int i, bool lo, bool hi)
{
    constexpr int H = kSegH;
    auto d4 = [&](int c) {
        return v[c - 2] - (T)4 * v[c - 1] + (T)6 * v[c] - (T)4 * v[c + 1] + v[c + 2];
    };
    if (i < 2 && lo) return d4(H + 2);
    if (i > M - 3 && hi) return d4(H + M - 3);
    return d4(H + i);
}

// nine-point truncated Gaussian, ends clamped
template <typename T, int M>
__device__ inline T seg_gauss9(const T (&v)[M + 2 * kSegH], int i, bool lo, bool hi)
{
    const T b[5] = {(T)(3565.0 / 10368.0), (T)(3091.0 / 12960.0), (T)(1997.0 / 25920.0),
                    (T)(149.0 / 12960.0), (T)(107.0 / 103680.0)};
    constexpr int H = kSegH;
    T acc = b[0] * v[H + i];
#pragma unroll
    for (int o = 1; o <= 4; ++o) {
        const T vm = (i - o < 0 && lo) ? v[H] : v[H + i - o];
        const T vp = (i + o > M - 1 && hi) ? v[H + M - 1] : v[H + i + o];
        acc += b[o] * (vm + vp);
    }
    return acc;
}

// ---------------------------------------------------------------------
// x = scale * A^{-1} r for this lane's segment, r in x for i < len
// (explicit schemes: x = scale * r).  Every lane of the wave must call it
// (the reduction shuffles across lanes).
template <typename T, int M>
__device__ inline void seg_solve(const SegGeo &sg, const SegOpDev &op, const T *tb,
                                 const SegLane &L, T scale, T (&x)[M])
{
    if (!op.solve) {
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] *= scale;
        return;
    }
    const int n2 = op.n + op.S, sb = L.b + L.s;   // the segment's table entries
    const T *ell = tb + sb, *ib = tb + n2 + sb, *cb = tb + 2 * n2 + sb;
    const T *vv = tb + 3 * n2 + sb, *ww = tb + 4 * n2 + sb;
    // rows i >= len (a short segment) read the next segment's table entries
    // and a zero right-hand side; the segment's own last row has cb = 0, so
    // they never reach it, and they are not stored
    T y = (T)0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        y = x[i] - ell[i] * y;
        x[i] = y;
    }
    T z = (T)0, zl = (T)0;
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        z = ib[i] * x[i] - cb[i] * z;
        x[i] = z;
        zl = i == L.len - 1 ? z : zl;
    }
    const T zf = x[0];
    T lp = (T)0, fn = (T)0;
    const int S = sg.S;
    if (S > 1 || op.periodic) {
        const T *red = tb + 5 * n2 + L.s * (4 * S + 1);
        const int base = L.w * S;
        for (int k = 0; k < S; ++k) {
            const T f = __shfl(zf, base + k, kSegThreads);
            const T la = __shfl(zl, base + k, kSegThreads);
            lp += red[k] * f + red[S + k] * la;
            fn += red[2 * S + k] * f + red[3 * S + k] * la;
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i)
        x[i] = (x[i] - vv[i] * lp - ww[i] * fn) * scale;
}

// where lane's segment sits in the grid: offset of position 0, stride
// along the line, and the lane's fixed grid indices (the index along l is
// the line position)
struct SegPos {
    int q0, gj;
    int idx[3];
    bool ok;     // a lane with a real segment of a line in the tile
};

__device__ inline void seg_pos(const GridDev &g, const Tile &tl, int l, const SegLane &L,
                               SegPos &P)
{
    P.ok = L.act && L.w < tl.wa;
    P.gj = (int)tl.gj;
    P.q0 = (int)tl.base + L.w * (int)tl.gw + L.b * (int)tl.gj;
    if (l == 0) {
        const int line = (int)tl.rest + L.w;
        P.idx[0] = 0;
        P.idx[1] = g.ndim == 2 ? line : line % g.n[1];
        P.idx[2] = g.ndim == 2 ? 0 : line / g.n[1];
    } else {
        P.idx[0] = (int)tl.i0s + L.w;
        P.idx[1] = l == 1 ? 0 : (int)tl.rest;
        P.idx[2] = l == 2 ? 0 : (int)tl.rest;
    }
}

// wall or solid at position i of the lane's segment (walls: the faces of
// the other directions, fixed per lane, and this line's two ends)
__device__ inline bool seg_zero(const GridDev &g, int l, const SegLane &L, int i, bool side_wall,
                                unsigned char solid)
{
    const int j = L.b + i;
    bool z = side_wall || solid;
    z |= j == 0 && g.wall_lo[l];
    z |= j == g.n[l] - 1 && g.wall_hi[l];
    return z;
}

// walls of the directions other than l at this lane's line
__device__ inline bool seg_side_wall(const GridDev &g, int l, const SegPos &P)
{
    bool z = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == l || d >= g.ndim) continue;
        z |= P.idx[d] == 0 && g.wall_lo[d];
        z |= P.idx[d] == g.n[d] - 1 && g.wall_hi[d];
    }
    return z;
}

// extrapolated face values at the line's ends, from the new values of the
// segments that hold them (first segment: positions 0..2, last: M-3..M-1)
template <typename T, int M>
__device__ inline void seg_face_fix(const GridDev &g, int l, bool lo, bool hi, bool z0, bool z1,
                                    T (&x)[M])
{
    const int c0 = g.xbc[2 * l], c1 = g.xbc[2 * l + 1];
    if (lo && c0 != XBC_NONE && !z0)
        x[0] = c0 == XBC_NEUMANN ? ((T)4 * x[1] - x[2]) * (T)(1.0 / 3.0) : (T)2 * x[1] - x[2];
    if (hi && c1 != XBC_NONE && !z1)
        x[M - 1] = c1 == XBC_NEUMANN ? ((T)4 * x[M - 2] - x[M - 3]) * (T)(1.0 / 3.0)
                                     : (T)2 * x[M - 2] - x[M - 3];
}

// Extrapolated faces normal to l on new values in the line buffer: lane
// (w, side) sets position 0 or n-1 of line w from the two values inward of
// it (Neumann (4 f1 - f2)/3, outflow 2 f1 - f2), unless the face point is a
// wall or solid point; 32 lines per round, barriers before and after.
template <typename T, int M>
__device__ __forceinline__ void seg_faces(const GridDev &g, const SegGeo &sg, const Tile &tl, int l, T *X)
{
    const int n = tl.n;
    for (int w0 = 0; w0 < sg.W; w0 += kSegThreads / 2) {
        const int w = w0 + ((int)threadIdx.x >> 1), side = threadIdx.x & 1;
        __syncthreads();
        T fv = (T)0;
        int sl = -1;
        if (w < tl.wa && g.xbc[2 * l + side] != XBC_NONE) {
            const int j0 = side ? n - 1 : 0, in = side ? -1 : 1;
            const int q = (int)tl.base + w * (int)tl.gw + j0 * (int)tl.gj;
            int idx[3];
            index_of(g, q, idx);
            if (!(wall_point(g, idx) || (g.mask && gmem(g.mask)[q]))) {
                const T a = X[seg_slot<M>(sg, w, j0 + in)];
                const T b = X[seg_slot<M>(sg, w, j0 + 2 * in)];
                fv = g.xbc[2 * l + side] == XBC_NEUMANN ? ((T)4 * a - b) * (T)(1.0 / 3.0)
                                                       : (T)2 * a - b;
                sl = seg_slot<M>(sg, w, j0);
            }
        }
        __syncthreads();
        if (sl >= 0) X[sl] = fv;
    }
    __syncthreads();
}

// one field of the lane's segment from global memory (positions past a
// short segment's end repeat its last one)
template <typename T, int M>
__device__ inline void seg_read(gptr<const T> f, const SegLane &L, const SegPos &P, T (&a)[M])
{
    if (!P.ok) {
#pragma unroll
        for (int i = 0; i < M; ++i) a[i] = (T)0;
        return;
    }
#pragma unroll
    for (int i = 0; i < M; ++i) a[i] = f[P.q0 + min(i, L.len - 1) * P.gj];
}

template <typename T, int M>
__device__ inline void seg_write(gptr<T> f, const SegLane &L, const SegPos &P, const T (&a)[M])
{
    if (!P.ok) return;
    if (L.len == M) {
#pragma unroll
        for (int i = 0; i < M; ++i) f[P.q0 + i * P.gj] = a[i];
        return;
    }
#pragma unroll
    for (int i = 0; i < M; ++i)
        if (i < L.len) f[P.q0 + i * P.gj] = a[i];
}

// Direction 0 (lines contiguous in memory): cooperative I/O through the
// line buffer, lanes on consecutive elements of the tile's rows.
template <typename T, int M>
__device__ inline void seg_coop_load(gptr<const T> f, const SegGeo &sg, const Tile &tl, T *X)
{
    const int nel = sg.W * tl.n;
    T a[M];
    int sl[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const int e = c * kSegThreads + (int)threadIdx.x;
        sl[c] = -1;
        if (e < nel) {
            const int w = sdiv(e, tl.rn);
            if (w < tl.wa) {
                a[c] = f[(int)tl.base + e];
                sl[c] = seg_slot<M>(sg, w, e - w * tl.n);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c)
        if (sl[c] >= 0) X[sl[c]] = a[c];
}

template <typename T, int M>
__device__ inline void seg_coop_store(gptr<T> f, const SegGeo &sg, const Tile &tl, const T *X)
{
    const int nel = sg.W * tl.n;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const int e = c * kSegThreads + (int)threadIdx.x;
        if (e < nel) {
            const int w = sdiv(e, tl.rn);
            if (w < tl.wa) f[(int)tl.base + e] = X[seg_slot<M>(sg, w, e - w * tl.n)];
        }
    }
}

// load a field into the line buffer: direction 0 cooperatively, the
// strided directions lane by lane (each lane's own segment)
template <typename T, int M>
__device__ inline void seg_fill(gptr<const T> f, int l, const SegGeo &sg, const Tile &tl,
                                const SegLane &L, const SegPos &P, T *X)
{
    if (l == 0) {
        seg_coop_load<T, M>(f, sg, tl, X);
    } else {
        T a[M];
        seg_read<T, M>(f, L, P, a);
        seg_put<T, M>(sg, L, X, a);
    }
}

// store this lane's segment values x to a field: the strided directions
// lane by lane, direction 0 through the line buffer (waits for every lane
// before and after)
template <typename T, int M>
__device__ inline void seg_emit(gptr<T> f, int l, const SegGeo &sg, const Tile &tl,
                                const SegLane &L, const SegPos &P, T *X, const T (&x)[M])
{
    if (l == 0) {
        __syncthreads();
        seg_put<T, M>(sg, L, X, x);
        __syncthreads();
        seg_coop_store<T, M>(f, sg, tl, X);
    } else {
        seg_write<T, M>(f, L, P, x);
    }
}

// ---------------------------------------------------------------------
// read this lane's segment values back from the line buffer (positions
// past a short segment's end repeat its last one)
template <typename T, int M>
__device__ inline void seg_get(const SegGeo &sg, const SegLane &L, const T *X, T (&x)[M])
{
    if (L.len == M) {
        const int base = seg_slot<M>(sg, L.w, L.b);
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] = X[base + i];
        return;
    }
#pragma unroll
    for (int i = 0; i < M; ++i) x[i] = X[seg_slot<M>(sg, L.w, L.b + min(i, L.len - 1))];
}

// Cartesian pass along direction l (uniform spacing, no curvature): U_l =
// D_l phi / h_l and D_l U_l / h_l from one tile; partial sums |grad phi|^2
// and Laplacian carried in HBM between the directions.  The last direction
// (LAST) finishes the stage (Sec. 3.3) in place: each lane ends its own
// segment's points (residual, local step at stage 0, RK update, walls and
// solids) and, when the grid keeps its extrapolated faces normal to this
// direction, the lanes holding a line's ends set them from the new values.
template <typename T, int M, bool LAST>
__global__ void __launch_bounds__(kSegThreads)
k_seg_cart(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems,
           int l, int stage)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int H = kSegH;
    T *tb = reinterpret_cast<T *>(smem), *X = nullptr;
    int cur = -1;
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const SegGeo &sg = g.sgeo[l];
        const SegOpDev &op = g.sdop[l];
        __syncthreads();
        if (item.grid != cur) {
            X = tb + (op.solve ? seg_table_len(op.n, op.S) : 0);
            seg_tables<T>(op, tb);
            cur = item.grid;
        }
        const Tile tl = decode_tile(g, l, item.tile);
        SegLane L;
        seg_lane<M>(sg, L);
        SegPos P;
        seg_pos(g, tl, l, L, P);
        const int n = tl.n, per = g.periodic[l];
        const bool lo = !per && L.s == 0, hi = !per && L.s == sg.S - 1;
        gptr<const T> src = gcast<const T>(stage == 0 ? g.phi : g.ps);
        const T ih = (T)g.invh[l];
        T v[M + 2 * H], x[M];
        seg_fill<T, M>(src, l, sg, tl, L, P, X);
        __syncthreads();
        seg_window<T, M>(sg, L, n, per, X, v);
        seg_deriv_all<T, M>(g, v, L.len, lo, hi, x);
        seg_solve<T, M>(sg, op, tb, L, ih, x);                 // U_l
        if (g.need_lap) {
            __syncthreads();
            seg_put<T, M>(sg, L, X, x);
            __syncthreads();
            seg_window<T, M>(sg, L, n, per, X, v);
            seg_deriv_all<T, M>(g, v, L.len, lo, hi, x);
            seg_solve<T, M>(sg, op, tb, L, ih, x);             // D_l U_l
        }
        // U_l^2: U_l from the line buffer when it holds it (then it is not
        // kept through the second solve), else x itself
        T a[M];
        if (g.need_lap) {
            seg_get<T, M>(sg, L, X, a);
#pragma unroll
            for (int i = 0; i < M; ++i) a[i] = a[i] * a[i];
        } else {
#pragma unroll
            for (int i = 0; i < M; ++i) a[i] = x[i] * x[i];
        }
        gptr<T> P0 = gcast<T>(g.P[0]);
        gptr<T> P1 = gcast<T>(g.P[1]);
        if constexpr (!LAST) {
            // carried sums, one field at a time
            if (l > 0) {
                T b[M];
                seg_read<T, M>(P0, L, P, b);
#pragma unroll
                for (int i = 0; i < M; ++i) a[i] += b[i];
            }
            seg_emit<T, M>(P0, l, sg, tl, L, P, X, a);
            if (g.need_lap) {
                if (l > 0) {
                    T b[M];
                    seg_read<T, M>(P1, L, P, b);
#pragma unroll
                    for (int i = 0; i < M; ++i) x[i] += b[i];
                }
                seg_emit<T, M>(P1, l, sg, tl, L, P, X, x);
            }
        } else {
            // stage finish of the lane's own points, eight at a time
            T S1 = (T)0, S2 = (T)0;
            for (int d = 0; d < g.ndim; ++d) {
                S1 += (T)g.invh[d];
                S2 += (T)g.invh[d] * (T)g.invh[d];
            }
            gptr<const T> P2 = gcast<const T>(g.P[2]);
            gptr<const unsigned char> mk = gmem(g.mask);
            const bool sw = seg_side_wall(g, l, P);
            bool z0 = false, z1 = false;
#pragma unroll
            for (int c0 = 0; c0 < M; c0 += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int i = c0 + u;
                    if (!P.ok || i >= L.len) {
                        x[i] = (T)0;
                        continue;
                    }
                    const int q = P.q0 + i * P.gj;
                    const T ph = src[q];
                    const T g2 = a[i] + (l > 0 ? P0[q] : (T)0);
                    const T lap = g.need_lap ? x[i] + (l > 0 ? P1[q] : (T)0) : (T)0;
                    const T lad = g.lad ? P2[q] : (T)0;
                    const FinIn<T> fin = fin_load<T>(g, stage, q, ph);
                    const bool z = seg_zero(g, l, L, i, sw, g.mask ? mk[q] : (unsigned char)0);
                    if (i == 0) z0 = z;
                    if (i == M - 1) z1 = z;
                    x[i] = finish_point<T>(g, stage, q, z, ph, g2, g2, lap, (T)0, lad, S1, S2, fin);
                }
            }
            if (g.fuse_faces) seg_face_fix<T, M>(g, l, lo, hi, z0, z1, x);
            seg_write<T, M>(gcast<T>(g.ps), L, P, x);
        }
    }
}

// ---------------------------------------------------------------------
// LAD diffusivity along direction l (Eq. Gamma_form2 with the smoothing
// reading): phase 0 adds |grad xi_l| d4_l phi^n to the sensor sum (the
// first direction starts it); the last direction also takes C |sum| and
// smooths it along itself.  Phase 1 smooths the field along l.
template <typename T, int M>
__global__ void __launch_bounds__(kSegThreads)
k_seg_lad(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems,
          int l, int phase)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int H = kSegH;
    T *X = reinterpret_cast<T *>(smem);
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const SegGeo &sg = g.sgeo[l];
        __syncthreads();
        const Tile tl = decode_tile(g, l, item.tile);
        SegLane L;
        seg_lane<M>(sg, L);
        SegPos P;
        seg_pos(g, tl, l, L, P);
        const int n = tl.n, per = g.periodic[l];
        const bool last = l == g.ndim - 1;
        const bool lo = !per && L.s == 0, hi = !per && L.s == sg.S - 1;
        gptr<T> S = gcast<T>(g.P[2]);
        T v[M + 2 * H], x[M];
        seg_fill<T, M>(phase == 0 ? gcast<const T>(g.phi) : gcast<const T>(g.P[2]), l, sg, tl, L,
                       P, X);
        __syncthreads();
        seg_window<T, M>(sg, L, n, per, X, v);
        if (phase == 0) {
            const T wl = (T)g.invh[l];   // |grad xi_l| on a uniform grid
#pragma unroll
            for (int i = 0; i < M; ++i) x[i] = wl * seg_fourth<T, M>(v, i, lo, hi);
            if (l > 0) {
                T a[M];
                seg_read<T, M>(S, L, P, a);
#pragma unroll
                for (int i = 0; i < M; ++i) x[i] += a[i];
            }
            if (!last) {
                seg_emit<T, M>(S, l, sg, tl, L, P, X, x);
                continue;
            }
#pragma unroll
            for (int i = 0; i < M; ++i) x[i] = (T)g.C * fabs(x[i]);
            __syncthreads();
            seg_put<T, M>(sg, L, X, x);
            __syncthreads();
            seg_window<T, M>(sg, L, n, per, X, v);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] = seg_gauss9<T, M>(v, i, lo, hi);
        seg_emit<T, M>(S, l, sg, tl, L, P, X, x);
    }
}

// ---------------------------------------------------------------------
// Filter pass along direction l (Sec. 3.4) in correction form; the last
// direction re-imposes walls and solids (and the extrapolated faces it
// keeps), takes the pseudo-step change (Eq. Con-criter) and stores the new
// iterate.
template <typename T, int M>
__global__ void __launch_bounds__(kSegThreads)
k_seg_filter(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems,
             int l)
{
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int H = kSegH;
    T *tb = reinterpret_cast<T *>(smem), *X = nullptr;
    int cur = -1;
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const SegGeo &sg = g.sgeo[l];
        const SegOpDev &op = g.sfop[l];
        __syncthreads();
        if (item.grid != cur) {
            X = tb + (op.solve ? seg_table_len(op.n, op.S) : 0);
            seg_tables<T>(op, tb);
            cur = item.grid;
        }
        const Tile tl = decode_tile(g, l, item.tile);
        SegLane L;
        seg_lane<M>(sg, L);
        SegPos P;
        seg_pos(g, tl, l, L, P);
        const int n = tl.n, per = g.periodic[l];
        const bool last = l == g.ndim - 1;
        const bool resid = last && g.fused_resid;
        const bool lo = !per && L.s == 0, hi = !per && L.s == sg.S - 1;
        gptr<T> ps = gcast<T>(g.ps);
        gptr<T> phi = gcast<T>(g.phi);
        T v[M + 2 * H], x[M];
        seg_fill<T, M>(ps, l, sg, tl, L, P, X);
        __syncthreads();
        seg_window<T, M>(sg, L, n, per, X, v);
        seg_frhs_all<T, M>(g, v, L.len, lo, hi, x);
        seg_solve<T, M>(sg, op, tb, L, (T)1, x);
#pragma unroll
        for (int i = 0; i < M; ++i) x[i] += v[H + i];
        if (!last) {
            seg_emit<T, M>(ps, l, sg, tl, L, P, X, x);
            continue;
        }
        const bool sw = seg_side_wall(g, l, P);
        bool z0 = false, z1 = false;
        unsigned char solid[M];
        gptr<const unsigned char> mk = gmem(g.mask);
#pragma unroll
        for (int i = 0; i < M; ++i)
            solid[i] = (g.mask && P.ok && i < L.len) ? mk[P.q0 + i * P.gj] : 0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
            if (!P.ok || i >= L.len) continue;
            const bool z = seg_zero(g, l, L, i, sw, solid[i]);
            if (i == 0) z0 = z;
            if (i == M - 1) z1 = z;
            if (z) x[i] = (T)0;
        }
        if (g.fuse_faces) seg_face_fix<T, M>(g, l, lo, hi, z0, z1, x);
        if (!resid) {
            seg_write<T, M>(ps, L, P, x);
            continue;
        }
        double mx = 0.0, sm = 0.0, ng = 0.0, mg = 0.0;
        {
            T po[M];
            seg_read<T, M>(phi, L, P, po);
#pragma unroll
            for (int i = 0; i < M; ++i) {
                if (!P.ok || i >= L.len) continue;
                const double d = fabs((double)x[i] - (double)po[i]);
                mx = nanmax(mx, d);
                sm += d * d;
                ng = nanmax(ng, -(double)x[i]);
                mg = nanmax(mg, fabs((double)x[i]));
            }
        }
        seg_write<T, M>(phi, L, P, x);
        for (int o = 32; o > 0; o >>= 1) {
            mx = nanmax(mx, __shfl_xor(mx, o, kSegThreads));
            sm += __shfl_xor(sm, o, kSegThreads);
            ng = nanmax(ng, __shfl_xor(ng, o, kSegThreads));
            mg = nanmax(mg, __shfl_xor(mg, o, kSegThreads));
        }
        if (threadIdx.x == 0) put_rpart(g, item.tile, mx, sm, ng, mg);
    }
}

}  // namespace wd
