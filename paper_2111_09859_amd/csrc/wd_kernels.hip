// wd_kernels.hip -- pointwise gfx950 kernels of the wall-distance
// pseudo-time march (stage finish without a second derivative level,
// pseudo-step change, extrapolated faces, initial field, stopping logic)
// and the FP64 helpers (precision conversion, metric inversion, Poisson
// distance), plus the launch dispatcher.  The line-tile passes live in
// wd_line.h and are instantiated per value type and tile size by
// wd_line.hip.
#include "wd_line.h"
#include "wd_kernels.h"

#include <algorithm>
#include <climits>
#include <atomic>
#include <mutex>

namespace wd {

// A field as a buffer resource (wave-uniform): an access is a per-lane
// 32-bit byte offset plus a wave-uniform one, so the neighbours of a point
// along a direction share one offset register and their strides are scalar.
// The grids served here hold fewer than 2^31 bytes per field.
struct XBuf {
    __amdgpu_buffer_rsrc_t r;
};


// A resource over `bytes` bytes: an access at a per-lane offset at or
// beyond that (kXOut, or any offset when bytes = 0) is out of range, which
// the buffer unit answers with 0 for a load and drops for a store (no
// memory is touched), so lanes without a point and fields a grid does not
// use need no branch around their accesses.
constexpr unsigned kXOut = 0x80000000u;
__device__ __forceinline__ XBuf xbuf_bytes(const void *p, long long bytes)
{
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000)};
}

template <typename T>
__device__ __forceinline__ T xload(XBuf b, unsigned vo, unsigned so);
template <>
__device__ __forceinline__ float xload<float>(XBuf b, unsigned vo, unsigned so)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, vo, so, 0));
}
template <>
__device__ __forceinline__ double xload<double>(XBuf b, unsigned vo, unsigned so)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, vo, so, 0));
}

__device__ __forceinline__ unsigned char xload_u8(XBuf b, unsigned vo, unsigned so)
{
    return __builtin_amdgcn_raw_buffer_load_b8(b.r, vo, so, 0);
}

template <typename T>
__device__ __forceinline__ void xstore(XBuf b, T v, unsigned vo, unsigned so);
template <>
__device__ __forceinline__ void xstore<float>(XBuf b, float v, unsigned vo, unsigned so)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.r, vo, so, 0);
}
template <>
__device__ __forceinline__ void xstore<double>(XBuf b, double v, unsigned vo, unsigned so)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), b.r, vo, so, 0);
}

// Pointwise stage finish for general grids without a second derivative
// level (Eikonal; for the upwind baseline also its advective term).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_final(const GridDev *__restrict__ grids, const Item *__restrict__ items,
        int nitems, int stage)
{
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const long long q0 = (long long)item.tile * kChunk;
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long qq = q0 + i;
            if (qq >= g.N) break;
            const int q = (int)qq;
            gptr<const T> src = gcast<const T>(stage == 0 ? g.phi : g.ps);
            T m9[9], g2, adv;
            metric_load<T>(g, q, m9);
            int idx[3];
            index_of(g, q, idx);
            if (g.uw) {
                // the upwind baseline's advective term, formed by k_uwadv
                // (this pass overwrites the stage value its stencil reads)
                adv = gcast<const T>(g.P[1])[q];
                g2 = gcast<const T>(g.uw2)[q];
            } else {
                T F3[3], U[3];
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    if (m < g.ndim) F3[m] = gcast<const T>(g.F[m])[q];
                grad_from<T>(g.ndim, m9, F3, U, g2);
                adv = g2;
            }
            const bool zero = wall_point(g, idx) || (g.mask && gmem(g.mask)[q]);
            const T phis = src[q];
            T S1, S2;
            metric_sums<T>(g.ndim, m9, S1, S2);
            gcast<T>(g.ps)[q] =
                finish_point<T>(g, stage, q, zero, phis, g2, adv, (T)0, (T)0, (T)0, S1, S2,
                                fin_load<T>(g, stage, q, phis));
        }
    }
}

// The method's fields the stage finish reads, held by a pointwise pass for
// the item it works on (already in T: the same values the finish forms
// from the grid record).
template <typename T>
struct XFin {
    int eq, lad, curv, rk;
    T eps, nu0, kp, kp2, sigma;
};

// Pointwise stage finish (Sec. 3.3) of a uniform Cartesian grid whose
// directional passes carried the whole |grad phi|^2 and Laplacian on
// (segmented passes, no extrapolated faces): every operand a plain field,
// the loads of a thread's points issued before any use, every access
// unconditional (buffer resources: out-of-range offsets and zero-sized
// fields select), the method's fields held per item.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_cart_finish(const GridDev *__restrict__ grids, const Item *__restrict__ items,
              int nitems, int stage)
{
    constexpr int K = kChunk / kThreads;
    constexpr unsigned E = sizeof(T);
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        T S1 = (T)0, S2 = (T)0;
        for (int d = 0; d < g.ndim; ++d) {
            S1 += (T)g.invh[d];
            S2 += (T)g.invh[d] * (T)g.invh[d];
        }
        XFin<T> fp;
        fp.eq = g.eq;
        fp.lad = g.lad;
        fp.curv = g.curv;
        fp.rk = g.rk;
        fp.eps = (T)g.eps;
        fp.nu0 = (T)g.nu0;
        fp.kp = (T)g.kp;
        fp.kp2 = (T)g.kp2;
        fp.sigma = (T)g.sigma;
        const long long fb = g.N * (long long)E;
        const XBuf srb = xbuf_bytes(stage == 0 ? g.phi : g.ps, fb);
        const XBuf psb = xbuf_bytes(g.ps, fb);
        const XBuf p0b = xbuf_bytes(g.P[0], fb);
        const XBuf p1b = xbuf_bytes(g.P[1], g.need_lap ? fb : 0);
        const XBuf p2b = xbuf_bytes(g.P[2], g.lad ? fb : 0);
        const XBuf pnb = xbuf_bytes(g.phi, stage > 0 ? fb : 0);
        const XBuf dtb = xbuf_bytes(g.dt, fb);
        const XBuf acb = xbuf_bytes(g.acc, g.rk == 1 ? fb : 0);
        const XBuf mkb = xbuf_bytes(g.mask, g.mask ? g.N : 0);
        const unsigned dtl = stage > 0 ? 0u : kXOut, dts = stage == 0 ? 0u : kXOut;
        const long long q0 = (long long)item.tile * kChunk;
        int qv[K];
        unsigned vo[K];
        T ph[K], g2[K], lap[K], lad[K], pn[K], dt[K], ac[K];
        unsigned char solid[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const long long qq = q0 + threadIdx.x + k * kThreads;
            qv[k] = qq < g.N ? (int)qq : 0;
            vo[k] = qq < g.N ? (unsigned)qq * E : kXOut;
            ph[k] = xload<T>(srb, vo[k], 0);
            g2[k] = xload<T>(p0b, vo[k], 0);
            lap[k] = xload<T>(p1b, vo[k], 0);
            lad[k] = xload<T>(p2b, vo[k], 0);
            pn[k] = xload<T>(pnb, vo[k], 0);
            dt[k] = xload<T>(dtb, vo[k] | dtl, 0);
            ac[k] = xload<T>(acb, vo[k], 0);
            solid[k] = xload_u8(mkb, vo[k] == kXOut ? kXOut : vo[k] / E, 0);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int idx[3];
            index_of(g, qv[k], idx);
            const bool zero = solid[k] || wall_point(g, idx);
            FinIn<T> fin;
            fin.pn = stage == 0 ? ph[k] : pn[k];
            fin.dt = dt[k];
            fin.acc = ac[k];
            T dto = (T)0, aco = (T)0;
            const T out = finish_core<T>(fp, stage, zero, ph[k], g2[k], g2[k], lap[k], (T)0,
                                         lad[k], S1, S2, fin, dto, aco);
            xstore<T>(psb, out, vo[k], 0);
            xstore<T>(dtb, dto, vo[k] | dts, 0);
            xstore<T>(acb, aco, vo[k], 0);
        }
    }
}

// ---------------------------------------------------------------------
// One-pass RK stage of a uniform Cartesian grid with an explicit scheme
// (E2/E4/E6, radius R; Sec. 3.2): every point forms U_l = D_l phi / h_l
// and D_l U_l / h_l along each direction straight from the stage value's
// neighbours (no line solve: D_l U_l at i needs U_l at i-R..i+R, which
// need phi at i-2R..i+2R), sums |grad phi|^2 and the Laplacian and finishes
// the stage.  The stage value is read from one buffer and written to
// another (the stencil reads neighbours the pass also writes).

// first derivative at end position A < R (index space, counted from a
// non-periodic end: A = 0 is the end point) from e[] (f at end positions
// 0 .. 4): the one-sided closure rows.  At the high end the end coordinate
// runs against the index, so the derivative there is the negative of this
// one (the second derivative is unchanged).
template <typename T, int R, int A>
__device__ inline T xend_row(const T *e)
{
    static_assert(A < R, "closure rows only");
    if (R == 1) return ((T)-3 * e[0] + (T)4 * e[1] - e[2]) * (T)0.5;
    if (A == 0)
        return ((T)-25 * e[0] + (T)48 * e[1] - (T)36 * e[2] + (T)16 * e[3] - (T)3 * e[4]) *
               (T)(1.0 / 12.0);
    if (A == 1)
        return ((T)-3 * e[0] - (T)10 * e[1] + (T)18 * e[2] - (T)6 * e[3] + e[4]) *
               (T)(1.0 / 12.0);
    return (e[0] - (T)8 * e[1] + (T)8 * e[3] - e[4]) * (T)(1.0 / 12.0);
}

// Tiles of the one-pass stage: kXTX x kXTY points of an x-y plane per
// workgroup, marched along z over a chunk of planes.  The tile's stage
// values and a halo of 2R points sit in LDS; U_x and U_y are formed there
// once per position (the tile and a halo of R), so each point's D_l U_l
// reads R neighbours of U on each side.  Along z every thread keeps a
// queue per point in registers (XZq: U_z of 2R + 1 planes and the stage
// values of the next 2R): a plane costs one new load and one new U_z per
// point, and near a non-periodic z end the queue is refilled with each
// position's own row.
constexpr int kXRow = kThreads / kXTX;   // rows the threads cover at once
constexpr int kXPY = kXTY / kXRow;       // points per thread and plane

template <typename T, int R>
struct XTile {
    static constexpr int PW = kXTX + 4 * R, PH = kXTY + 4 * R;
    static constexpr int UW = kXTX + 2 * R, UH = kXTY + 2 * R;
    T ph[2][PH * PW];    // stage value at x0-2R .. x0+TX+2R-1, y0-2R .. y0+TY+2R-1
                         // (this plane's and the next one's)
    T ux[kXTY * UW];     // U_x at x0-R .. x0+TX+R-1 of rows y0 .. y0+TY-1
    T uy[UH * kXTX];     // U_y at rows y0-R .. y0+TY+R-1 of columns x0 .. x0+TX-1
};


// D f at position j of a line of n points (index space, not scaled by
// 1/h), f(m) the value at index m: the interior central row, or within R
// of a non-periodic end that end's closure row over the points counted
// from the end (negated at the high end, where that count runs against the
// index).  The periodic rows read f at j - R .. j + R unwrapped: the
// caller's f holds the wrapped values there.
template <typename T>
struct XCo {
    T a, b, c;   // interior first-derivative weights of f(j +- 1, 2, 3)
};

template <typename T, int R, typename F>
__device__ __forceinline__ T xrow(const XCo<T> &co, int j, int n, bool per, const F &f)
{
    if (per || (j >= R && j <= n - 1 - R)) {
        const T a = co.a, b = co.b, c = co.c;
        T s = a * (f(j + 1) - f(j - 1));
        if (R >= 2) s += b * (f(j + 2) - f(j - 2));
        if (R >= 3) s += c * (f(j + 3) - f(j - 3));
        return s;
    }
    const bool low = j < R;
    const int A = low ? j : n - 1 - j;
    T e[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) e[m] = (R == 1 && m > 2) ? (T)0 : f(low ? m : n - 1 - m);
    T d;
    if (R >= 3 && A == 2) d = xend_row<T, R, (R >= 3 ? 2 : 0)>(e);
    else if (R >= 2 && A == 1) d = xend_row<T, R, (R >= 2 ? 1 : 0)>(e);
    else d = xend_row<T, R, 0>(e);
    return low ? d : -d;
}

template <typename T, int R>
__device__ __forceinline__ T xcentral(const XCo<T> &co, const T *v)
{
    // the interior row on v[0 .. 2R] (centre v[R])
    const T a = co.a, b = co.b, c = co.c;
    T s = a * (v[R + 1] - v[R - 1]);
    if (R >= 2) s += b * (v[R + 2] - v[R - 2]);
    if (R >= 3) s += c * (v[R + 3] - v[R - 3]);
    return s;
}

// Workgroup barrier ordering LDS accesses only: global loads in flight
// (the next plane's prefetch) stay in flight across it.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// U_z queue (3D grids): U_z of planes jb .. jb + 2R (index space, scaled
// by 1/h_z) and the stage values of planes jb + R + 1 .. jb + 3R, from which
// the next U_z follows with one more plane.  Filled from the stage values
// around plane jb with each position's own row (closure rows of either
// end from the end's five points); moved on one plane at a time while the
// new position takes the interior row.
template <typename T, int R>
struct XZq {
    T u[2 * R + 1];
    T p[2 * R];
};

template <typename T, int R>
__device__ __forceinline__ void xz_fill(const XCo<T> &co, XBuf sb, unsigned vo,
                                        int jb, int n2, int s2, bool pz, T ih2, XZq<T, R> &z)
{
    constexpr unsigned E = sizeof(T);
    T v[4 * R + 1];
#pragma unroll
    for (int m = 0; m <= 4 * R; ++m) {
        int kk = jb - R + m;
        if (pz) kk = kk < 0 ? kk + n2 : (kk >= n2 ? kk - n2 : kk);
        else kk = kk < 0 ? 0 : (kk >= n2 ? n2 - 1 : kk);
        v[m] = xload<T>(sb, vo, (unsigned)(kk * s2) * E);
    }
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) z.u[i] = xcentral<T, R>(co, &v[i]);
    if (!pz && (jb < R || jb + 2 * R > n2 - 1 - R)) {
        // closure rows: the five points of each end
        T lo[5], hi[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            const int a = min(m, n2 - 1), b = max(n2 - 1 - m, 0);
            lo[m] = xload<T>(sb, vo, (unsigned)(a * s2) * E);
            hi[m] = xload<T>(sb, vo, (unsigned)(b * s2) * E);
        }
        T cl[3], ch[3];
        cl[0] = xend_row<T, R, 0>(lo);
        ch[0] = -xend_row<T, R, 0>(hi);
        cl[1] = cl[2] = ch[1] = ch[2] = (T)0;
        if (R >= 2) {
            cl[1] = xend_row<T, R, (R >= 2 ? 1 : 0)>(lo);
            ch[1] = -xend_row<T, R, (R >= 2 ? 1 : 0)>(hi);
        }
        if (R >= 3) {
            cl[2] = xend_row<T, R, (R >= 3 ? 2 : 0)>(lo);
            ch[2] = -xend_row<T, R, (R >= 3 ? 2 : 0)>(hi);
        }
#pragma unroll
        for (int i = 0; i <= 2 * R; ++i) {
            const int j = jb + i, A = n2 - 1 - j;
#pragma unroll
            for (int a = 0; a < R; ++a) {
                z.u[i] = j == a ? cl[a] : z.u[i];
                z.u[i] = A == a ? ch[a] : z.u[i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i <= 2 * R; ++i) z.u[i] *= ih2;
#pragma unroll
    for (int m = 0; m < 2 * R; ++m) z.p[m] = v[2 * R + 1 + m];
}

// u_z and D_z u_z at plane k from the queue (base jb: k - R inside,
// 0 or n2 - 1 - 2R within R of a non-periodic end)
template <typename T, int R>
__device__ __forceinline__ void xz_terms(const XCo<T> &co, const XZq<T, R> &z,
                                         int k, int jb, int n2, bool pz, T ih2, T &u2, T &l2)
{
    if (pz || (k >= R && k <= n2 - 1 - R)) {
        u2 = z.u[R];
        l2 = xcentral<T, R>(co, z.u) * ih2;
        return;
    }
    const int d = k - jb;
    T e[5];
    const bool low = k < R;
#pragma unroll
    for (int m = 0; m < 5; ++m) e[m] = low ? z.u[m < 2 * R + 1 ? m : 0] : z.u[2 * R - m >= 0 ? 2 * R - m : 0];
    u2 = z.u[0];
#pragma unroll
    for (int i = 1; i <= 2 * R; ++i) u2 = d == i ? z.u[i] : u2;
    const int A = low ? k : n2 - 1 - k;
    T l = xend_row<T, R, 0>(e);
    if (R >= 2 && A == 1) l = xend_row<T, R, (R >= 2 ? 1 : 0)>(e);
    if (R >= 3 && A == 2) l = xend_row<T, R, (R >= 3 ? 2 : 0)>(e);
    l2 = (low ? l : -l) * ih2;
}

// The interior row on values S apart around c[0].
template <typename T, int R, int S>
__device__ __forceinline__ T xcentral_at(const XCo<T> &co, const T *c)
{
    T v = co.a * (c[S] - c[-S]);
    if (R >= 2) v += co.b * (c[2 * S] - c[-2 * S]);
    if (R >= 3) v += co.c * (c[3 * S] - c[-3 * S]);
    return v;
}

template <typename T, int R, bool FAST>
__global__ void __launch_bounds__(kThreads)
k_xstage(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems,
         int stage)
{
    using Tile = XTile<T, R>;
    constexpr int PW = Tile::PW, PH = Tile::PH, UW = Tile::UW, UH = Tile::UH;
    constexpr int NT = (PH * PW + kThreads - 1) / kThreads;       // tile loads per thread
    constexpr int NUX = (kXTY * UW + kThreads - 1) / kThreads;    // U_x positions per thread
    constexpr int NUY = (UH * kXTX + kThreads - 1) / kThreads;    // U_y positions per thread
    constexpr unsigned E = sizeof(T);
    __shared__ Tile sm;
    const int tid = threadIdx.x, cx = tid % kXTX, r0 = tid / kXTX;
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const int n0 = g.n[0], n1 = g.n[1];
        const bool d3 = g.ndim == 3;
        const int n2 = d3 ? g.n[2] : 1;
        const int ntx = (n0 + kXTX - 1) / kXTX, nty = (n1 + kXTY - 1) / kXTY;
        const int tx = item.tile % ntx, ty = (item.tile / ntx) % nty;
        const int zc = item.tile / (ntx * nty);
        const int x0 = xtile_origin(tx, kXTX, n0), y0 = xtile_origin(ty, kXTY, n1);
        const int wx = min(kXTX, n0), wy = min(kXTY, n1);
        const int kz = FAST ? g.xkz : g.xkz2;
        const int z0 = zc * kz, z1 = min(z0 + kz, n2);
        const bool px = g.periodic[0] != 0, py = g.periodic[1] != 0;
        const bool pz = d3 && g.periodic[2] != 0;
        const int s1 = (int)g.stride[1], s2 = d3 ? (int)g.stride[2] : 0;
        const T ih0 = (T)g.invh[0], ih1 = (T)g.invh[1], ih2 = (T)g.invh[2];
        T S1 = (T)0, S2 = (T)0;
        for (int d = 0; d < g.ndim; ++d) {
            S1 += (T)g.invh[d];
            S2 += (T)g.invh[d] * (T)g.invh[d];
        }
        XCo<T> co;
        co.a = (T)(0.5 * g.da);
        co.b = (T)(0.25 * g.db);
        co.c = (T)(g.dc / 6.0);
        XFin<T> fp;
        fp.eq = g.eq;
        fp.lad = g.lad;
        fp.curv = g.curv;
        fp.rk = g.rk;
        fp.eps = (T)g.eps;
        fp.nu0 = (T)g.nu0;
        fp.kp = (T)g.kp;
        fp.kp2 = (T)g.kp2;
        fp.sigma = (T)g.sigma;
        const bool need_lap = g.need_lap != 0;
        // walls on the faces normal to z (the x and y ones are per point)
        const bool wz_lo = d3 && g.wall_lo[2], wz_hi = d3 && g.wall_hi[2];
        // stage values alternate between ps and P[0] so that the last
        // stage ends in ps
        const bool to_ps = ((g.stages - 1 - stage) & 1) == 0;
        const void *srcp = stage == 0 ? g.phi : (to_ps ? g.P[0] : g.ps);
        const long long fb = g.N * (long long)E;
        const XBuf sb = xbuf_bytes(srcp, fb);
        const XBuf db = xbuf_bytes(to_ps ? g.ps : g.P[0], fb);
        // the finish's other fields (zero-sized where the method does not
        // use them); phi^n and the local step are read after stage 0, the
        // local step written at stage 0 (offsets or-ed with kXOut select)
        const XBuf pnb = xbuf_bytes(g.phi, stage > 0 ? fb : 0);
        const XBuf dtb = xbuf_bytes(g.dt, fb);
        const XBuf acb = xbuf_bytes(g.acc, g.rk == 1 ? fb : 0);
        const XBuf ldb = xbuf_bytes(g.P[2], g.lad ? fb : 0);
        const XBuf mkb = xbuf_bytes(g.mask, g.mask ? g.N : 0);
        const unsigned dtl = stage > 0 ? 0u : kXOut, dts = stage == 0 ? 0u : kXOut;

        // the tile's stage values: element tid + m kThreads of the LDS tile
        // is read at byte offset toff[m] of each plane (kXOut: none)
        unsigned toff[NT];
#pragma unroll
        for (int m = 0; m < NT; ++m) {
            const int e = tid + m * kThreads;
            const int ey = e / PW, ex = e - ey * PW;
            int jx = x0 - 2 * R + ex, jy = y0 - 2 * R + ey;
            bool ok = e < PH * PW && ex < wx + 4 * R && ey < wy + 4 * R;
            if (px) jx = jx < 0 ? jx + n0 : (jx >= n0 ? jx - n0 : jx);
            else ok = ok && jx >= 0 && jx < n0;
            if (py) jy = jy < 0 ? jy + n1 : (jy >= n1 ? jy - n1 : jy);
            else ok = ok && jy >= 0 && jy < n1;
            toff[m] = ok ? (unsigned)(jy * s1 + jx) * E : kXOut;
        }
        // this thread's points: column x0 + cx, rows y0 + r0 + kXRow p;
        // byte offsets within a plane for loads (kXOut outside the grid)
        // and for stores (kXOut unless the point is this tile's own)
        const int gx = x0 + cx;
        unsigned vin[kXPY], vown[kXPY];
        bool wxy[kXPY];   // the point lies on a wall normal to x or y
#pragma unroll
        for (int p = 0; p < kXPY; ++p) {
            const int ry = r0 + kXRow * p, gy = y0 + ry;
            const bool in = cx < wx && ry < wy;
            const bool own = in && gx >= tx * kXTX && gy >= ty * kXTY;
            const unsigned off = (unsigned)(gy * s1 + gx);
            vin[p] = in ? off * E : kXOut;
            vown[p] = own ? off * E : kXOut;
            wxy[p] = (gx == 0 && g.wall_lo[0]) || (gx == n0 - 1 && g.wall_hi[0]) ||
                     (gy == 0 && g.wall_lo[1]) || (gy == n1 - 1 && g.wall_hi[1]);
        }
        XZq<T, R> zq[kXPY];
        int jb = INT_MIN;   // the queue's base plane (none yet)
        T tv[NT];
        auto tile_put = [&](T *ph) {
#pragma unroll
            for (int m = 0; m < NT; ++m)
                if (m < NT - 1 || tid + m * kThreads < PH * PW) ph[tid + m * kThreads] = tv[m];
        };
        auto zbase = [&](int k) {
            return pz ? k - R : min(max(k - R, 0), n2 - 1 - 2 * R);
        };
#pragma unroll
        for (int m = 0; m < NT; ++m) tv[m] = xload<T>(sb, toff[m], (unsigned)(z0 * s2) * E);
        lds_barrier();   // the previous item's reads of the tiles are done
        tile_put(sm.ph[0]);
        int cur = 0;
        for (int k = z0; k < z1; ++k) {
            const unsigned so = (unsigned)(k * s2) * E;
            if (d3 && zbase(k) != jb) {
                jb = zbase(k);
#pragma unroll
                for (int p = 0; p < kXPY; ++p)
                    xz_fill<T, R>(co, sb, vin[p], jb, n2, s2, pz, ih2, zq[p]);
            }
            // the queue moves on after this plane when the next plane's base
            // is one further and its new position takes the interior row
            const bool adv = d3 && k + 1 < z1 && zbase(k + 1) == jb + 1 &&
                             (pz || jb + 2 * R + 1 <= n2 - 1 - R);
            // this plane's tile is in sm.ph[cur]; the previous plane's
            // reads of U and of the other tile buffer are done
            lds_barrier();
            const T *ph = sm.ph[cur];
            // issued now, used later in the plane: the finish inputs, the
            // stage value the z queue takes in next, and the next plane's
            // tile (every access unconditional: offsets and sizes select)
            T fpn[kXPY], fdt[kXPY], fac[kXPY], fld[kXPY], znx[kXPY];
            unsigned char fmk[kXPY];
            int kn = adv ? jb + 3 * R + 1 : k;
            kn = kn >= n2 ? kn - n2 : kn;
#pragma unroll
            for (int p = 0; p < kXPY; ++p) {
                fpn[p] = xload<T>(pnb, vown[p], so);
                fdt[p] = xload<T>(dtb, vown[p] | dtl, so);
                fac[p] = xload<T>(acb, vown[p], so);
                fld[p] = xload<T>(ldb, vown[p], so);
                fmk[p] = xload_u8(mkb, vown[p] == kXOut ? kXOut : vown[p] / E, (unsigned)(k * s2));
                znx[p] = xload<T>(sb, vin[p], (unsigned)(kn * s2) * E);
            }
            {
                const unsigned sn = (unsigned)(min(k + 1, z1 - 1) * s2) * E;
#pragma unroll
                for (int m = 0; m < NT; ++m) tv[m] = xload<T>(sb, toff[m], sn);
            }
            if constexpr (FAST) {
#pragma unroll
                for (int i = 0; i < NUX; ++i) {
                    const int e = tid + i * kThreads;
                    if (i < NUX - 1 || e < kXTY * UW) {
                        const int ry = e / UW, ex = e - ry * UW;
                        sm.ux[e] = xcentral_at<T, R, 1>(co, ph + (ry + 2 * R) * PW + ex + R) * ih0;
                    }
                }
#pragma unroll
                for (int i = 0; i < NUY; ++i) {
                    const int e = tid + i * kThreads;
                    if (i < NUY - 1 || e < UH * kXTX) {
                        const int ey = e / kXTX, c = e - ey * kXTX;
                        sm.uy[e] = xcentral_at<T, R, PW>(co, ph + (ey + R) * PW + c + 2 * R) * ih1;
                    }
                }
            } else {
                for (int e = tid; e < kXTY * UW; e += kThreads) {
                    const int ry = e / UW, ex = e - ry * UW;
                    const int jx = x0 - R + ex;
                    T v = (T)0;
                    if (ry < wy && ex < wx + 2 * R && (px || (jx >= 0 && jx < n0))) {
                        const int base = (ry + 2 * R) * PW - (x0 - 2 * R);
                        v = xrow<T, R>(co, jx, n0, px, [&](int m) { return ph[base + m]; }) *
                            ih0;
                    }
                    sm.ux[e] = v;
                }
                for (int e = tid; e < UH * kXTX; e += kThreads) {
                    const int ey = e / kXTX, c = e - ey * kXTX;
                    const int jy = y0 - R + ey;
                    T v = (T)0;
                    if (c < wx && ey < wy + 2 * R && (py || (jy >= 0 && jy < n1))) {
                        const int base = 2 * R + c - (y0 - 2 * R) * PW;
                        v = xrow<T, R>(co, jy, n1, py,
                                       [&](int m) { return ph[base + m * PW]; }) *
                            ih1;
                    }
                    sm.uy[e] = v;
                }
            }
            lds_barrier();
            T out[kXPY], dto[kXPY], aco[kXPY];
#pragma unroll
            for (int p = 0; p < kXPY; ++p) {
                const int ry = r0 + kXRow * p, gy = y0 + ry;
                out[p] = dto[p] = aco[p] = (T)0;
                if (FAST || vin[p] != kXOut) {
                    // U and D U along x and y from the tile's U fields
                    const T *ucx = sm.ux + ry * UW + cx + R;
                    const T *ucy = sm.uy + (ry + R) * kXTX + cx;
                    const T u0 = *ucx, u1 = *ucy;
                    T l0, l1;
                    if constexpr (FAST) {
                        l0 = xcentral_at<T, R, 1>(co, ucx) * ih0;
                        l1 = xcentral_at<T, R, kXTX>(co, ucy) * ih1;
                    } else {
                        const int ub = ry * UW - (x0 - R);
                        l0 = xrow<T, R>(co, gx, n0, px, [&](int m) { return sm.ux[ub + m]; }) *
                             ih0;
                        const int vb = cx - (y0 - R) * kXTX;
                        l1 = xrow<T, R>(co, gy, n1, py,
                                        [&](int m) { return sm.uy[vb + m * kXTX]; }) *
                             ih1;
                    }
                    T g2 = (T)0, lap = (T)0;
                    g2 += u0 * u0;
                    lap += l0;
                    g2 += u1 * u1;
                    lap += l1;
                    if (d3) {
                        T u2, l2;
                        xz_terms<T, R>(co, zq[p], k, jb, n2, pz, ih2, u2, l2);
                        g2 += u2 * u2;
                        lap += l2;
                    }
                    const T phs = ph[(ry + 2 * R) * PW + cx + 2 * R];
                    FinIn<T> fin;
                    fin.pn = stage == 0 ? phs : fpn[p];
                    fin.dt = fdt[p];
                    fin.acc = fac[p];
                    const bool zero = fmk[p] != 0 || wxy[p] || (k == 0 && wz_lo) ||
                                      (k == n2 - 1 && wz_hi);
                    out[p] = finish_core<T>(fp, stage, zero, phs, g2, g2, need_lap ? lap : (T)0,
                                            (T)0, fld[p], S1, S2, fin, dto[p], aco[p]);
                }
            }
            // the next plane's tile into the other buffer (before this
            // plane's stores, so that waiting for its loads waits for no
            // store), then this plane's results
            if (k + 1 < z1) tile_put(sm.ph[cur ^ 1]);
            cur ^= 1;
#pragma unroll
            for (int p = 0; p < kXPY; ++p) {
                xstore<T>(db, out[p], vown[p], so);
                xstore<T>(dtb, dto[p], vown[p] | dts, so);
                xstore<T>(acb, aco[p], vown[p], so);
            }
            // the z queue moves on by one plane
            if (adv) {
                ++jb;
#pragma unroll
                for (int p = 0; p < kXPY; ++p) {
                    XZq<T, R> &z = zq[p];
                    T v[2 * R + 1];
#pragma unroll
                    for (int m = 0; m < 2 * R; ++m) v[m] = z.p[m];
                    v[2 * R] = znx[p];
#pragma unroll
                    for (int m = 0; m < 2 * R; ++m) z.u[m] = z.u[m + 1];
                    z.u[2 * R] = xcentral<T, R>(co, v) * ih2;
#pragma unroll
                    for (int m = 0; m < 2 * R - 1; ++m) z.p[m] = z.p[m + 1];
                    z.p[2 * R - 1] = znx[p];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------
// LAD diffusivity of a uniform Cartesian grid (Eq. Gamma_form2 with the
// smoothing reading) in two passes over kXTX x kXTY x-y tiles marched along
// z, as the one-pass stage: the sensor C |sum_l d4_l phi^n / h_l| (d4 the
// five-point fourth difference along l, its centre moved inward of the
// two points next to a non-periodic end) into P[1], then the nine-point
// truncated Gaussian along x, y and z (ends clamped, periodic lines wrap)
// into P[2].

constexpr int kLadS = 2;   // sensor tile halo (the fourth difference)
constexpr int kLadG = 4;   // smoothing tile halo (the Gaussian)

template <typename T>
__device__ __forceinline__ T xd4(const T *c, int s)
{
    return c[-2 * s] - (T)4 * c[-s] + (T)6 * c[0] - (T)4 * c[s] + c[2 * s];
}

// nine-point truncated Gaussian around c[0], neighbours at lo[o] / hi[o]
template <typename T>
__device__ __forceinline__ T xgauss(T c0, const T *lo, const T *hi)
{
    const T b[5] = {(T)(3565.0 / 10368.0), (T)(3091.0 / 12960.0), (T)(1997.0 / 25920.0),
                    (T)(149.0 / 12960.0), (T)(107.0 / 103680.0)};
    T acc = b[0] * c0;
#pragma unroll
    for (int o = 1; o <= 4; ++o) acc += b[o] * (lo[o] + hi[o]);
    return acc;
}

// The tile decoding shared by both passes: origin, extent and z range of
// work item `tile` of grid g (chunks of g.xlkz planes).
struct XTileGeo {
    int tx, ty, x0, y0, wx, wy, z0, z1, n0, n1, n2;
    bool d3, px, py, pz;
    int s1, s2;
};

__device__ inline XTileGeo xlad_geo(const GridDev &g, int tile)
{
    XTileGeo t;
    t.n0 = g.n[0];
    t.n1 = g.n[1];
    t.d3 = g.ndim == 3;
    t.n2 = t.d3 ? g.n[2] : 1;
    const int ntx = (t.n0 + kXTX - 1) / kXTX, nty = (t.n1 + kXTY - 1) / kXTY;
    t.tx = tile % ntx;
    t.ty = (tile / ntx) % nty;
    const int zc = tile / (ntx * nty);
    t.x0 = xtile_origin(t.tx, kXTX, t.n0);
    t.y0 = xtile_origin(t.ty, kXTY, t.n1);
    t.wx = min(kXTX, t.n0);
    t.wy = min(kXTY, t.n1);
    t.z0 = zc * g.xlkz;
    t.z1 = min(t.z0 + g.xlkz, t.n2);
    t.px = g.periodic[0] != 0;
    t.py = g.periodic[1] != 0;
    t.pz = t.d3 && g.periodic[2] != 0;
    t.s1 = (int)g.stride[1];
    t.s2 = t.d3 ? (int)g.stride[2] : 0;
    return t;
}

// byte offsets within a plane of element e of a tile with halo H (kXOut:
// outside a non-periodic grid), and of this thread's points (loads: in the
// grid; stores: the tile's own)
template <int H>
__device__ inline unsigned xtile_off(const XTileGeo &t, int e, unsigned E)
{
    constexpr int W = kXTX + 2 * H, Hh = kXTY + 2 * H;
    const int ey = e / W, ex = e - ey * W;
    int jx = t.x0 - H + ex, jy = t.y0 - H + ey;
    bool ok = e < W * Hh && ex < t.wx + 2 * H && ey < t.wy + 2 * H;
    if (t.px) jx = jx < 0 ? jx + t.n0 : (jx >= t.n0 ? jx - t.n0 : jx);
    else ok = ok && jx >= 0 && jx < t.n0;
    if (t.py) jy = jy < 0 ? jy + t.n1 : (jy >= t.n1 ? jy - t.n1 : jy);
    else ok = ok && jy >= 0 && jy < t.n1;
    return ok ? (unsigned)(jy * t.s1 + jx) * E : kXOut;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_xlad_sens(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems)
{
    constexpr int H = kLadS, PW = kXTX + 2 * H, PH = kXTY + 2 * H;
    constexpr int NT = (PW * PH + kThreads - 1) / kThreads;
    constexpr unsigned E = sizeof(T);
    __shared__ T sm[2][PW * PH];
    const int tid = threadIdx.x, cx = tid % kXTX, r0 = tid / kXTX;
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const XTileGeo t = xlad_geo(g, item.tile);
        const T w0 = (T)g.invh[0], w1 = (T)g.invh[1], w2 = (T)g.invh[2], C = (T)g.C;
        const long long fb = g.N * (long long)E;
        const XBuf sb = xbuf_bytes(g.phi, fb);
        const XBuf ob = xbuf_bytes(g.P[1], fb);
        unsigned toff[NT];
#pragma unroll
        for (int m = 0; m < NT; ++m) toff[m] = xtile_off<H>(t, tid + m * kThreads, E);
        const int gx = t.x0 + cx;
        unsigned vin[kXPY], vown[kXPY];
        int lx;   // the x centre of this thread's fourth difference, in the tile
        {
            const int c = t.px ? gx : min(max(gx, 2), t.n0 - 3);
            lx = c - (t.x0 - H);
        }
        int ly[kXPY];
#pragma unroll
        for (int p = 0; p < kXPY; ++p) {
            const int ry = r0 + kXRow * p, gy = t.y0 + ry;
            const bool in = cx < t.wx && ry < t.wy;
            const bool own = in && gx >= t.tx * kXTX && gy >= t.ty * kXTY;
            const unsigned off = (unsigned)(gy * t.s1 + gx);
            vin[p] = in ? off * E : kXOut;
            vown[p] = own ? off * E : kXOut;
            const int c = t.py ? gy : min(max(gy, 2), t.n1 - 3);
            ly[p] = c - (t.y0 - H);
        }
        // z: the five planes of the fourth difference, zb .. zb + 4 (its
        // centre zb + 2 stays inward of the two planes next to an end)
        auto zbase = [&](int k) { return t.pz ? k - 2 : min(max(k - 2, 0), t.n2 - 5); };
        T zq[kXPY][5];
        int jb = INT_MIN;
        T tv[NT];
#pragma unroll
        for (int m = 0; m < NT; ++m) tv[m] = xload<T>(sb, toff[m], (unsigned)(t.z0 * t.s2) * E);
        lds_barrier();   // the previous item's reads of the tiles are done
#pragma unroll
        for (int m = 0; m < NT; ++m)
            if (m < NT - 1 || tid + m * kThreads < PW * PH) sm[0][tid + m * kThreads] = tv[m];
        int cur = 0;
        for (int k = t.z0; k < t.z1; ++k) {
            const unsigned so = (unsigned)(k * t.s2) * E;
            if (t.d3 && zbase(k) != jb) {
                jb = zbase(k);
#pragma unroll
                for (int p = 0; p < kXPY; ++p)
#pragma unroll
                    for (int m = 0; m < 5; ++m) {
                        int kk = jb + m;
                        kk = kk < 0 ? kk + t.n2 : (kk >= t.n2 ? kk - t.n2 : kk);
                        zq[p][m] = xload<T>(sb, vin[p], (unsigned)(kk * t.s2) * E);
                    }
            }
            const bool adv = t.d3 && k + 1 < t.z1 && zbase(k + 1) == jb + 1;
            lds_barrier();
            const T *ph = sm[cur];
            T znx[kXPY];
            {
                int kn = adv ? jb + 5 : k;
                kn = kn >= t.n2 ? kn - t.n2 : kn;
#pragma unroll
                for (int p = 0; p < kXPY; ++p)
                    znx[p] = xload<T>(sb, vin[p], (unsigned)(kn * t.s2) * E);
                const unsigned sn = (unsigned)(min(k + 1, t.z1 - 1) * t.s2) * E;
#pragma unroll
                for (int m = 0; m < NT; ++m) tv[m] = xload<T>(sb, toff[m], sn);
            }
            T out[kXPY];
#pragma unroll
            for (int p = 0; p < kXPY; ++p) {
                const int ry = r0 + kXRow * p;
                // sum over l in the order x, y, z
                T sx = w0 * xd4<T>(ph + (ry + H) * PW + lx, 1);
                sx = w1 * xd4<T>(ph + ly[p] * PW + cx + H, PW) + sx;
                if (t.d3) sx = w2 * xd4<T>(&zq[p][2], 1) + sx;
                out[p] = C * fabs(sx);
            }
            if (k + 1 < t.z1) {
#pragma unroll
                for (int m = 0; m < NT; ++m)
                    if (m < NT - 1 || tid + m * kThreads < PW * PH)
                        sm[cur ^ 1][tid + m * kThreads] = tv[m];
            }
            cur ^= 1;
#pragma unroll
            for (int p = 0; p < kXPY; ++p) xstore<T>(ob, out[p], vown[p], so);
            if (adv) {
                ++jb;
#pragma unroll
                for (int p = 0; p < kXPY; ++p) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) zq[p][m] = zq[p][m + 1];
                    zq[p][4] = znx[p];
                }
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_xlad_smooth(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems)
{
    constexpr int H = kLadG, SW = kXTX + 2 * H, SH = kXTY + 2 * H;
    constexpr int NT = (SW * SH + kThreads - 1) / kThreads;
    constexpr int NGX = (SH * kXTX + kThreads - 1) / kThreads;
    constexpr unsigned E = sizeof(T);
    __shared__ T st[2][SW * SH];   // sensor tile (this plane's and the next one's)
    __shared__ T gxs[SH * kXTX];   // smoothed along x, rows y0-H .. y0+TY+H-1
    const int tid = threadIdx.x, cx = tid % kXTX, r0 = tid / kXTX;
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        const XTileGeo t = xlad_geo(g, item.tile);
        const long long fb = g.N * (long long)E;
        const XBuf sb = xbuf_bytes(g.P[1], fb);
        const XBuf ob = xbuf_bytes(g.P[2], fb);
        unsigned toff[NT];
#pragma unroll
        for (int m = 0; m < NT; ++m) toff[m] = xtile_off<H>(t, tid + m * kThreads, E);
        const int gx = t.x0 + cx;
        unsigned vown[kXPY];
#pragma unroll
        for (int p = 0; p < kXPY; ++p) {
            const int ry = r0 + kXRow * p, gy = t.y0 + ry;
            const bool own = cx < t.wx && ry < t.wy && gx >= t.tx * kXTX && gy >= t.ty * kXTY;
            vown[p] = own ? (unsigned)(gy * t.s1 + gx) * E : kXOut;
        }
        // tile index of position j along a direction of n points (tile
        // origin o0 - H): periodic lines read the wrapped copies the tile
        // holds, non-periodic ones clamp to the end
        auto tix = [&](int j, int n, bool per, int o0) {
            return (per ? j : min(max(j, 0), n - 1)) - (o0 - H);
        };
        // virtual planes z0 - 4 .. z1 + 3 of the z smoothing, each the
        // plane it reads (clamped or wrapped)
        auto zmap = [&](int v) {
            return t.pz ? (v < 0 ? v + t.n2 : (v >= t.n2 ? v - t.n2 : v))
                        : min(max(v, 0), t.n2 - 1);
        };
        const int v0 = t.d3 ? t.z0 - 4 : 0, v1 = t.d3 ? t.z1 + 4 : 1;
        T zq[kXPY][9];
        T tv[NT];
#pragma unroll
        for (int m = 0; m < NT; ++m)
            tv[m] = xload<T>(sb, toff[m], (unsigned)(zmap(v0) * t.s2) * E);
        lds_barrier();   // the previous item's reads of the tiles are done
#pragma unroll
        for (int m = 0; m < NT; ++m)
            if (m < NT - 1 || tid + m * kThreads < SW * SH) st[0][tid + m * kThreads] = tv[m];
        int cur = 0, aprev = INT_MIN;
        T sxy[kXPY];
        for (int v = v0; v < v1; ++v) {
            const int a = zmap(v);
            if (a != aprev || t.pz) {
                // this plane's sensor tile is in st[cur]
                lds_barrier();
                const T *sp = st[cur];
                const int an = t.pz ? zmap(v + 1) : min(a + 1, t.n2 - 1);
#pragma unroll
                for (int m = 0; m < NT; ++m)
                    tv[m] = xload<T>(sb, toff[m], (unsigned)(an * t.s2) * E);
                // along x, every row of the tile
#pragma unroll
                for (int i = 0; i < NGX; ++i) {
                    const int e = tid + i * kThreads;
                    if (i < NGX - 1 || e < SH * kXTX) {
                        const int r = e / kXTX, c = e - r * kXTX;
                        const int j = t.x0 + c;
                        const T *row = sp + r * SW;
                        T lo[5], hi[5];
#pragma unroll
                        for (int o = 1; o <= 4; ++o) {
                            lo[o] = row[tix(j - o, t.n0, t.px, t.x0)];
                            hi[o] = row[tix(j + o, t.n0, t.px, t.x0)];
                        }
                        gxs[e] = xgauss<T>(row[tix(j, t.n0, t.px, t.x0)], lo, hi);
                    }
                }
                lds_barrier();
                // along y, this thread's points
#pragma unroll
                for (int p = 0; p < kXPY; ++p) {
                    const int gy = t.y0 + r0 + kXRow * p;
                    T lo[5], hi[5];
#pragma unroll
                    for (int o = 1; o <= 4; ++o) {
                        lo[o] = gxs[tix(gy - o, t.n1, t.py, t.y0) * kXTX + cx];
                        hi[o] = gxs[tix(gy + o, t.n1, t.py, t.y0) * kXTX + cx];
                    }
                    sxy[p] = xgauss<T>(gxs[tix(gy, t.n1, t.py, t.y0) * kXTX + cx], lo, hi);
                }
#pragma unroll
                for (int m = 0; m < NT; ++m)
                    if (m < NT - 1 || tid + m * kThreads < SW * SH)
                        st[cur ^ 1][tid + m * kThreads] = tv[m];
                cur ^= 1;
                aprev = a;
            }
            if (!t.d3) {
#pragma unroll
                for (int p = 0; p < kXPY; ++p) xstore<T>(ob, sxy[p], vown[p], 0);
                continue;
            }
            // along z: planes v - 8 .. v in the queue, the output at v - 4
#pragma unroll
            for (int p = 0; p < kXPY; ++p) {
#pragma unroll
                for (int m = 0; m < 8; ++m) zq[p][m] = zq[p][m + 1];
                zq[p][8] = sxy[p];
            }
            if (v >= t.z0 + 4) {
                const unsigned so = (unsigned)((v - 4) * t.s2) * E;
#pragma unroll
                for (int p = 0; p < kXPY; ++p) {
                    T lo[5], hi[5];
#pragma unroll
                    for (int o = 1; o <= 4; ++o) {
                        lo[o] = zq[p][4 - o];
                        hi[o] = zq[p][4 + o];
                    }
                    xstore<T>(ob, xgauss<T>(zq[p][4], lo, hi), vown[p], so);
                }
            }
        }
    }
}

// Advective term of the upwind baseline for grids whose stage finish is
// pointwise (Eikonal): P[1] <- U.grad(phi) of Eqs. UW1-UW5, uw2 <- |U|^2,
// from the stage value, before the finish overwrites it.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_uwadv(const GridDev *__restrict__ grids, const Item *__restrict__ items,
        int nitems, int stage)
{
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        gptr<const T> src = gcast<const T>(stage == 0 ? g.phi : g.ps);
        gptr<T> adv = gcast<T>(g.P[1]);
        gptr<T> u2 = gcast<T>(g.uw2);
        const long long q0 = (long long)item.tile * kChunk;
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long qq = q0 + i;
            if (qq >= g.N) break;
            const int q = (int)qq;
            T m9[9], a, g2;
            metric_load<T>(g, q, m9);
            int idx[3];
            index_of(g, q, idx);
            uw_term<T>(g, src, q, idx, m9, a, g2);
            adv[q] = a;
            u2[q] = g2;
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
    __shared__ double sh[4 * kThreads / 64];
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        if (gmem(g.state)->done) continue;
        gptr<T> phi = gcast<T>(g.phi);
        gptr<const T> ps = gcast<const T>(g.ps);
        const long long q0 = (long long)item.tile * kChunk;
        double mx = 0.0, sm = 0.0, ng = 0.0, mg = 0.0;
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long q = q0 + i;
            if (q >= g.N) break;
            const T nv = ps[q];
            const double e = fabs((double)nv - (double)phi[q]);
            mx = nanmax(mx, e);
            sm += e * e;
            ng = nanmax(ng, -(double)nv);
            mg = nanmax(mg, fabs((double)nv));
            phi[q] = nv;
        }
        block_reduce(mx, sm, ng, mg, sh);
        if (threadIdx.x == 0) put_rpart(g, item.tile, mx, sm, ng, mg);
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
        if (gmem(g.state)->done && target == 1) continue;
        const int code = g.xbc[face];
        if (code == XBC_NONE) continue;
        gptr<T> f = gcast<T>(target ? g.ps : g.phi);
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
            if (wall_point(g, idx) || (g.mask && gmem(g.mask)[q])) continue;
            const T a = f[q + in], b = f[q + 2 * in];
            f[q] = code == XBC_NEUMANN ? ((T)4 * a - b) / (T)3 : (T)2 * a - b;
        }
    }
}

// Initial field (Sec. 3.5): zero (cold) or the given guess, walls/solids
// set to zero; resets the grid's stopping state; copies the caller's
// field-major metrics into the grid's point-major array (the passes read a
// point's metrics with one or two wide loads).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_init(const GridDev *__restrict__ grids, const Item *__restrict__ items,
       int nitems, int unused)
{
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        gptr<T> phi = gcast<T>(g.phi);
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
            const bool zero = !g.warm || wall_point(g, idx) || (g.mask && gmem(g.mask)[q]);
            if (zero) phi[q] = (T)0;
            if (g.rk == 1) gcast<T>(g.acc)[q] = (T)0;   // no carried remainder yet
        }
        if (!g.uniform) {
            // element e of this chunk's point-major block: point e / dd,
            // component e % dd (coalesced writes)
            const int dd = g.ndim * g.ndim;
            gptr<const T> src = gcast<const T>(g.met_src);
            gptr<T> dst = gcast<T>(const_cast<void *>(g.met));
            const long long e0 = q0 * dd;
            const long long e1 = min(g.N, q0 + kChunk) * dd;
            for (long long e = e0 + threadIdx.x; e < e1; e += kThreads) {
                const long long q = e / dd;
                const int c = (int)(e - q * dd);
                dst[e] = src[(long long)c * g.N + q];
            }
        }
    }
}

// Per-grid stopping logic (Eq. Con-criter) on the FP64 partials.
__global__ void __launch_bounds__(kThreads)
k_finalize(const GridDev *__restrict__ grids, int ngrids)
{
    __shared__ double sh[4 * kThreads / 64];
    const GridDev &g = grids[blockIdx.x];
    if (gmem(g.state)->done) return;
    double mx = 0.0, sm = 0.0, ng = 0.0, mg = 0.0;
    for (int i = threadIdx.x; i < g.nparts; i += kThreads) {
        gptr<const double> r = gmem(g.rpart) + 4 * (long long)i;
        mx = nanmax(mx, r[0]);
        sm += r[1];
        ng = nanmax(ng, r[2]);
        mg = nanmax(mg, r[3]);
    }
    block_reduce(mx, sm, ng, mg, sh);
    if (threadIdx.x != 0) return;
    GridState st = *g.state;
    const int it = st.iter;
    const double l2 = sqrt(sm / (double)g.N);
    if (it < g.hist_cap) {
        gmem(g.hist)[2 * it] = mx;
        gmem(g.hist)[2 * it + 1] = l2;
    }
    const int nit = it + 1;
    st.iter = nit;
    st.last = mx;
    if (!(fabs(mx) <= 1.0e300) || !(fabs(l2) <= 1.0e300)) {
        st.status = -3;
        st.done = 1;
    } else if (g.warm_probe > 0 && nit == g.warm_probe && ng > 0.1 * mg) {
        // warm-start guard: after the probe window the field lies below
        // -0.1 of its largest magnitude somewhere -- an undershoot beside a
        // wall that Gamma = 0 cannot damp, which only grows (WD_ERR_WARM_RUNAWAY)
        st.status = -8;
        st.done = 1;
    } else if (mx <= g.tol) {
        st.status = 0;
        st.done = 1;
    } else {
        if (mx < st.best) {
            st.best = mx;
            st.best_iter = nit;
        }
        // the stall window is the rounding floor's: it counts only once the
        // change has come within 10 tol (a moving front keeps the change
        // level for a long time without being stuck)
        if (g.stall > 0 && mx <= 10.0 * g.tol && nit - st.best_iter >= g.stall) {
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

// ---------------------------------------------------------------------
// Level-set burnback (Sec. 5.5, Eq. levelset with its right-hand side read
// as 0): d phi_s / dt = -F |grad phi_s| on a uniform grid, classical RK4 in
// physical time, the upwind switch of Eqs. UW3-UW5 for each one-sided
// difference, zero normal gradient on every non-periodic face.  phi_s is
// positive on the solid side, so the front moves into the solid.

// |grad f| at point q from the switch-selected index differences
template <typename T>
__device__ inline T ls_grad(const GridDev &g, gptr<const T> f, long long q, const int *idx)
{
    T s2 = (T)0;
    const T f0 = f[q];
    for (int l = 0; l < g.ndim; ++l) {
        const int n = g.n[l], i = idx[l];
        const long long s = g.stride[l];
        const bool per = g.periodic[l] != 0;
        const bool hm = i > 0 || per, hp = i < n - 1 || per;
        const long long qm = i > 0 ? q - s : q + (long long)(n - 1) * s;
        const long long qp = i < n - 1 ? q + s : q - (long long)(n - 1) * s;
        T b = hm ? f0 - f[qm] : (T)0;
        T fw = hp ? f[qp] - f0 : (T)0;
        if (!hm) b = fw;
        if (!hp) fw = b;
        T d;
        if (fw + b >= (T)0) d = b >= (T)0 ? b : (T)0;
        else d = fw < (T)0 ? fw : (T)0;
        d *= (T)g.invh[l];
        s2 += d * d;
    }
    return sqrt(s2);
}

// stage buffers: values in phi (start), ps, P[0], ps, phi (end)
template <typename T>
__device__ inline void ls_buffers(const GridDev &g, int stage, gptr<const T> &src, gptr<T> &dst)
{
    void *b[5] = {g.phi, g.ps, g.P[0], g.ps, g.phi};
    src = gcast<const T>(b[stage]);
    dst = gcast<T>(b[stage + 1]);
}

// one RK4 stage over a chunk of points (accumulator form, fdt = F dt)
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_ls_stage(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems,
           int stage, double fdt, int chunk)
{
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        gptr<const T> src;
        gptr<T> dst;
        ls_buffers<T>(g, stage, src, dst);
        gptr<const T> phi = gcast<const T>(g.phi);
        gptr<T> acc = gcast<T>(g.acc);
        const T h = (T)fdt;
        const long long q0 = (long long)item.tile * chunk;
        // the chunk's points of this thread together, so their loads overlap
#pragma unroll
        for (int i = threadIdx.x; i < kLsChunk; i += kThreads) {
            const long long q = q0 + i;
            if (i >= chunk || q >= g.N) continue;
            int idx[3];
            index_of(g, q, idx);
            const T gm = ls_grad<T>(g, src, q, idx);
            if (stage == 0) {
                const T pn = phi[q];
                acc[q] = pn - h * (T)(1.0 / 6.0) * gm;
                dst[q] = pn - h * (T)0.5 * gm;
            } else if (stage == 1) {
                acc[q] = acc[q] - h * (T)(1.0 / 3.0) * gm;
                dst[q] = phi[q] - h * (T)0.5 * gm;
            } else if (stage == 2) {
                acc[q] = acc[q] - h * (T)(1.0 / 3.0) * gm;
                dst[q] = phi[q] - h * gm;
            } else {
                dst[q] = acc[q] - h * (T)(1.0 / 6.0) * gm;
            }
        }
    }
}

// Upwind-switched one-sided difference of one direction (the choice of
// ls_grad), scaled by 1/h: b = f0 - f_minus, fw = f_plus - f0; a missing
// side copies the other (none: zero).
template <typename T>
__device__ inline T ls_side(T b, T fw, bool hm, bool hp, T ih)
{
    if (!hm && !hp) return (T)0;
    if (!hm) b = fw;
    if (!hp) fw = b;
    T d;
    if (fw + b >= (T)0) d = b >= (T)0 ? b : (T)0;
    else d = fw < (T)0 ? fw : (T)0;
    return d * ih;
}

// One RK4 stage on a 2D or 3D grid: lanes along x (one point per thread
// and row, every load coalesced), each thread taking kLsRows rows of one
// z plane (blockIdx.z) with the column of rows shared between them, so a
// point costs three loads of its own row (and two of the planes beside it
// in 3D) and no index division.  Same arithmetic as k_ls_stage.
template <typename T>
__global__ void __launch_bounds__(kLsLanes)
k_ls_stage_rows(const GridDev *__restrict__ grids, int stage, double fdt)
{
    const GridDev &g = grids[0];
    const int n0 = g.n[0], n1 = g.n[1];
    const int x = blockIdx.x * kLsLanes + threadIdx.x;
    const int y0 = blockIdx.y * kLsRows;
    if (x >= n0 || y0 >= n1) return;
    gptr<const T> src;
    gptr<T> dst;
    ls_buffers<T>(g, stage, src, dst);
    gptr<const T> phi = gcast<const T>(g.phi);
    gptr<T> acc = gcast<T>(g.acc);
    const T h = (T)fdt;
    const bool px = g.periodic[0] != 0, py = g.periodic[1] != 0;
    const bool hm0 = x > 0 || px, hp0 = x < n0 - 1 || px;
    const int xm = x > 0 ? x - 1 : n0 - 1, xp = x < n0 - 1 ? x + 1 : 0;
    const T ih0 = (T)g.invh[0], ih1 = (T)g.invh[1];
    const long long s1 = g.stride[1];
    // third direction: this plane and its neighbours' offsets
    const bool three = g.ndim == 3;
    const int z = blockIdx.z, n2 = three ? g.n[2] : 1;
    const long long s2 = three ? g.stride[2] : 0;
    const bool pz = three && g.periodic[2] != 0;
    const bool hm2 = z > 0 || pz, hp2 = z < n2 - 1 || pz;
    const long long plane = (long long)z * s2;
    const long long dzm = z > 0 ? -s2 : (long long)(n2 - 1) * s2;
    const long long dzp = z < n2 - 1 ? s2 : -(long long)(n2 - 1) * s2;
    const T ih2 = three ? (T)g.invh[2] : (T)0;
    // every load before the first store (the stage buffers could alias as
    // far as the compiler knows): the thread's column of rows y0 - 1 ..
    // y0 + nr, then each row's other operands; both loops fully unrolled,
    // so every array index is a constant and the arrays stay in registers
    // (no access past an array's end, not even on a path never taken)
    const int nr = min(kLsRows, n1 - y0);
    T col[kLsRows + 2], lft[kLsRows], rgt[kLsRows], bk[kLsRows], fr[kLsRows];
    T p0[kLsRows], a0[kLsRows];
    col[0] = (T)0;
    if (y0 > 0) col[0] = src[plane + (long long)(y0 - 1) * s1 + x];
    else if (py) col[0] = src[plane + (long long)(n1 - 1) * s1 + x];
#pragma unroll
    for (int r = 0; r <= kLsRows; ++r) {
        const int y = y0 + r;
        T v = (T)0;
        if (r <= nr) {   // rows y0 .. y0 + nr - 1 and the row after them
            if (y < n1) v = src[plane + (long long)y * s1 + x];
            else if (py) v = src[plane + x];
        }
        col[r + 1] = v;
    }
#pragma unroll
    for (int r = 0; r < kLsRows; ++r) {
        lft[r] = rgt[r] = bk[r] = fr[r] = p0[r] = a0[r] = (T)0;
        if (r >= nr) continue;
        const long long row = plane + (long long)(y0 + r) * s1;
        lft[r] = src[row + xm];
        rgt[r] = src[row + xp];
        if (three) {
            bk[r] = src[row + x + dzm];
            fr[r] = src[row + x + dzp];
        }
        if (stage == 1 || stage == 2) p0[r] = phi[row + x];
        if (stage > 0) a0[r] = acc[row + x];
    }
#pragma unroll
    for (int r = 0; r < kLsRows; ++r) {
        if (r >= nr) break;
        const int y = y0 + r;
        const long long q = plane + (long long)y * s1 + x;
        const T here = col[r + 1], below = col[r], above = col[r + 2];
        const bool hm1 = y > 0 || py, hp1 = y < n1 - 1 || py;
        const T d0 = ls_side<T>(here - lft[r], rgt[r] - here, hm0, hp0, ih0);
        const T d1 = ls_side<T>(here - below, above - here, hm1, hp1, ih1);
        T s2sum = (T)0;
        s2sum += d0 * d0;
        s2sum += d1 * d1;
        if (three) {
            const T d2 = ls_side<T>(here - bk[r], fr[r] - here, hm2, hp2, ih2);
            s2sum += d2 * d2;
        }
        const T gm = sqrt(s2sum);
        if (stage == 0) {
            acc[q] = here - h * (T)(1.0 / 6.0) * gm;
            dst[q] = here - h * (T)0.5 * gm;
        } else if (stage == 1) {
            acc[q] = a0[r] - h * (T)(1.0 / 3.0) * gm;
            dst[q] = p0[r] - h * (T)0.5 * gm;
        } else if (stage == 2) {
            acc[q] = a0[r] - h * (T)(1.0 / 3.0) * gm;
            dst[q] = p0[r] - h * gm;
        } else {
            dst[q] = a0[r] - h * (T)(1.0 / 6.0) * gm;
        }
    }
}

// zero normal gradient on both faces normal to l of the stage's output:
// f_b = (4 f_1 - f_2) / 3 along the grid line
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_ls_face(const GridDev *__restrict__ grids, const Item *__restrict__ items, int nitems,
          int l, int stage)
{
    int step, end;
    for (int it = item_begin(nitems, step, end); it < end; it += step) {
        const Item item = items[it];
        const GridDev &g = grids[item.grid];
        gptr<const T> src;
        gptr<T> f;
        ls_buffers<T>(g, stage, src, f);
        const long long nface = g.N / g.n[l];
        const long long k0 = (long long)item.tile * kChunk;
        const long long s = g.stride[l];
        for (int i = threadIdx.x; i < kChunk; i += kThreads) {
            const long long k = k0 + i;
            if (k >= nface) break;
            // face point k in (dir-0, dir-1, dir-2) order with index l removed
            long long q;
            const int n0 = g.n[0];
            if (l == 0) q = k * n0;
            else if (l == 1) q = (k % n0) + (k / n0) * (long long)n0 * g.n[1];
            else q = k;
            const long long qe = q + (long long)(g.n[l] - 1) * s;
            f[q] = ((T)4 * f[q + s] - f[q + 2 * s]) * (T)(1.0 / 3.0);
            f[qe] = ((T)4 * f[qe - s] - f[qe - 2 * s]) * (T)(1.0 / 3.0);
        }
    }
}

// The zero-gradient faces of a 2D stage output (both directions, at least
// 4 x 4 points) in one launch, with the result of the x faces followed by
// the y faces: thread t < n1 takes the x faces of row t (rows 1 .. n1 - 2;
// the y faces overwrite rows 0 and n1 - 1, so with y faces present those
// rows are skipped), thread n1 + i the y faces of column i.  A corner
// column's y face reads rows 1, 2 (n1 - 2, n1 - 3) after their x faces, so
// it forms those two values itself from the same interior points.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_ls_face2d(const GridDev *__restrict__ grids, int stage)
{
    const GridDev &g = grids[0];
    gptr<const T> src;
    gptr<T> f;
    ls_buffers<T>(g, stage, src, f);
    const int n0 = g.n[0], n1 = g.n[1];
    const bool xf = !g.periodic[0], yf = !g.periodic[1];
    const long long s1 = g.stride[1];
    const T third = (T)(1.0 / 3.0);
    const long long t = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (t < n1) {
        const int y = (int)t;
        if (!xf || (yf && (y == 0 || y == n1 - 1))) return;
        const long long r = (long long)y * s1;
        f[r] = ((T)4 * f[r + 1] - f[r + 2]) * third;
        f[r + n0 - 1] = ((T)4 * f[r + n0 - 2] - f[r + n0 - 3]) * third;
        return;
    }
    if (t >= (long long)n1 + n0 || !yf) return;
    const int x = (int)(t - n1);
    // value of row y at column x as the x faces leave it
    auto at = [&](int y) -> T {
        const long long r = (long long)y * s1;
        if (xf && x == 0) return ((T)4 * f[r + 1] - f[r + 2]) * third;
        if (xf && x == n0 - 1) return ((T)4 * f[r + n0 - 2] - f[r + n0 - 3]) * third;
        return f[r + x];
    };
    f[x] = ((T)4 * at(1) - at(2)) * third;
    f[(long long)(n1 - 1) * s1 + x] = ((T)4 * at(n1 - 2) - at(n1 - 3)) * third;
}

// phi_s = d_solid on solid points, -d_gas elsewhere
template <typename T>
__global__ void k_ls_signed(long long n, const unsigned char *__restrict__ solid,
                            const T *__restrict__ ds, const T *__restrict__ dg, T *__restrict__ out)
{
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        out[q] = solid[q] ? ds[q] : -dg[q];
}

// Lengths of the iso-lines phi = levels[k] of a uniform 2D grid (linear
// interpolation on the cell edges, a saddle split by the cell mean): FP64
// partial sums per workgroup and level, [block][level].
struct LsLevels {
    double v[kMaxLevels];
    int n;
};

template <typename T>
__device__ inline double ls_cell_length(const T *c, double level, double hx, double hy)
{
    // corners counter-clockwise from (i, j)
    const double v[4] = {(double)c[0] - level, (double)c[1] - level, (double)c[2] - level,
                         (double)c[3] - level};
    const double cx[4] = {0.0, hx, hx, 0.0}, cy[4] = {0.0, 0.0, hy, hy};
    double px[4] = {0.0, 0.0, 0.0, 0.0}, py[4] = {0.0, 0.0, 0.0, 0.0};
    int np = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int a = e, b = (e + 1) & 3;
        if ((v[a] >= 0.0) != (v[b] >= 0.0)) {
            const double t = v[a] / (v[a] - v[b]);
            const double x = cx[a] + t * (cx[b] - cx[a]), y = cy[a] + t * (cy[b] - cy[a]);
            px[np] = x;   // np < 4 here: at most four edges cross
            py[np] = y;
            ++np;
        }
    }
    if (np == 2) return hypot(px[1] - px[0], py[1] - py[0]);
    if (np != 4) return 0.0;
    const double mean = 0.25 * (v[0] + v[1] + v[2] + v[3]);
    if ((mean >= 0.0) == (v[0] >= 0.0))
        return hypot(px[1] - px[0], py[1] - py[0]) + hypot(px[3] - px[2], py[3] - py[2]);
    return hypot(px[3] - px[0], py[3] - py[0]) + hypot(px[2] - px[1], py[2] - py[1]);
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_ls_length(const T *__restrict__ phi, int nx, int ny, double hx, double hy, LsLevels lv,
            double *__restrict__ part)
{
    __shared__ double sh[kMaxLevels][kThreads / 64];
    double acc[kMaxLevels];
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) acc[k] = 0.0;
    const long long cells = (long long)(nx - 1) * (ny - 1);
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
         c += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(c / (nx - 1)), i = (int)(c - (long long)j * (nx - 1));
        const long long q = (long long)j * nx + i;
        const T cv[4] = {phi[q], phi[q + 1], phi[q + nx + 1], phi[q + nx]};
#pragma unroll
        for (int k = 0; k < kMaxLevels; ++k)
            if (k < lv.n) acc[k] += ls_cell_length<T>(cv, lv.v[k], hx, hy);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kMaxLevels; ++k) {
        double a = acc[k];
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
        if (lane == 0) sh[k][wv] = a;
    }
    __syncthreads();
    if (threadIdx.x < kMaxLevels) {
        double a = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) a += sh[threadIdx.x][w];
        part[(long long)blockIdx.x * kMaxLevels + threadIdx.x] = a;
    }
}

void launch_ls_stage(int fp64, const GridDev *g, const Item *it, int nitems, int stage,
                     double fdt, int chunk, int nwg, hipStream_t s)
{
    if (nitems <= 0) return;
    nwg = std::min(nwg, nitems);
    if (fp64)
        hipLaunchKernelGGL(k_ls_stage<double>, dim3(nwg), dim3(kThreads), 0, s, g, it, nitems,
                           stage, fdt, chunk);
    else
        hipLaunchKernelGGL(k_ls_stage<float>, dim3(nwg), dim3(kThreads), 0, s, g, it, nitems,
                           stage, fdt, chunk);
}

int launch_ls_stage_rows(int fp64, const GridDev *g, int n0, int n1, int n2, int stage,
                         double fdt, hipStream_t s)
{
    const long long bx = (n0 + kLsLanes - 1) / kLsLanes;
    const long long by = (n1 + kLsRows - 1) / kLsRows;
    if (bx < 1 || by < 1 || n2 < 1 || bx > 0x7fffffffLL || by > 65535 || n2 > 65535)
        return -1;
    dim3 grid((unsigned)bx, (unsigned)by, (unsigned)n2), block(kLsLanes);
    if (fp64)
        hipLaunchKernelGGL(k_ls_stage_rows<double>, grid, block, 0, s, g, stage, fdt);
    else
        hipLaunchKernelGGL(k_ls_stage_rows<float>, grid, block, 0, s, g, stage, fdt);
    return 0;
}

void launch_ls_face2d(int fp64, const GridDev *g, int n0, int n1, int stage, hipStream_t s)
{
    const long long n = (long long)n0 + n1;
    dim3 grid((unsigned)((n + kThreads - 1) / kThreads)), block(kThreads);
    if (fp64)
        hipLaunchKernelGGL(k_ls_face2d<double>, grid, block, 0, s, g, stage);
    else
        hipLaunchKernelGGL(k_ls_face2d<float>, grid, block, 0, s, g, stage);
}

void launch_ls_face(int fp64, const GridDev *g, const Item *it, int nitems, int l, int stage,
                    int nwg, hipStream_t s)
{
    if (nitems <= 0) return;
    nwg = std::min(nwg, nitems);
    if (fp64)
        hipLaunchKernelGGL(k_ls_face<double>, dim3(nwg), dim3(kThreads), 0, s, g, it, nitems,
                           l, stage);
    else
        hipLaunchKernelGGL(k_ls_face<float>, dim3(nwg), dim3(kThreads), 0, s, g, it, nitems,
                           l, stage);
}

void launch_ls_signed(int fp64, long long n, const unsigned char *solid, const void *ds,
                      const void *dg, void *out, hipStream_t s)
{
    if (n <= 0) return;
    const int nb = (int)std::min<long long>((n + kThreads - 1) / kThreads, 4096);
    if (fp64)
        hipLaunchKernelGGL(k_ls_signed<double>, dim3(nb), dim3(kThreads), 0, s, n, solid,
                           static_cast<const double *>(ds), static_cast<const double *>(dg),
                           static_cast<double *>(out));
    else
        hipLaunchKernelGGL(k_ls_signed<float>, dim3(nb), dim3(kThreads), 0, s, n, solid,
                           static_cast<const float *>(ds), static_cast<const float *>(dg),
                           static_cast<float *>(out));
}

void launch_ls_length(int fp64, const void *phi, int nx, int ny, double hx, double hy,
                      const double *levels, int nlev, double *part, int nb, hipStream_t s)
{
    LsLevels lv;
    lv.n = nlev;
    for (int k = 0; k < kMaxLevels; ++k) lv.v[k] = k < nlev ? levels[k] : 0.0;
    if (fp64)
        hipLaunchKernelGGL(k_ls_length<double>, dim3(nb), dim3(kThreads), 0, s,
                           static_cast<const double *>(phi), nx, ny, hx, hy, lv, part);
    else
        hipLaunchKernelGGL(k_ls_length<float>, dim3(nb), dim3(kThreads), 0, s,
                           static_cast<const float *>(phi), nx, ny, hx, hy, lv, part);
}

// field-major metrics [c][q] -> point-major [q][c] (dd components)
template <typename T>
__global__ void k_met_points(const T *__restrict__ src, T *__restrict__ dst, long long N, int dd)
{
    const long long n = N * dd;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const long long q = e / dd;
        dst[e] = src[(e - q * dd) * N + q];
    }
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

// Conservative metric form (3D): the coordinate products
//   Q[p][m] = x_b J[a][p] - x_a J[b][p]   ((m, a, b) cyclic; J[a][p] = D_p x_a)
// whose derivatives give J xi_{l,m} in curl form.
__global__ void k_gcl_products(const double *__restrict__ x, const double *__restrict__ J,
                               double *__restrict__ Q, long long N)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N;
         q += (long long)gridDim.x * blockDim.x) {
        double xv[3], a[3][3];
        for (int m = 0; m < 3; ++m) xv[m] = x[m * N + q];
        for (int m = 0; m < 3; ++m)
            for (int l = 0; l < 3; ++l) a[m][l] = J[(m * 3 + l) * N + q];
        for (int p = 0; p < 3; ++p)
            for (int m = 0; m < 3; ++m) {
                const int ia = (m + 1) % 3, ib = (m + 2) % 3;
                Q[(p * 3 + m) * N + q] = xv[ib] * a[ia][p] - xv[ia] * a[ib][p];
            }
    }
}

// xi_{l,m} = (D_q Q[p][m] - D_p Q[q][m]) / (2 det J)  ((l, p, q) cyclic);
// D[(l * 3 + m) * 2] holds D_q Q[p][m], D[(l * 3 + m) * 2 + 1] D_p Q[q][m]
template <typename T>
__global__ void k_gcl_combine(const double *__restrict__ J, const double *__restrict__ D,
                              T *__restrict__ out, long long N)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < N;
         q += (long long)gridDim.x * blockDim.x) {
        double a[3][3];
        for (int m = 0; m < 3; ++m)
            for (int l = 0; l < 3; ++l) a[m][l] = J[(m * 3 + l) * N + q];
        const double det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1])
                         - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
                         + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
        for (int l = 0; l < 3; ++l)
            for (int m = 0; m < 3; ++m) {
                const int k = (l * 3 + m) * 2;
                out[(l * 3 + m) * N + q] = (T)(0.5 * (D[k * N + q] - D[(k + 1) * N + q]) / det);
            }
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
                u += (double)metric<T>(g, l, m, q) * gcast<const double>(g.F[l])[q];
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
static void point_launch(int kind, const GridDev *g, const Item *it, int nitems,
                         int l, int stage, int nwg, hipStream_t s, int np = 1)
{
    dim3 grid(nwg), block(kThreads);
    switch (kind) {
    case PASS_FINAL: hipLaunchKernelGGL(k_final<T>, grid, block, 0, s, g, it, nitems, stage); break;
    case PASS_CFIN: hipLaunchKernelGGL(k_cart_finish<T>, grid, block, 0, s, g, it, nitems, stage); break;
    // explicit one-pass stages: l carries the scheme radius
    case PASS_XSTAGE:
        if (np == 2) {
            if (l == 1) hipLaunchKernelGGL((k_xstage<T, 1, true>), grid, block, 0, s, g, it, nitems, stage);
            else if (l == 2) hipLaunchKernelGGL((k_xstage<T, 2, true>), grid, block, 0, s, g, it, nitems, stage);
            else hipLaunchKernelGGL((k_xstage<T, 3, true>), grid, block, 0, s, g, it, nitems, stage);
        } else {
            if (l == 1) hipLaunchKernelGGL((k_xstage<T, 1, false>), grid, block, 0, s, g, it, nitems, stage);
            else if (l == 2) hipLaunchKernelGGL((k_xstage<T, 2, false>), grid, block, 0, s, g, it, nitems, stage);
            else hipLaunchKernelGGL((k_xstage<T, 3, false>), grid, block, 0, s, g, it, nitems, stage);
        }
        break;
    case PASS_XLAD:
        if (np == 2) hipLaunchKernelGGL(k_xlad_smooth<T>, grid, block, 0, s, g, it, nitems);
        else hipLaunchKernelGGL(k_xlad_sens<T>, grid, block, 0, s, g, it, nitems);
        break;
    case PASS_UWADV: hipLaunchKernelGGL(k_uwadv<T>, grid, block, 0, s, g, it, nitems, stage); break;
    case PASS_RESID: hipLaunchKernelGGL(k_resid<T>, grid, block, 0, s, g, it, nitems); break;
    case PASS_FACE: hipLaunchKernelGGL(k_face<T>, grid, block, 0, s, g, it, nitems, l, stage); break;
    case PASS_INIT: hipLaunchKernelGGL(k_init<T>, grid, block, 0, s, g, it, nitems, stage); break;
    default: break;
    }
}

void launch_pass(int kind, int fp64, int np, const GridDev *g, const Item *it, int nitems,
                 int l, int stage, int nwg, hipStream_t s)
{
    if (nitems <= 0) return;
    if (nwg > nitems) nwg = nitems;
    switch (kind) {
    case PASS_FINAL:
    case PASS_CFIN:
    case PASS_XSTAGE:
    case PASS_XLAD:
    case PASS_UWADV:
    case PASS_RESID:
    case PASS_FACE:
    case PASS_INIT:
        if (fp64) point_launch<double>(kind, g, it, nitems, l, stage, nwg, s, np);
        else point_launch<float>(kind, g, it, nitems, l, stage, nwg, s, np);
        return;
    default:
        break;
    }
    if (fp64) {
        switch (np) {
        case 1: line_launch_f64_1(kind, g, it, nitems, l, stage, nwg, s); break;
        case 2: line_launch_f64_2(kind, g, it, nitems, l, stage, nwg, s); break;
        case 4: line_launch_f64_4(kind, g, it, nitems, l, stage, nwg, s); break;
        default: line_launch_f64_8(kind, g, it, nitems, l, stage, nwg, s); break;
        }
    } else {
        switch (np) {
        case 1: line_launch_f32_1(kind, g, it, nitems, l, stage, nwg, s); break;
        case 2: line_launch_f32_2(kind, g, it, nitems, l, stage, nwg, s); break;
        case 4: line_launch_f32_4(kind, g, it, nitems, l, stage, nwg, s); break;
        default: line_launch_f32_8(kind, g, it, nitems, l, stage, nwg, s); break;
        }
    }
}

template <typename T>
static const void *xstage_fn(int r, bool fast)
{
    if (fast)
        return r == 1 ? reinterpret_cast<const void *>(&k_xstage<T, 1, true>)
             : r == 2 ? reinterpret_cast<const void *>(&k_xstage<T, 2, true>)
                      : reinterpret_cast<const void *>(&k_xstage<T, 3, true>);
    return r == 1 ? reinterpret_cast<const void *>(&k_xstage<T, 1, false>)
         : r == 2 ? reinterpret_cast<const void *>(&k_xstage<T, 2, false>)
                  : reinterpret_cast<const void *>(&k_xstage<T, 3, false>);
}

int xstage_blocks_per_cu(int fp64, int r, int fast)
{
    static std::atomic<int> cache[2][3][2];
    if (r < 1 || r > 3) return 1;
    std::atomic<int> &c = cache[fp64 ? 1 : 0][r - 1][fast ? 1 : 0];
    int v = c.load(std::memory_order_relaxed);
    if (v > 0) return v;
    const void *f = fp64 ? xstage_fn<double>(r, fast != 0) : xstage_fn<float>(r, fast != 0);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kThreads, 0) != hipSuccess) n = 0;
    v = std::max(1, n);
    c.store(v, std::memory_order_relaxed);
    return v;
}

int xlad_blocks_per_cu(int fp64, int np)
{
    static std::atomic<int> cache[2][2];
    std::atomic<int> &c = cache[fp64 ? 1 : 0][np == 2 ? 1 : 0];
    int v = c.load(std::memory_order_relaxed);
    if (v > 0) return v;
    const void *f;
    if (fp64)
        f = np == 2 ? reinterpret_cast<const void *>(&k_xlad_smooth<double>)
                    : reinterpret_cast<const void *>(&k_xlad_sens<double>);
    else
        f = np == 2 ? reinterpret_cast<const void *>(&k_xlad_smooth<float>)
                    : reinterpret_cast<const void *>(&k_xlad_sens<float>);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kThreads, 0) != hipSuccess) n = 0;
    v = std::max(1, n);
    c.store(v, std::memory_order_relaxed);
    return v;
}

int line_blocks_per_cu(int kind, int fp64, int np)
{
    if (fp64) {
        switch (np) {
        case 1: return line_launch_f64_1_occ(kind);
        case 2: return line_launch_f64_2_occ(kind);
        case 4: return line_launch_f64_4_occ(kind);
        default: return line_launch_f64_8_occ(kind);
        }
    }
    switch (np) {
    case 1: return line_launch_f32_1_occ(kind);
    case 2: return line_launch_f32_2_occ(kind);
    case 4: return line_launch_f32_4_occ(kind);
    default: return line_launch_f32_8_occ(kind);
    }
}

void launch_met_points(int fp64, const void *src, void *dst, long long N, int dd, hipStream_t s)
{
    if (N <= 0 || !src || !dst) return;
    const long long n = N * dd;
    const int nb = (int)std::min<long long>((n + kThreads - 1) / kThreads, 4096);
    if (fp64)
        hipLaunchKernelGGL(k_met_points<double>, dim3(nb), dim3(kThreads), 0, s,
                           static_cast<const double *>(src), static_cast<double *>(dst), N, dd);
    else
        hipLaunchKernelGGL(k_met_points<float>, dim3(nb), dim3(kThreads), 0, s,
                           static_cast<const float *>(src), static_cast<float *>(dst), N, dd);
}

void launch_mirror(const GridDev *g, int ngrids, hipStream_t s)
{
    if (ngrids <= 0) return;
    hipLaunchKernelGGL(k_mirror, dim3((ngrids + 255) / 256), dim3(256), 0, s, g, ngrids);
}

// Scratch of the calls that allocate nothing: workspace and line-operator
// tables of one solve, one copy per GPU the library runs on, held until the
// process ends.  Host code must use the address hipGetSymbolAddress gives
// for the current device, never the array's name.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

int noalloc_scratch(int device, void **ptr)
{
    static std::mutex mu;
    static void *addr[64] = {nullptr};
    if (device < 0 || device >= 64) return -5;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) return -5;
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -5;
        addr[device] = p;
    }
    *ptr = addr[device];
    return 0;
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

void launch_gcl_products(const double *x, const double *J, double *Q, long long N, hipStream_t s)
{
    dim3 grid(blocks_for(N)), block(kThreads);
    hipLaunchKernelGGL(k_gcl_products, grid, block, 0, s, x, J, Q, N);
}

void launch_gcl_combine(const double *J, const double *D, void *out, int out_fp64, long long N,
                        hipStream_t s)
{
    dim3 grid(blocks_for(N)), block(kThreads);
    if (out_fp64)
        hipLaunchKernelGGL(k_gcl_combine<double>, grid, block, 0, s, J, D, (double *)out, N);
    else
        hipLaunchKernelGGL(k_gcl_combine<float>, grid, block, 0, s, J, D, (float *)out, N);
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
