// wd_host.cpp -- host side of the wall-distance library: contexts, line
// operator tables, batch planning, graph-captured iteration and the C ABI
// entry points declared in include/wd.h (except the server).
#include "wd_host.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace wd {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// ---------------------------------------------------------------------
// Line systems.  Rows a_i x_{i-1} + b_i x_i + c_i x_{i+1}; for periodic
// lines a_0 multiplies x_{n-1} and c_{n-1} multiplies x_0.

// compact first derivative (Sec. 3.2): interior (al, 1, al); non-periodic
// ends: the fourth-order one-sided relation f'_0 + 3 f'_1 (and mirror),
// and for C6 the C4 row (1/4, 1, 1/4) next to it.
static void deriv_rows(int n, int periodic, int scheme, std::vector<double> &a,
                       std::vector<double> &b, std::vector<double> &c)
{
    const double al = scheme == SCHEME_C4 ? 0.25 : 1.0 / 3.0;
    a.assign(n, al);
    b.assign(n, 1.0);
    c.assign(n, al);
    if (periodic) return;
    a[0] = 0.0; c[0] = 3.0;
    a[n - 1] = 3.0; c[n - 1] = 0.0;
    if (scheme == SCHEME_C6) {
        a[1] = c[1] = 0.25;
        a[n - 2] = c[n - 2] = 0.25;
    }
}

// filter correction (Sec. 3.4): (af, 1, af); non-periodic boundary points
// are not filtered (identity rows with zero right-hand side).
static void filter_rows(int n, int periodic, double af, std::vector<double> &a,
                        std::vector<double> &b, std::vector<double> &c)
{
    a.assign(n, af);
    b.assign(n, 1.0);
    c.assign(n, af);
    if (periodic) return;
    a[0] = c[0] = 0.0;
    a[n - 1] = c[n - 1] = 0.0;
}

// Parallel cyclic reduction of a fixed matrix, FP64.  Level k folds the
// rows at distance s = 2^k (mod n) into each row: multipliers
//   left_i = -a_i / b_{i-s},  right_i = -c_i / b_{i+s}.
// Stops when every row's off-diagonal weight is below `tol` relative to its
// diagonal, or, on a periodic line, when the distance wraps onto the point
// itself (then the couplings fold into the diagonal exactly).
int pcr_reduce(int n, int periodic, std::vector<double> a, std::vector<double> b,
               std::vector<double> c, double tol, std::vector<int> &smod,
               std::vector<double> &left, std::vector<double> &right,
               std::vector<double> &scale)
{
    smod.clear();
    left.clear();
    right.clear();
    long long s = 1;
    int lev = 0;
    for (;;) {
        double worst = 0.0;
        for (int i = 0; i < n; ++i)
            worst = std::max(worst, (std::fabs(a[i]) + std::fabs(c[i])) / std::fabs(b[i]));
        if (worst <= tol) break;
        if (periodic && s % n == 0) {
            for (int i = 0; i < n; ++i) {
                b[i] += a[i] + c[i];
                a[i] = c[i] = 0.0;
            }
            break;
        }
        if (!periodic && s >= n) break;
        if (lev == kMaxLev) return -1;
        const int sm = (int)(periodic ? s % n : s);
        std::vector<double> a2(n), b2(n), c2(n);
        left.resize((size_t)(lev + 1) * n);
        right.resize((size_t)(lev + 1) * n);
        for (int i = 0; i < n; ++i) {
            int im = i - sm, ip = i + sm;
            const bool hm = periodic || im >= 0;
            const bool hp = periodic || ip < n;
            if (periodic) {
                im = (im + n) % n;
                ip = ip % n;
            }
            const double L = hm ? -a[i] / b[im] : 0.0;
            const double R = hp ? -c[i] / b[ip] : 0.0;
            a2[i] = hm ? L * a[im] : 0.0;
            c2[i] = hp ? R * c[ip] : 0.0;
            b2[i] = b[i] + (hm ? L * c[im] : 0.0) + (hp ? R * a[ip] : 0.0);
            left[(size_t)lev * n + i] = L;
            right[(size_t)lev * n + i] = R;
        }
        a.swap(a2);
        b.swap(b2);
        c.swap(c2);
        smod.push_back(sm);
        ++lev;
        s *= 2;
    }
    scale.resize(n);
    for (int i = 0; i < n; ++i) scale[i] = 1.0 / b[i];
    return lev;
}

static double pcr_tol(int fp64) { return fp64 ? std::ldexp(1.0, -57) : std::ldexp(1.0, -30); }

int build_line_system(int kind, int n, int periodic, int scheme, double af,
                      int fp64, std::vector<int> &smod, std::vector<double> &left,
                      std::vector<double> &right, std::vector<double> &scale)
{
    std::vector<double> a, b, c;
    if (kind == OP_FILTER)
        filter_rows(n, periodic, af, a, b, c);
    else
        deriv_rows(n, periodic, scheme, a, b, c);
    return pcr_reduce(n, periodic, a, b, c, pcr_tol(fp64), smod, left, right, scale);
}

const LineOpDev *ctx_lineop(wd_ctx *ctx, int kind, int n, int periodic, int scheme,
                            double af, int fp64, TableArena *ar)
{
    OpKey key{kind, n, periodic, kind == OP_FILTER ? -1 : scheme, fp64,
              kind == OP_FILTER ? af : 0.0};
    if (ar) {
        for (auto &kv : ar->ops)
            if (!(kv.first < key) && !(key < kv.first)) return &kv.second.dev;
    } else {
        auto it = ctx->ops.find(key);
        if (it != ctx->ops.end()) return &it->second.dev;
    }
    OpEntry e;
    std::memset(&e.dev, 0, sizeof e.dev);
    e.dev.n = n;
    e.dev.periodic = periodic;
    const bool solve = kind == OP_FILTER || scheme == SCHEME_C4 || scheme == SCHEME_C6;
    std::vector<int> smod;
    std::vector<double> left, right, scale;
    int nlev = 0;
    if (solve) {
        nlev = build_line_system(kind, n, periodic, scheme, af, fp64, smod, left, right, scale);
        if (nlev < 0) {
            fail(WD_ERR_UNSUPPORTED, "line system (n=%d) did not reduce within %d levels", n, kMaxLev);
            return nullptr;
        }
    } else {
        scale.assign(n, 1.0);
    }
    e.dev.nlev = nlev;
    for (int k = 0; k < nlev; ++k) e.dev.smod[k] = smod[k];
    // periodic constant-coefficient lines reduce to the same multipliers on
    // every row: keep them as per-level scalars
    bool uniform = true;
    for (int k = 0; k < nlev && uniform; ++k)
        for (int i = 1; i < n && uniform; ++i)
            uniform = left[(size_t)k * n + i] == left[(size_t)k * n] &&
                      right[(size_t)k * n + i] == right[(size_t)k * n];
    for (int i = 1; i < n && uniform; ++i) uniform = scale[i] == scale[0];
    e.dev.uniform = uniform ? 1 : 0;
    if (uniform) {
        for (int k = 0; k < nlev; ++k) {
            e.dev.lr[k][0] = left[(size_t)k * n];
            e.dev.lr[k][1] = right[(size_t)k * n];
        }
        e.dev.usc = scale[0];
    }
    const size_t es = fp64 ? 8 : 4;
    const size_t tab_bytes = (size_t)nlev * n * 2 * es;
    const size_t bytes = tab_bytes + (size_t)n * es + 256;
    std::vector<unsigned char> host(bytes, 0);
    for (size_t i = 0; i < (size_t)nlev * n; ++i) {
        if (fp64) {
            double *t = reinterpret_cast<double *>(host.data());
            t[2 * i] = left[i];
            t[2 * i + 1] = right[i];
        } else {
            float *t = reinterpret_cast<float *>(host.data());
            t[2 * i] = (float)left[i];
            t[2 * i + 1] = (float)right[i];
        }
    }
    const size_t soff = (tab_bytes + 255) & ~(size_t)255;
    for (int i = 0; i < n; ++i) {
        if (fp64)
            reinterpret_cast<double *>(host.data() + soff)[i] = scale[i];
        else
            reinterpret_cast<float *>(host.data() + soff)[i] = (float)scale[i];
    }
    void *mem = nullptr;
    if (ar) {
        mem = ar->carve(bytes);
        if (!mem) {
            fail(WD_ERR_NO_MEMORY, "line-operator tables exceed the %zu-byte scratch", ar->cap);
            return nullptr;
        }
        ar->host.push_back(std::move(host));
        if (hipMemcpyAsync(mem, ar->host.back().data(), bytes, hipMemcpyHostToDevice, ar->stream) !=
            hipSuccess) {
            fail(WD_ERR_HIP, "upload of a line operator failed");
            return nullptr;
        }
    } else {
        if (hipMalloc(&mem, bytes) != hipSuccess) {
            fail(WD_ERR_NO_MEMORY, "hipMalloc of %zu bytes for a line operator failed", bytes);
            return nullptr;
        }
        if (hipMemcpy(mem, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(mem);
            fail(WD_ERR_HIP, "upload of a line operator failed");
            return nullptr;
        }
    }
    e.mem = ar ? nullptr : mem;
    e.dev.tab = mem;
    e.dev.scale = static_cast<unsigned char *>(mem) + soff;
    if (ar) {
        ar->ops.emplace_back(key, e);
        return &ar->ops.back().second.dev;
    }
    auto ins = ctx->ops.emplace(key, e);
    return &ins.first->second.dev;
}

// ---------------------------------------------------------------------
// Segmented line systems.  The rows of a line (the same a, b, c as above)
// are split into S segments of m = ceil(n / S) rows; every segment is
// factored on its own (no coupling to its neighbours), and its two
// coupling columns (the previous segment's last unknown through a_{b_s},
// the next segment's first through c_{e_s - 1}) are solved against the
// segment's block once: the spikes vv, ww.  The true end values of all
// segments then solve a 2S x 2S reduced system whose right-hand side is
// the segments' local end values; its inverse, computed here in FP64,
// gives each segment the two neighbouring values it needs.

// Segmentation of a line of n points (SegGeo): segments of M = 32, 24 or
// 16 positions (FP64: 16, 24, 32, the first that fits), at most 16 of them; the one shorter segment (if M does not
// divide n) holds >= 2 positions and sits second (>= 3 segments) or first
// (2 segments, >= 5 positions), so the first and last segments hold the
// line's five end rows at fixed positions; a single segment must be full.
// Returns false when no M fits.
bool seg_plan(int n, int fp64, SegGeo &sg, int prefer)
{
    std::memset(&sg, 0, sizeof sg);
    // FP64 segments of 16 first (twice the registers per value); `prefer`
    // (16, 24, 32) tries that length first
    int order[4] = {32, 24, 16, 0};
    if (fp64) {
        order[0] = 16;
        order[2] = 32;
    }
    if (prefer == 16 || prefer == 24 || prefer == 32) {
        order[3] = order[0];
        order[0] = prefer;
    }
    for (int M : order) {
        if (M == 0) break;
        const int S = (n + M - 1) / M;
        const int r = n - (S - 1) * M;
        if (S > 16) continue;
        int ks, bk;
        if (r == M) {
            ks = S;
            bk = n;
        } else if (S == 1) {
            continue;
        } else if (S == 2) {
            if (r < 5) continue;
            ks = 0;
            bk = 0;
        } else {
            if (r < 2) continue;
            ks = 1;
            bk = M;
        }
        sg.S = S;
        sg.W = 64 / S;
        sg.M = M;
        sg.ks = ks;
        sg.bk = bk;
        sg.r = ks < S ? r : M;
        // line pitch: >= n + S slots, = S (M + 1) mod 64, so lane w S + s
        // starts its segment near (M + 1)(w S + s) mod 64: distinct banks
        int P = n + S;
        while ((P - S * (M + 1)) % 64 != 0) ++P;
        sg.P = P;
        sg.xsize = sg.W * P;
        return true;
    }
    return false;
}

// first position and length of segment s
static void seg_bounds(const SegGeo &sg, int s, int &b, int &len)
{
    if (s < sg.ks) {
        b = s * sg.M;
        len = sg.M;
    } else if (s == sg.ks) {
        b = sg.bk;
        len = sg.r;
    } else {
        b = sg.bk + sg.r + (s - sg.ks - 1) * sg.M;
        len = sg.M;
    }
}

int build_seg_tables(int kind, int n, int periodic, int scheme, double af, const SegGeo &sg,
                     std::vector<double> &out)
{
    std::vector<double> a, b, c;
    if (kind == OP_FILTER)
        filter_rows(n, periodic, af, a, b, c);
    else
        deriv_rows(n, periodic, scheme, a, b, c);
    const int S = sg.S;
    out.assign((size_t)5 * n + (size_t)4 * S * S, 0.0);
    double *ell = &out[0], *ib = &out[n], *cb = &out[2 * (size_t)n];
    double *vv = &out[3 * (size_t)n], *ww = &out[4 * (size_t)n], *red = &out[5 * (size_t)n];
    std::vector<double> beta(n), y(n), x(n);
    std::vector<int> sb(S), se(S);
    for (int s = 0; s < S; ++s) {
        int bs, len;
        seg_bounds(sg, s, bs, len);
        if (len < 2 || bs + len > n) return -1;
        sb[s] = bs;
        se[s] = bs + len;
    }
    if (se[S - 1] != n) return -1;
    // local solve of segment [bs, es) for right-hand side y, result in x
    auto local = [&](int bs, int es) {
        for (int j = bs + 1; j < es; ++j) y[j] -= ell[j] * y[j - 1];
        x[es - 1] = ib[es - 1] * y[es - 1];
        for (int j = es - 2; j >= bs; --j) x[j] = ib[j] * y[j] - cb[j] * x[j + 1];
    };
    for (int s = 0; s < S; ++s) {
        const int bs = sb[s], es = se[s];
        beta[bs] = b[bs];
        ell[bs] = 0.0;
        for (int j = bs + 1; j < es; ++j) {
            ell[j] = a[j] / beta[j - 1];
            beta[j] = b[j] - ell[j] * c[j - 1];
        }
        for (int j = bs; j < es; ++j) {
            if (beta[j] == 0.0) return -1;
            ib[j] = 1.0 / beta[j];
            cb[j] = j < es - 1 ? c[j] / beta[j] : 0.0;
        }
        const bool prev = s > 0 || periodic, next = s < S - 1 || periodic;
        for (int j = bs; j < es; ++j) y[j] = 0.0;
        y[bs] = prev ? a[bs] : 0.0;
        local(bs, es);
        for (int j = bs; j < es; ++j) vv[j] = x[j];
        for (int j = bs; j < es; ++j) y[j] = 0.0;
        y[es - 1] = next ? c[es - 1] : 0.0;
        local(bs, es);
        for (int j = bs; j < es; ++j) ww[j] = x[j];
    }
    // reduced system over u = (first_0..first_{S-1}, last_0..last_{S-1})
    const int R = 2 * S;
    std::vector<double> Mx((size_t)R * R, 0.0), Inv((size_t)R * R, 0.0);
    for (int k = 0; k < R; ++k) Mx[(size_t)k * R + k] = 1.0;
    for (int s = 0; s < S; ++s) {
        const int bs = sb[s], es = se[s];
        const int pv = s > 0 ? s - 1 : (periodic ? S - 1 : -1);
        const int nx = s < S - 1 ? s + 1 : (periodic ? 0 : -1);
        if (pv >= 0) {
            Mx[(size_t)s * R + S + pv] += vv[bs];
            Mx[(size_t)(S + s) * R + S + pv] += vv[es - 1];
        }
        if (nx >= 0) {
            Mx[(size_t)s * R + nx] += ww[bs];
            Mx[(size_t)(S + s) * R + nx] += ww[es - 1];
        }
    }
    // Gauss-Jordan with partial pivoting
    for (int k = 0; k < R; ++k) Inv[(size_t)k * R + k] = 1.0;
    for (int col = 0; col < R; ++col) {
        int piv = col;
        for (int r = col + 1; r < R; ++r)
            if (std::fabs(Mx[(size_t)r * R + col]) > std::fabs(Mx[(size_t)piv * R + col])) piv = r;
        if (Mx[(size_t)piv * R + col] == 0.0) return -1;
        if (piv != col)
            for (int k = 0; k < R; ++k) {
                std::swap(Mx[(size_t)piv * R + k], Mx[(size_t)col * R + k]);
                std::swap(Inv[(size_t)piv * R + k], Inv[(size_t)col * R + k]);
            }
        const double d = 1.0 / Mx[(size_t)col * R + col];
        for (int k = 0; k < R; ++k) {
            Mx[(size_t)col * R + k] *= d;
            Inv[(size_t)col * R + k] *= d;
        }
        for (int r = 0; r < R; ++r) {
            if (r == col) continue;
            const double f = Mx[(size_t)r * R + col];
            if (f == 0.0) continue;
            for (int k = 0; k < R; ++k) {
                Mx[(size_t)r * R + k] -= f * Mx[(size_t)col * R + k];
                Inv[(size_t)r * R + k] -= f * Inv[(size_t)col * R + k];
            }
        }
    }
    for (int s = 0; s < S; ++s) {
        const int pv = s > 0 ? s - 1 : (periodic ? S - 1 : -1);
        const int nx = s < S - 1 ? s + 1 : (periodic ? 0 : -1);
        double *rs = red + (size_t)s * 4 * S;
        for (int k = 0; k < S; ++k) {
            rs[k] = pv >= 0 ? Inv[(size_t)(S + pv) * R + k] : 0.0;
            rs[S + k] = pv >= 0 ? Inv[(size_t)(S + pv) * R + S + k] : 0.0;
            rs[2 * S + k] = nx >= 0 ? Inv[(size_t)nx * R + k] : 0.0;
            rs[3 * S + k] = nx >= 0 ? Inv[(size_t)nx * R + S + k] : 0.0;
        }
    }
    return 0;
}

const SegOpDev *ctx_segop(wd_ctx *ctx, int kind, int n, int periodic, int scheme, double af,
                          int fp64, const SegGeo &sg, TableArena *ar)
{
    OpKey key{kind + 2 + 4 * (sg.M + 64 * sg.S), n, periodic, kind == OP_FILTER ? -1 : scheme,
              fp64, kind == OP_FILTER ? af : 0.0};
    if (ar) {
        for (auto &kv : ar->segops)
            if (!(kv.first < key) && !(key < kv.first)) return &kv.second.dev;
    } else {
        auto it = ctx->segops.find(key);
        if (it != ctx->segops.end()) return &it->second.dev;
    }
    SegEntry e;
    e.dev.n = n;
    e.dev.S = sg.S;
    e.dev.periodic = periodic;
    e.dev.solve = kind == OP_FILTER || scheme == SCHEME_C4 || scheme == SCHEME_C6;
    e.dev.tab = nullptr;
    if (e.dev.solve) {
        std::vector<double> t;
        if (build_seg_tables(kind, n, periodic, scheme, af, sg, t)) {
            fail(WD_ERR_UNSUPPORTED, "segmented line system (n=%d, S=%d) is singular", n, sg.S);
            return nullptr;
        }
        // device layout: each row array n + S long with position j at
        // j + (segment of j), and the reduced rows S (4S + 1) apart, so the
        // lanes of one step (segments M apart) read distinct LDS banks
        const int n2 = n + sg.S, rs = 4 * sg.S + 1;
        std::vector<double> d((size_t)5 * n2 + (size_t)sg.S * rs, 0.0);
        for (int s = 0; s < sg.S; ++s) {
            int bs, len;
            seg_bounds(sg, s, bs, len);
            for (int a = 0; a < 5; ++a)
                for (int j = bs; j < bs + len; ++j)
                    d[(size_t)a * n2 + j + s] = t[(size_t)a * n + j];
            for (int k = 0; k < 4 * sg.S; ++k)
                d[(size_t)5 * n2 + (size_t)s * rs + k] = t[(size_t)5 * n + (size_t)s * 4 * sg.S + k];
        }
        const size_t es = fp64 ? 8 : 4;
        std::vector<unsigned char> host(d.size() * es);
        for (size_t i = 0; i < d.size(); ++i) {
            if (fp64) reinterpret_cast<double *>(host.data())[i] = d[i];
            else reinterpret_cast<float *>(host.data())[i] = (float)d[i];
        }
        void *mem = nullptr;
        if (ar) {
            mem = ar->carve(host.size());
            if (!mem) {
                fail(WD_ERR_NO_MEMORY, "line-operator tables exceed the %zu-byte scratch", ar->cap);
                return nullptr;
            }
            const size_t bytes = host.size();
            ar->host.push_back(std::move(host));
            if (hipMemcpyAsync(mem, ar->host.back().data(), bytes, hipMemcpyHostToDevice,
                               ar->stream) != hipSuccess) {
                fail(WD_ERR_HIP, "upload of a line operator failed");
                return nullptr;
            }
        } else {
            if (hipMalloc(&mem, host.size()) != hipSuccess) {
                fail(WD_ERR_NO_MEMORY, "hipMalloc of %zu bytes for a line operator failed",
                     host.size());
                return nullptr;
            }
            if (hipMemcpy(mem, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
                (void)hipFree(mem);
                fail(WD_ERR_HIP, "upload of a line operator failed");
                return nullptr;
            }
            e.mem = mem;
        }
        e.dev.tab = mem;
    }
    if (ar) {
        ar->segops.emplace_back(key, e);
        return &ar->segops.back().second.dev;
    }
    auto ins = ctx->segops.emplace(key, e);
    return &ins.first->second.dev;
}

// dynamic LDS bytes of a segmented pass (kind: PASS_SCART / SFILTER / SLAD)
size_t seg_lds_bytes(const GridDev &g, int kind, int l, int fp64)
{
    const SegGeo &sg = g.sgeo[l];
    const SegOpDev &op = kind == PASS_SFILTER ? g.sfop[l] : g.sdop[l];
    size_t el = (size_t)sg.xsize;
    if (kind != PASS_SLAD && op.solve) el += seg_table_len(op.n, op.S);
    return el * (fp64 ? 8 : 4);
}

// ---------------------------------------------------------------------
// validation
int check_desc(const wd_grid_desc *d)
{
    if (!d) return fail(WD_ERR_INVALID_ARG, "null grid descriptor");
    if (d->ndim != 2 && d->ndim != 3) return fail(WD_ERR_INVALID_ARG, "ndim must be 2 or 3");
    long long N = 1;
    for (int l = 0; l < d->ndim; ++l) {
        if (d->n[l] < 8) return fail(WD_ERR_INVALID_ARG, "n[%d] = %d < 8", l, d->n[l]);
        if (d->n[l] > kMaxLine)
            return fail(WD_ERR_UNSUPPORTED, "n[%d] = %d exceeds the line limit %d", l, d->n[l], kMaxLine);
        for (int s = 0; s < 2; ++s)
            if (d->bc[l][s] < WD_BC_WALL || d->bc[l][s] > WD_BC_PERIODIC)
                return fail(WD_ERR_INVALID_ARG, "bad face code on direction %d", l);
        if ((d->bc[l][0] == WD_BC_PERIODIC) != (d->bc[l][1] == WD_BC_PERIODIC))
            return fail(WD_ERR_INVALID_ARG, "PERIODIC must be set on both faces of direction %d", l);
        N *= d->n[l];
    }
    if (d->ndim == 2 && d->n[2] != 1) return fail(WD_ERR_INVALID_ARG, "2D grids need n[2] == 1");
    if (N >= (1LL << 31)) return fail(WD_ERR_UNSUPPORTED, "grid of %lld points is too large", N);
    if (d->metric_mode == WD_METRIC_UNIFORM) {
        for (int l = 0; l < d->ndim; ++l)
            if (!(d->h[l] > 0.0)) return fail(WD_ERR_INVALID_ARG, "h[%d] must be > 0", l);
    } else if (d->metric_mode == WD_METRIC_FIELDS) {
        if (!d->metrics) return fail(WD_ERR_INVALID_ARG, "metric fields pointer is null");
    } else {
        return fail(WD_ERR_INVALID_ARG, "bad metric mode");
    }
    return WD_OK;
}

// A solve needs something to measure the distance from: a wall face or a
// solid mask (the caller's mask may still hold no solid point).
int check_walls(const wd_grid_desc *d)
{
    if (d->mask) return WD_OK;
    for (int l = 0; l < d->ndim; ++l)
        for (int s = 0; s < 2; ++s)
            if (d->bc[l][s] == WD_BC_WALL) return WD_OK;
    return fail(WD_ERR_INVALID_ARG, "no wall face and no solid mask: the distance is undefined");
}

int check_method(const wd_method *m)
{
    if (!m) return fail(WD_ERR_INVALID_ARG, "null method");
    if (m->equation < WD_EQ_EIKONAL || m->equation > WD_EQ_POISSON) return fail(WD_ERR_INVALID_ARG, "bad equation");
    if (m->gamma != WD_GAMMA_LINEAR && m->gamma != WD_GAMMA_LAD) return fail(WD_ERR_INVALID_ARG, "bad gamma");
    if (m->scheme < WD_E2 || m->scheme > WD_UW) return fail(WD_ERR_INVALID_ARG, "bad scheme");
    if (m->scheme == WD_UW && m->equation == WD_EQ_HJ && m->curvature)
        return fail(WD_ERR_UNSUPPORTED, "the upwind baseline has no curvature correction");
    if (m->rk != WD_RK3_SSP && m->rk != WD_RK4) return fail(WD_ERR_INVALID_ARG, "bad rk");
    if (m->precision != WD_FP32 && m->precision != WD_FP64) return fail(WD_ERR_INVALID_ARG, "bad precision");
    if (m->filter && !(m->alpha_f >= 0.0 && m->alpha_f < 0.5))
        return fail(WD_ERR_INVALID_ARG, "alpha_f must be in [0, 0.5) when the filter is on");
    if (!(m->sigma > 0.0)) return fail(WD_ERR_INVALID_ARG, "sigma must be > 0");
    if (m->max_iter < 1) return fail(WD_ERR_INVALID_ARG, "max_iter must be >= 1");
    if (m->warm_probe < 0) return fail(WD_ERR_INVALID_ARG, "warm_probe must be >= 0");
    if (!(m->tol >= 0.0)) return fail(WD_ERR_INVALID_ARG, "tol must be >= 0");
    if (m->stall_window < 0) return fail(WD_ERR_INVALID_ARG, "stall_window must be >= 0");
    if (m->equation == WD_EQ_HJ && m->curvature && !(m->eps0 > 0.0))
        return fail(WD_ERR_INVALID_ARG, "eps0 must be > 0");
    return WD_OK;
}

static long long npoints(const wd_grid_desc &d)
{
    long long N = 1;
    for (int l = 0; l < d.ndim; ++l) N *= d.n[l];
    return N;
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

int grid_mode(const wd_grid_desc &d, const wd_method &m)
{
    const bool curv = m.equation == WD_EQ_HJ && m.curvature;
    const bool uw = m.scheme == WD_UW && m.equation != WD_EQ_POISSON;
    return (d.metric_mode == WD_METRIC_UNIFORM && !curv && !uw) ? MODE_CART : MODE_GENERAL;
}

int hist_dev_cap(const wd_method &m) { return std::min(m.max_iter, 1 << 17); }

// device bytes of one grid's own region: its fields, partial sums,
// residual partials, history and stopping state
size_t grid_region_bytes(const wd_grid_desc &d, const wd_method &m)
{
    const long long N = npoints(d);
    const size_t S = m.precision == WD_FP64 ? 8 : 4;
    const size_t f = al256((size_t)N * S);
    size_t b = 0;
    b += f;                                      // ps
    if (m.rk == WD_RK4) b += f;                  // acc
    b += f;                                      // dt
    if (d.metric_mode == WD_METRIC_FIELDS)
        b += (size_t)d.ndim * d.ndim * f;        // point-major metrics
    if (grid_mode(d, m) == MODE_GENERAL) b += (size_t)d.ndim * f;  // F_l
    b += 3 * f;                                  // partial sums / LAD field
    if (m.scheme == WD_UW && m.equation != WD_EQ_POISSON) b += f;   // upwind |U|^2
    if (m.equation == WD_EQ_POISSON)
        b += (size_t)(d.ndim + 1) * al256((size_t)N * 8);  // FP64 conversion
    long long parts = N / d.n[d.ndim - 1];
    parts = std::max(parts, (N + kChunk - 1) / kChunk);
    b += al256((size_t)parts * 32);
    b += al256((size_t)hist_dev_cap(m) * 16);
    b += al256(sizeof(GridState));
    return b;
}

// worst-case work items of one grid (tile width 1), plus room for the
// one-grid FP64 Poisson passes
long long grid_items(const wd_grid_desc &d)
{
    const long long N = npoints(d);
    long long lines = 0;
    for (int l = 0; l < d.ndim; ++l) lines += N / d.n[l];
    const long long chunks = (N + kChunk - 1) / kChunk;
    long long face = 0;
    for (int l = 0; l < d.ndim; ++l) face += 2 * ((N / d.n[l] + kChunk - 1) / kChunk);
    return 5 * lines + 5 * chunks + 2 * face + 8;
}

// batch tables: grid array, state mirrors, two one-grid views, items
size_t table_bytes(int n, long long items)
{
    return al256((size_t)n * sizeof(GridDev)) + 2 * al256(sizeof(GridDev)) +
           al256((size_t)(n + 1) * sizeof(GridState)) + al256((size_t)items * sizeof(Item)) + 1024;
}

size_t batch_bytes(int n, const wd_grid_desc *d, const wd_method *m)
{
    long long items = 0;
    size_t b = 0;
    for (int i = 0; i < n; ++i) {
        b += grid_region_bytes(d[i], m[i]);
        items += grid_items(d[i]);
    }
    return b + table_bytes(n, items);
}

// ---------------------------------------------------------------------
// tile widths
int pick_tile(wd_ctx *ctx, const wd_grid_desc &d, int l, int fp64)
{
    TuneKey key{d.ndim, d.n[0], d.n[1], d.n[2], l, fp64};
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) return it->second;
    const long long N = npoints(d);
    const int n = d.n[l];
    const long long target = 2LL * ctx->cus;
    int w;
    if (l == 0) {
        const long long lines = N / n;
        w = std::max(1, kTileMax / n);
        while (w > 1 && (lines + w - 1) / w < target) w /= 2;
    } else {
        int wmax = std::max(1, std::min(64, kTileMax / n));
        w = 1;
        while (w * 2 <= wmax) w *= 2;
        const long long planes = N / ((long long)d.n[0] * n);
        while (w > 4 && planes * ((d.n[0] + w - 1) / w) < target) w /= 2;
    }
    return w;
}

static double kprime(int scheme)
{
    switch (scheme) {
    case WD_UW: return 2.0;    // |1 - e^{-iw}| <= 2 of the one-sided differences
    case WD_E2: return 1.0;
    case WD_E4: return 1.372;
    case WD_E6: return 1.586;
    case WD_C4: return 1.732;
    default: return 1.989;
    }
}

// ---------------------------------------------------------------------
// planning
// Describe one grid in `g`, its buffers carved from `region` (at least
// grid_region_bytes).  The stopping state lives in the region, so a grid
// keeps its progress when the batch around it changes.
int layout_grid(wd_ctx *ctx, const wd_grid_desc &d, const wd_method &m, void *phi,
                void *region, GridDev &g, GridHost &h, TableArena *ar)
{
    std::memset(&g, 0, sizeof g);
    h = GridHost();
    const int fp64 = m.precision == WD_FP64;
    const long long N = npoints(d);
    unsigned char *base = static_cast<unsigned char *>(region);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void *p = base + off;
        off += al256(bytes);
        return p;
    };
    g.ndim = d.ndim;
    g.mode = grid_mode(d, m);
    g.N = N;
    long long st = 1;
    for (int l = 0; l < 3; ++l) {
        g.n[l] = l < d.ndim ? d.n[l] : 1;
        g.stride[l] = st;
        st *= g.n[l];
    }
    for (int l = 0; l < d.ndim; ++l) {
        g.periodic[l] = d.bc[l][0] == WD_BC_PERIODIC;
        g.wall_lo[l] = d.bc[l][0] == WD_BC_WALL;
        g.wall_hi[l] = d.bc[l][1] == WD_BC_WALL;
        for (int s = 0; s < 2; ++s) {
            const int b = d.bc[l][s];
            g.xbc[2 * l + s] = b == WD_BC_NEUMANN ? XBC_NEUMANN : b == WD_BC_OUTFLOW ? XBC_OUTFLOW : XBC_NONE;
        }
    }
    g.uniform = d.metric_mode == WD_METRIC_UNIFORM;
    for (int l = 0; l < 3; ++l) g.invh[l] = (g.uniform && l < d.ndim) ? 1.0 / d.h[l] : 0.0;
    g.met_src = d.metrics;
    g.mask = d.mask;
    g.eq = m.equation;
    g.lad = m.equation == WD_EQ_HJ && m.gamma == WD_GAMMA_LAD;
    g.curv = m.equation == WD_EQ_HJ && m.curvature;
    // the upwind baseline evaluates its advective term pointwise and all its
    // central derivatives (Laplacian, Poisson) with E2
    g.uw = m.scheme == WD_UW && m.equation != WD_EQ_POISSON;
    const int dscheme = m.scheme == WD_UW ? WD_E2 : m.scheme;
    g.scheme = dscheme;
    g.rk = m.rk == WD_RK4;
    g.stages = g.rk ? 4 : 3;
    g.need_lap = m.equation != WD_EQ_EIKONAL;
    g.filter = m.filter;
    bool has_x = false, only_last = true;
    for (int f = 0; f < 6; ++f)
        if (g.xbc[f] != XBC_NONE) {
            has_x = true;
            only_last &= (f >> 1) == d.ndim - 1;
        }
    // faces normal to the last direction are applied inside its passes
    // (that direction's tiles hold whole lines); otherwise face kernels
    g.fuse_faces = has_x && only_last && !(g.mode == MODE_GENERAL && !g.need_lap);
    g.fused_resid = m.filter && (!has_x || g.fuse_faces);
    // a general grid's finishing pass holds whole lines of the new stage
    // value (no face pass after it) and forms the next stage's F there
    g.fnext = g.mode == MODE_GENERAL && g.need_lap && (!has_x || g.fuse_faces);
    g.eps = m.eps;
    g.C = m.c_lad;
    g.nu0 = m.nu0;
    g.eps0 = m.eps0;
    g.sigma = m.sigma;
    g.kp = kprime(g.uw ? WD_UW : dscheme);   // advective term
    g.kp2 = kprime(dscheme);                  // diffusive term
    g.tol = m.tol;
    g.max_iter = m.max_iter;
    g.stall = m.stall_window;
    g.warm = m.warm_start;
    g.warm_probe = m.warm_start ? std::max(0, m.warm_probe) : 0;
    // filter correction factor -(1 - 2 af)(-1)^N / 4^N
    for (int N5 = 1; N5 <= 5; ++N5)
        g.fcoef[N5] = -(1.0 - 2.0 * m.alpha_f) * ((N5 & 1) ? -1.0 : 1.0) / std::ldexp(1.0, 2 * N5);
    switch (dscheme) {
    case WD_E2: g.da = 1.0; g.dradius = 1; break;
    case WD_E4: g.da = 4.0 / 3.0; g.db = -1.0 / 3.0; g.dradius = 2; break;
    case WD_E6: g.da = 1.5; g.db = -0.6; g.dc = 0.1; g.dradius = 3; break;
    case WD_C4: g.da = 1.5; g.dradius = 1; g.compact = 1; break;
    default: g.da = 14.0 / 9.0; g.db = 1.0 / 9.0; g.dradius = 2; g.compact = 1; break;
    }
    // uniform Cartesian grid, explicit central scheme, no extrapolated
    // face: each RK stage in one pointwise pass (lines of at least 4R + 2
    // points, so that the two ends' closure rows never meet in a stencil)
    g.xstage = ctx->use_xstage && g.mode == MODE_CART && !g.compact && !g.uw && !has_x;
    for (int l = 0; l < d.ndim; ++l)
        if (d.n[l] < 4 * g.dradius + 2) g.xstage = 0;
    if ((double)N * (fp64 ? 8 : 4) >= 2147483648.0) g.xstage = 0;   // 32-bit buffer offsets
    if (g.xstage) {
        // x-y tiles of kXTX x kXTY points, fast (interior) and general ones;
        // each kind's z march cut into chunks of at least 8 planes, as many
        // as fit its kernel's resident workgroups in one round
        const int ntx = (d.n[0] + kXTX - 1) / kXTX, nty = (d.n[1] + kXTY - 1) / kXTY;
        const int n2 = d.ndim == 3 ? d.n[2] : 1;
        int nf = 0;
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx)
                nf += xtile_fast(xtile_origin(tx, kXTX, d.n[0]), xtile_origin(ty, kXTY, d.n[1]),
                                 d.n[0], d.n[1], g.periodic[0] != 0, g.periodic[1] != 0,
                                 g.dradius);
        const int ng = ntx * nty - nf;
        auto chunk = [&](int tiles, int fast) {
            if (tiles == 0) return n2;
            const int slots = ctx->cus * xstage_blocks_per_cu(fp64, g.dradius, fast);
            const int nzc = std::max(1, std::min(slots / tiles, n2 / 8));
            return (n2 + nzc - 1) / nzc;
        };
        g.xkz = chunk(nf, 1);
        g.xkz2 = chunk(ng, 0);
    }
    // LAD field of a uniform Cartesian grid: two passes over x-y tiles (the
    // fourth difference needs 5 points per line), z chunks of at least 8
    // planes as many as fill one round of the smoothing pass's workgroups
    g.xlad = ctx->use_xlad && g.lad && g.mode == MODE_CART &&
             (double)N * (fp64 ? 8 : 4) < 2147483648.0;
    for (int l = 0; l < d.ndim; ++l)
        if (d.n[l] < 5) g.xlad = 0;
    if (g.xlad) {
        const int ntx = (d.n[0] + kXTX - 1) / kXTX, nty = (d.n[1] + kXTY - 1) / kXTY;
        const int n2 = d.ndim == 3 ? d.n[2] : 1;
        const int slots = ctx->cus * xlad_blocks_per_cu(fp64, 2);
        const int nzc = std::max(1, std::min(slots / (ntx * nty), n2 / 8));
        g.xlkz = (n2 + nzc - 1) / nzc;
    }
    const size_t f = (size_t)N * (fp64 ? 8 : 4);
    g.phi = phi;
    g.ps = take(f);
    g.acc = m.rk == WD_RK4 ? take(f) : nullptr;
    g.dt = take(f);
    if (!g.uniform) g.met = take((size_t)d.ndim * d.ndim * f);
    if (g.mode == MODE_GENERAL)
        for (int l = 0; l < d.ndim; ++l) g.F[l] = take(f);
    for (int k = 0; k < 3; ++k) g.P[k] = take(f);
    if (g.uw) g.uw2 = take(f);
    if (m.equation == WD_EQ_POISSON) {
        h.pois_phip = take((size_t)N * 8);
        for (int l = 0; l < d.ndim; ++l) h.pois_F[l] = take((size_t)N * 8);
    }
    long long parts = N / d.n[d.ndim - 1];
    parts = std::max(parts, (N + kChunk - 1) / kChunk);
    g.rpart = static_cast<double *>(take((size_t)parts * 32));
    g.hist_cap = hist_dev_cap(m);
    g.hist = static_cast<double *>(take((size_t)g.hist_cap * 16));
    g.state = static_cast<GridState *>(take(sizeof(GridState)));
    // segmented passes: uniform Cartesian grids whose lines all have >= 16
    // points and whose tiles fit the LDS budget
    g.seg = 0;
    if (ctx->use_seg && g.mode == MODE_CART) {
        bool ok = true;
        for (int l = 0; l < d.ndim; ++l) ok &= d.n[l] >= 16;
        for (int l = 0; l < d.ndim && ok; ++l) {
            if (!seg_plan(d.n[l], fp64, g.sgeo[l], ctx->use_seg)) {
                ok = false;
                break;
            }
            const SegOpDev *sd = ctx_segop(ctx, OP_DERIV, d.n[l], g.periodic[l], dscheme, 0.0, fp64,
                                           g.sgeo[l], ar);
            if (!sd) return WD_ERR_NO_MEMORY;
            g.sdop[l] = *sd;
            if (m.filter) {
                const SegOpDev *sf = ctx_segop(ctx, OP_FILTER, d.n[l], g.periodic[l], dscheme,
                                               m.alpha_f, fp64, g.sgeo[l], ar);
                if (!sf) return WD_ERR_NO_MEMORY;
                g.sfop[l] = *sf;
            }
            for (int kind : {PASS_SCART, PASS_SCART_LAST, PASS_SFILTER, PASS_SLAD})
                ok &= seg_lds_bytes(g, kind, l, fp64) <= (size_t)65536;
        }
        g.seg = ok ? 1 : 0;
        // grids without extrapolated faces: the last direction carries the
        // sums on and a pointwise pass finishes the stage (coalesced: on the
        // 256^3 duct 111 us against 320 us when each lane of the z pass
        // finishes its own strided points); otherwise the last direction's
        // pass finishes the stage and sets the faces normal to it (and for
        // fields of 2^31 bytes or more, which the pointwise pass's 32-bit
        // buffer offsets do not reach)
        g.seg_split = g.seg && !has_x && ctx->seg_split_finish &&
                      (double)N * (fp64 ? 8 : 4) < 2147483648.0;
    }
    for (int l = 0; l < d.ndim; ++l) {
        const LineOpDev *dop = ctx_lineop(ctx, OP_DERIV, d.n[l], g.periodic[l], dscheme, 0.0, fp64, ar);
        if (!dop) return WD_ERR_NO_MEMORY;
        g.dop[l] = *dop;
        if (m.filter) {
            const LineOpDev *fop = ctx_lineop(ctx, OP_FILTER, d.n[l], g.periodic[l], dscheme, m.alpha_f, fp64, ar);
            if (!fop) return WD_ERR_NO_MEMORY;
            g.fop[l] = *fop;
        }
        g.tw[l] = g.seg ? g.sgeo[l].W : pick_tile(ctx, d, l, fp64);
        if (l == 0)
            g.ntiles[l] = (int)((N / d.n[0] + g.tw[0] - 1) / g.tw[0]);
        else
            g.ntiles[l] = (int)((N / ((long long)d.n[0] * d.n[l])) * ((d.n[0] + g.tw[l] - 1) / g.tw[l]));
    }
    g.nchunks = (int)((N + kChunk - 1) / kChunk);
    g.nparts = g.fused_resid ? g.ntiles[d.ndim - 1] : g.nchunks;
    if (off > grid_region_bytes(d, m)) return fail(WD_ERR_INVALID_ARG, "internal: grid layout overflow");
    return WD_OK;
}

// Batch tables in `tables` (table_bytes of the grids' worst-case items);
// P.grids / P.host must be filled.  Sets mirrors and builds the work lists.
int plan_tables(Plan &P, void *tables, size_t bytes, long long items_cap)
{
    const int n = (int)P.grids.size();
    P.n = n;
    if (bytes < table_bytes(n, items_cap)) return fail(WD_ERR_NO_MEMORY, "table space too small");
    unsigned char *base = static_cast<unsigned char *>(tables);
    size_t off = 0;
    auto take = [&](size_t b) {
        void *p = base + off;
        off += al256(b);
        return p;
    };
    P.d_grids = static_cast<GridDev *>(take((size_t)n * sizeof(GridDev)));
    P.d_aux = static_cast<GridDev *>(take(sizeof(GridDev)));
    P.d_aux2 = static_cast<GridDev *>(take(sizeof(GridDev)));
    P.d_states = static_cast<GridState *>(take((size_t)(n + 1) * sizeof(GridState)));
    P.d_items = static_cast<Item *>(take((size_t)items_cap * sizeof(Item)));
    P.maxdim = 0;
    for (int i = 0; i < n; ++i) {
        P.grids[i].mirror = P.d_states + i;
        P.maxdim = std::max(P.maxdim, P.grids[i].ndim);
    }
    build_items(P);
    if ((long long)P.items.size() > items_cap) return fail(WD_ERR_INVALID_ARG, "internal: item overflow");
    P.items_cap = items_cap;
    return WD_OK;
}

// one workspace: tables first, then each grid's region
int plan_batch(wd_ctx *ctx, int n, const wd_grid_desc *descs, const wd_method *meths,
               void *const *phis, void *ws, size_t ws_bytes, Plan &P, TableArena *ar)
{
    P = Plan();
    P.arena = ar;
    P.fp64 = meths[0].precision == WD_FP64;
    P.rk = meths[0].rk;
    P.stages = P.rk == WD_RK4 ? 4 : 3;
    const size_t need = batch_bytes(n, descs, meths);
    if (!ws || ws_bytes < need)
        return fail(WD_ERR_NO_MEMORY, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
    long long items_cap = 0;
    for (int i = 0; i < n; ++i) items_cap += grid_items(descs[i]);
    const size_t tb = table_bytes(n, items_cap);
    unsigned char *base = static_cast<unsigned char *>(ws);
    size_t off = tb;
    P.grids.resize(n);
    P.host.resize(n);
    for (int i = 0; i < n; ++i) {
        int rc = layout_grid(ctx, descs[i], meths[i], phis ? phis[i] : nullptr, base + off,
                             P.grids[i], P.host[i], ar);
        if (rc) return rc;
        off += grid_region_bytes(descs[i], meths[i]);
    }
    return plan_tables(P, ws, tb, items_cap);
}

// points-per-thread variant of grid g's tiles along direction l
int tile_np(const GridDev &g, int l)
{
    const long long pts = (long long)g.tw[l] * g.n[l];
    int np = 1;
    while (np < 8 && (long long)kThreads * np < pts) np *= 2;
    return np;
}

// work lists in launch order; a line pass gets one list per tile variant
// present among its grids
void build_items(Plan &P)
{
    P.items.clear();
    P.lists.clear();
    const int n = P.n;
    auto live = [&](int i) { return P.live.empty() || P.live[i] != 0; };
    auto add_list = [&](int kind, int l, int arg, int np) {
        ItemList L;
        L.kind = kind;
        L.l = l;
        L.arg = arg;
        L.np = np;
        L.first = (int)P.items.size();
        L.count = 0;
        P.lists.push_back(L);
        return (int)P.lists.size() - 1;
    };
    // one line pass: tiles of the grids selected by `use`, grouped by variant
    auto line_slot = [&](Slot &S, int kind, int l, int arg, auto use) {
        for (int c = 0; c < 4; ++c) {
            S.list[c] = -1;
            const int np = 1 << c;
            int li = -1;
            for (int i = 0; i < n; ++i) {
                if (!live(i)) continue;
                const GridDev &g = P.grids[i];
                if (l >= g.ndim || !use(g) || tile_np(g, l) != np) continue;
                if (li < 0) li = add_list(kind, l, arg, np);
                for (int t = 0; t < g.ntiles[l]; ++t) P.items.push_back(Item{i, t});
                P.lists[li].count += g.ntiles[l];
            }
            S.list[c] = li;
        }
    };
    auto point_list = [&](int kind, int l, int arg, auto count) {
        const int li = add_list(kind, l, arg, 1);
        for (int i = 0; i < n; ++i) {
            if (!live(i)) continue;
            const int nt = count(i);
            for (int t = 0; t < nt; ++t) P.items.push_back(Item{i, t});
            P.lists[li].count += nt;
        }
        return li;
    };
    auto cart = [](const GridDev &g) { return g.mode == MODE_CART && !g.seg && !g.xstage; };
    // segmented pass: one list of the tiles of every segmented grid
    // segmented pass: one list per segment length M (16, 24, 32) present
    // among the segmented grids (the list's np field holds M)
    auto seg_list = [&](Slot &Sl, int kind, int l, int arg, auto use) {
        const int Ms[3] = {16, 24, 32};
        for (int c = 0; c < 4; ++c) Sl.list[c] = -1;
        for (int c = 0; c < 3; ++c) {
            int li = -1;
            for (int i = 0; i < n; ++i) {
                if (!live(i)) continue;
                const GridDev &g = P.grids[i];
                if (!g.seg || l >= g.ndim || !use(g) || g.sgeo[l].M != Ms[c]) continue;
                if (li < 0) li = add_list(kind, l, arg, Ms[c]);
                for (int t = 0; t < g.ntiles[l]; ++t) P.items.push_back(Item{i, t});
                P.lists[li].count += g.ntiles[l];
            }
            Sl.list[c] = li;
        }
    };
    for (int l = 0; l < 3; ++l)
        seg_list(P.scart[l], PASS_SCART, l, 0, [l](const GridDev &g) {
            return !g.xstage && (l < g.ndim - 1 || g.seg_split);
        });
    for (int l = 0; l < 3; ++l)
        seg_list(P.scartl[l], PASS_SCART_LAST, l, 0, [l](const GridDev &g) {
            return !g.xstage && l == g.ndim - 1 && !g.seg_split;
        });
    P.cfin = point_list(PASS_CFIN, 0, 0, [&](int i) {
        return P.grids[i].seg_split && !P.grids[i].xstage ? P.grids[i].nchunks : 0;
    });
    // one-pass explicit stages: per scheme radius (the list's l) one list of
    // general tiles (np 1) and one of fast tiles (np 2), each item a tile
    // and a chunk of its z march
    for (int r = 1; r <= 3; ++r)
        for (int fast = 0; fast < 2; ++fast) {
            const int li = add_list(PASS_XSTAGE, r, 0, 1 + fast);
            for (int i = 0; i < n; ++i) {
                if (!live(i)) continue;
                const GridDev &g = P.grids[i];
                if (!g.xstage || g.dradius != r) continue;
                const int ntx = (g.n[0] + kXTX - 1) / kXTX, nty = (g.n[1] + kXTY - 1) / kXTY;
                const int n2 = g.ndim == 3 ? g.n[2] : 1;
                const int kz = fast ? g.xkz : g.xkz2;
                const int nzc = (n2 + kz - 1) / kz;
                for (int zc = 0; zc < nzc; ++zc)
                    for (int ty = 0; ty < nty; ++ty)
                        for (int tx = 0; tx < ntx; ++tx) {
                            const bool f = xtile_fast(xtile_origin(tx, kXTX, g.n[0]),
                                                      xtile_origin(ty, kXTY, g.n[1]), g.n[0],
                                                      g.n[1], g.periodic[0] != 0,
                                                      g.periodic[1] != 0, r);
                            if (f != (fast != 0)) continue;
                            P.items.push_back(Item{i, (zc * nty + ty) * ntx + tx});
                            ++P.lists[li].count;
                        }
            }
            P.xstage[r - 1][fast] = li;
        }
    // two-pass LAD field: items are x-y tiles times z chunks, the same for
    // the sensor (np 1) and the smoothing (np 2)
    for (int ph = 0; ph < 2; ++ph) {
        const int li = add_list(PASS_XLAD, 0, 0, 1 + ph);
        for (int i = 0; i < n; ++i) {
            if (!live(i)) continue;
            const GridDev &g = P.grids[i];
            if (!g.xlad) continue;
            const int ntx = (g.n[0] + kXTX - 1) / kXTX, nty = (g.n[1] + kXTY - 1) / kXTY;
            const int n2 = g.ndim == 3 ? g.n[2] : 1;
            const int nt = ntx * nty * ((n2 + g.xlkz - 1) / g.xlkz);
            for (int t = 0; t < nt; ++t) P.items.push_back(Item{i, t});
            P.lists[li].count += nt;
        }
        P.xlad[ph] = li;
    }
    for (int l = 0; l < 3; ++l)
        seg_list(P.slad0[l], PASS_SLAD, l, 0, [](const GridDev &g) {
            return g.lad != 0 && !g.xlad;
        });
    for (int l = 0; l < 3; ++l)
        seg_list(P.slad1[l], PASS_SLAD, l, 1, [l](const GridDev &g) {
            return g.lad != 0 && !g.xlad && l < g.ndim - 1;
        });
    for (int l = 0; l < 3; ++l)
        seg_list(P.sfilt[l], PASS_SFILTER, l, 0, [](const GridDev &g) { return g.filter != 0; });
    auto gen_lap = [](const GridDev &g) { return g.mode == MODE_GENERAL && g.need_lap; };
    auto gen_eik = [](const GridDev &g) { return g.mode == MODE_GENERAL && !g.need_lap; };
    // first-derivative fields: every general grid but the upwind Eikonal
    // (its stage finish takes one-sided differences of phi itself)
    auto gen_f = [](const GridDev &g) { return g.mode == MODE_GENERAL && (g.need_lap || !g.uw); };
    auto gen_eik_f = [](const GridDev &g) { return g.mode == MODE_GENERAL && !g.need_lap && !g.uw; };
    for (int l = 0; l < 3; ++l) line_slot(P.cart[l], PASS_CART, l, 0, cart);
    // general grids: F_l for l >= 1 first (all l for the Eikonal), then the
    // fused pass along 0, then pass 2 along l >= 1 (the last one finishes)
    line_slot(P.d1[0], PASS_D1, 0, 0, gen_eik_f);
    for (int l = 1; l < 3; ++l) line_slot(P.d1[l], PASS_D1, l, 0, gen_f);
    // stages > 0: the finishing pass of the previous stage formed F_{d-1}
    line_slot(P.d1n[0], PASS_D1, 0, 0, gen_eik_f);
    for (int l = 1; l < 3; ++l)
        line_slot(P.d1n[l], PASS_D1, l, 0, [&gen_f, l](const GridDev &g) {
            return gen_f(g) && !(g.fnext && l == g.ndim - 1);
        });
    line_slot(P.d12, PASS_D12, 0, 0, gen_lap);
    P.d2[0] = Slot();
    for (int l = 1; l < 3; ++l) line_slot(P.d2[l], PASS_D2, l, 0, gen_lap);
    P.uwadv = point_list(PASS_UWADV, 0, 0, [&](int i) {
        return (gen_eik(P.grids[i]) && P.grids[i].uw) ? P.grids[i].nchunks : 0;
    });
    P.fin = point_list(PASS_FINAL, 0, 0, [&](int i) {
        return gen_eik(P.grids[i]) ? P.grids[i].nchunks : 0;
    });
    // LAD on Cartesian grids: sensor per direction (the last also smooths
    // along itself), then smoothing along the other directions.  General
    // grids form the field inside their stage-0 passes.
    for (int l = 0; l < 3; ++l)
        line_slot(P.lad0[l], PASS_LAD, l, 0, [](const GridDev &g) {
            return g.lad != 0 && g.mode == MODE_CART && !g.seg && !g.xlad;
        });
    for (int l = 0; l < 3; ++l)
        line_slot(P.lad1[l], PASS_LAD, l, 1, [l](const GridDev &g) {
            return g.lad != 0 && g.mode == MODE_CART && !g.seg && !g.xlad && l < g.ndim - 1;
        });
    for (int l = 0; l < 3; ++l)
        line_slot(P.filt[l], PASS_FILTER, l, 0, [](const GridDev &g) {
            return g.filter != 0 && !g.seg;
        });
    P.resid = point_list(PASS_RESID, 0, 0, [&](int i) {
        return P.grids[i].fused_resid ? 0 : P.grids[i].nchunks;
    });
    for (int target = 0; target < 2; ++target)
        for (int f = 0; f < 6; ++f) {
            const int li = point_list(PASS_FACE, f, target, [&](int i) {
                const GridDev &g = P.grids[i];
                const int l = f >> 1;
                if (l >= g.ndim || g.xbc[f] == XBC_NONE) return 0;
                if (target == 1 && g.fuse_faces) return 0;   // done inside the passes
                if (target == 0 && !P.host[i].init) return 0;
                const long long nf = g.N / g.n[l];
                return (int)((nf + kChunk - 1) / kChunk);
            });
            (target ? P.face : P.face_init)[f] = li;
        }
    P.init = point_list(PASS_INIT, 0, 0, [&](int i) {
        return P.host[i].init ? P.grids[i].nchunks : 0;
    });
}

// ---------------------------------------------------------------------
// live kernel timing
static const char *kind_name(int kind)
{
    switch (kind) {
    case PASS_CART: return "k_cart";
    case PASS_D1: return "k_d1";
    case PASS_D2: return "k_d2";
    case PASS_D12: return "k_d12";
    case PASS_UWADV: return "k_uwadv";
    case PASS_FILTER: return "k_filter";
    case PASS_FINAL: return "k_final";
    case PASS_RESID: return "k_resid";
    case PASS_FACE: return "k_face";
    case PASS_INIT: return "k_init";
    case PASS_LAD: return "k_lad";
    case PASS_SCART: return "k_seg_cart";
    case PASS_SCART_LAST: return "k_seg_cart_fin";
    case PASS_CFIN: return "k_cart_finish";
    case PASS_XSTAGE: return "k_xstage";
    case PASS_XLAD: return "k_xlad";
    case PASS_SFILTER: return "k_seg_filter";
    case PASS_SLAD: return "k_seg_lad";
    default: return "k_finalize";
    }
}

// Compulsory field accesses per point of one launch of `kind` on grid g:
// every distinct field the pass must read or write once.
static double point_accesses(const GridDev &g, int kind, int l, int stage)
{
    const int d = g.ndim;
    const bool last = l == d - 1;
    const int met = g.uniform ? 0 : d * d;
    const int rk4 = g.rk;
    // fields touched by the pointwise stage finish
    auto finish = [&](int src_counted) {
        double r = src_counted ? 0 : 1;            // stage value
        if (stage > 0) r += 1;                     // phi^n
        if (rk4) r += 1;                           // acc read (stage 0: the carried remainder)
        if (stage > 0) r += 1;                     // dt read
        double w = 1;                              // new stage value
        if (rk4) w += 1;                           // acc write (stage 3: the remainder)
        if (stage == 0) w += 1;                    // dt write
        if (g.lad) r += 1;                         // LAD field
        return r + w;
    };
    if (kind == PASS_SCART || kind == PASS_SCART_LAST) kind = PASS_CART;
    if (kind == PASS_SFILTER) kind = PASS_FILTER;
    if (kind == PASS_SLAD) kind = PASS_LAD;
    switch (kind) {
    case PASS_CART: {
        const int np = 1 + g.need_lap;             // partial sums
        double a = 1;                              // source line
        if (l > 0) a += np;
        if (!last || g.seg_split) a += np;
        else a += finish(1) - (g.lad ? 0 : 0);
        return a;
    }
    case PASS_CFIN:
        return (1 + g.need_lap) + finish(0);       // the two sums + the finish's fields
    case PASS_XSTAGE:
        return finish(0);                          // the stage value (and its neighbours) + the finish's fields
    case PASS_XLAD:
        return 2;                                  // phi^n in, sensor out; sensor in, field out
    case PASS_D1:
        // phi in, F_l out; at stage 0 of an LAD grid the sensor part:
        // metrics in, sensor sum in (after the first direction) and out
        return 2 + ((stage == 0 && g.lad) ? (met / d) + (l > 1 ? 1 : 0) + 1 : 0);
    case PASS_D2: {
        const int np = 1 + g.curv;
        double a = d + met;                        // F and metrics
        if (l > 0) a += np;
        if (!last) a += np;
        else a += finish(0);
        if (stage == 0 && g.lad) a += last ? 1 : 2;   // LAD field smoothed in place
        if (last && g.fnext && stage < g.stages - 1) a += 1;   // next stage's F_l out
        return a;
    }
    case PASS_D12:
        // phi in, F_0 out, the other F and the metrics in, partial sums out
        // (+ the LAD sensor sum in and the smoothed field out at stage 0)
        return 2 + (d - 1) + met + (1 + g.curv) + ((stage == 0 && g.lad) ? 2 : 0);
    case PASS_FINAL:
        return (g.uw ? 2 : d) + met + finish(0);
    case PASS_UWADV:
        return 1 + met + 2;                        // phi (and neighbours), metrics in; adv, |U|^2 out
    case PASS_FILTER:
        return last && g.fused_resid ? 3 : 2;      // (+ phi read/write when fused)
    case PASS_RESID:
        return 3;
    case PASS_LAD:
        return stage == 0 ? (l == 0 ? 2 : 3) + met / d : 2;
    case PASS_INIT:
        return 1;
    default:
        return 0;
    }
}

static double launch_bytes(const Plan &P, const ItemList &L, int stage)
{
    if (L.kind == PASS_FACE) return 0.0;
    const double S = P.fp64 ? 8.0 : 4.0;
    double b = 0.0;
    if (L.kind == PASS_XSTAGE || L.kind == PASS_XLAD) {
        // the points each item finishes (its tile's own part of its chunk)
        for (int i = 0; i < L.count; ++i) {
            const Item &it = P.items[L.first + i];
            const GridDev &g = P.grids[it.grid];
            const int ntx = (g.n[0] + kXTX - 1) / kXTX, nty = (g.n[1] + kXTY - 1) / kXTY;
            const int n2 = g.ndim == 3 ? g.n[2] : 1;
            const int kz = L.kind == PASS_XLAD ? g.xlkz : L.np == 2 ? g.xkz : g.xkz2;
            const int tx = it.tile % ntx, ty = (it.tile / ntx) % nty, zc = it.tile / (ntx * nty);
            const double pts = (double)std::min(kXTX, g.n[0] - tx * kXTX) *
                               std::min(kXTY, g.n[1] - ty * kXTY) * std::min(kz, n2 - zc * kz);
            b += pts * point_accesses(g, L.kind, L.l, stage) * S;
        }
        return b;
    }
    int last_grid = -1;
    for (int i = 0; i < L.count; ++i) {
        const int gi = P.items[L.first + i].grid;
        if (gi == last_grid) continue;
        last_grid = gi;
        const GridDev &g = P.grids[gi];
        b += (double)g.N * point_accesses(g, L.kind, L.l, stage) * S;
    }
    return b;
}

static hipEvent_t pool_event(wd_ctx *ctx)
{
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

static void prof_begin(wd_ctx *ctx, PendingLaunch &pl, const char *name, double bytes, hipStream_t s)
{
    pl.a = pool_event(ctx);
    pl.b = pool_event(ctx);
    pl.name = name;
    pl.bytes = bytes;
    (void)hipEventRecord(pl.a, s);
}

static void prof_end(wd_ctx *ctx, PendingLaunch &pl, hipStream_t s)
{
    (void)hipEventRecord(pl.b, s);
    ctx->pending.push_back(pl);
}

// after a stream sync: fold finished launches into the statistics
void prof_collect(wd_ctx *ctx)
{
    for (auto &pl : ctx->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pl.a, pl.b) == hipSuccess) {
            KStat &k = ctx->kstats[pl.name];
            k.launches += 1;
            k.ms += ms;
            k.bytes += pl.bytes;
        } else {
            (void)hipGetLastError();   // do not leave a sticky error behind
        }
        ctx->ev_pool.push_back(pl.a);
        ctx->ev_pool.push_back(pl.b);
    }
    ctx->pending.clear();
}

// ---------------------------------------------------------------------
// issuing work
// Workgroups of one launch: a line pass gets as many as the chip holds at
// once (its kernel's occupancy times the compute units), so a persistent
// loop over more items never leaves a partial second round of workgroups;
// pointwise passes get up to 4 (FP32) or 2 (FP64) per compute unit.
static int nwg_for(wd_ctx *ctx, int fp64, int kind, int np, int count, int l = 0)
{
    int per = fp64 ? 2 : 4;
    switch (kind) {
    case PASS_CART: case PASS_D1: case PASS_D2: case PASS_D12: case PASS_FILTER: case PASS_LAD:
        per = std::min(4, line_blocks_per_cu(kind, fp64, np));
        break;
    case PASS_XSTAGE:
        per = xstage_blocks_per_cu(fp64, l, np == 2);
        break;
    case PASS_XLAD:
        per = xlad_blocks_per_cu(fp64, np);
        break;
    default:
        break;
    }
    int cap = ctx->cus * per;
    cap = std::max(8, cap & ~7);
    return std::min(count, cap);
}

void issue_list(wd_ctx *ctx, const Plan &P, int li, int stage, hipStream_t s)
{
    const ItemList &L = P.lists[li];
    if (L.count == 0) return;
    const int arg = (L.kind == PASS_FACE || L.kind == PASS_INIT) ? L.arg : stage;
    PendingLaunch pl;
    if (ctx->profile) {
        // line passes are timed per direction (and LAD phase)
        std::string name = kind_name(L.kind);
        switch (L.kind) {
        case PASS_LAD: case PASS_SLAD:
            name += "/p" + std::to_string(stage);
            [[fallthrough]];
        case PASS_CART: case PASS_D1: case PASS_D2: case PASS_FILTER: case PASS_SCART:
        case PASS_SCART_LAST: case PASS_SFILTER:
            name += "/d" + std::to_string(L.l);
            break;
        case PASS_XSTAGE:
            name += L.np == 2 ? "/fast" : "/edge";
            break;
        case PASS_XLAD:
            name += L.np == 2 ? "/smooth" : "/sensor";
            break;
        default:
            break;
        }
        prof_begin(ctx, pl, name.c_str(), launch_bytes(P, L, stage), s);
    }
    if (L.kind == PASS_SCART || L.kind == PASS_SCART_LAST || L.kind == PASS_SFILTER ||
        L.kind == PASS_SLAD) {
        size_t lds = 0;
        int last = -1;
        for (int i = 0; i < L.count; ++i) {
            const int gi = P.items[L.first + i].grid;
            if (gi == last) continue;
            last = gi;
            lds = std::max(lds, seg_lds_bytes(P.grids[gi], L.kind, L.l, P.fp64));
        }
        // workgroups the chip holds at once: registers and LDS (160 KiB per
        // compute unit) permitting
        int per = seg_blocks_per_cu_regs(L.kind, P.fp64, L.np);
        per = std::max(1, std::min(per, (int)(163840 / std::max<size_t>(lds, 1))));
        int nwg = std::min(L.count, std::max(8, (ctx->cus * per) & ~7));
        launch_seg(L.kind, P.fp64, L.np, P.d_grids, P.d_items + L.first, L.count, L.l, arg, nwg,
                   lds, s);
    } else {
        launch_pass(L.kind, P.fp64, L.np, P.d_grids, P.d_items + L.first, L.count, L.l, arg,
                    nwg_for(ctx, P.fp64, L.kind, L.np, L.count, L.l), s);
    }
    if (ctx->profile) prof_end(ctx, pl, s);
}

static void issue_seg(wd_ctx *ctx, const Plan &P, const Slot &Sl, int stage, hipStream_t s)
{
    for (int c = 0; c < 4; ++c)
        if (Sl.list[c] >= 0) issue_list(ctx, P, Sl.list[c], stage, s);
}

void issue_slot(wd_ctx *ctx, const Plan &P, const Slot &S, int stage, hipStream_t s)
{
    for (int c = 0; c < 4; ++c)
        if (S.list[c] >= 0) issue_list(ctx, P, S.list[c], stage, s);
}

void issue_faces(wd_ctx *ctx, const Plan &P, int target, hipStream_t s)
{
    for (int f = 0; f < 6; ++f) {
        const ItemList &L = P.lists[target ? P.face[f] : P.face_init[f]];
        if (L.count == 0) continue;
        PendingLaunch pl;
        if (ctx->profile) prof_begin(ctx, pl, "k_face", 0.0, s);
        launch_pass(PASS_FACE, P.fp64, 1, P.d_grids, P.d_items + L.first, L.count, f, target,
                    nwg_for(ctx, P.fp64, L.kind, L.np, L.count), s);
        if (ctx->profile) prof_end(ctx, pl, s);
    }
}

void issue_iteration(wd_ctx *ctx, const Plan &P, hipStream_t s)
{
    // LAD diffusivity from phi^n: sensor per direction (the last one also
    // smooths along itself), then smoothing along the other directions
    issue_list(ctx, P, P.xlad[0], 0, s);
    issue_list(ctx, P, P.xlad[1], 0, s);
    for (int l = 0; l < P.maxdim; ++l) issue_slot(ctx, P, P.lad0[l], 0, s);
    for (int l = 0; l < P.maxdim; ++l) issue_seg(ctx, P, P.slad0[l], 0, s);
    for (int l = 0; l < P.maxdim; ++l) issue_slot(ctx, P, P.lad1[l], 1, s);
    for (int l = 0; l < P.maxdim; ++l) issue_seg(ctx, P, P.slad1[l], 1, s);
    for (int st = 0; st < P.stages; ++st) {
        for (int l = 0; l < P.maxdim; ++l) issue_slot(ctx, P, P.cart[l], st, s);
        for (int l = 0; l < P.maxdim; ++l) {
            issue_seg(ctx, P, P.scart[l], st, s);
            issue_seg(ctx, P, P.scartl[l], st, s);
        }
        for (int r = 0; r < 3; ++r)
            for (int f = 1; f >= 0; --f) issue_list(ctx, P, P.xstage[r][f], st, s);
        issue_list(ctx, P, P.cfin, st, s);
        for (int l = 0; l < P.maxdim; ++l) issue_slot(ctx, P, st == 0 ? P.d1[l] : P.d1n[l], st, s);
        issue_slot(ctx, P, P.d12, st, s);
        for (int l = 1; l < P.maxdim; ++l) issue_slot(ctx, P, P.d2[l], st, s);
        issue_list(ctx, P, P.uwadv, st, s);
        issue_list(ctx, P, P.fin, st, s);
        issue_faces(ctx, P, 1, s);
    }
    for (int l = 0; l < P.maxdim; ++l) issue_slot(ctx, P, P.filt[l], 0, s);
    for (int l = 0; l < P.maxdim; ++l) issue_seg(ctx, P, P.sfilt[l], 0, s);
    issue_faces(ctx, P, 1, s);
    issue_list(ctx, P, P.resid, 0, s);
    PendingLaunch pl;
    if (ctx->profile) prof_begin(ctx, pl, "k_finalize", 0.0, s);
    launch_finalize(P.d_grids, P.n, s);
    if (ctx->profile) prof_end(ctx, pl, s);
}

void issue_init(wd_ctx *ctx, const Plan &P, hipStream_t s)
{
    issue_list(ctx, P, P.init, 0, s);
    issue_faces(ctx, P, 0, s);
}

int upload_plan(wd_ctx *ctx, const Plan &P, hipStream_t s)
{
    if (hipMemcpyAsync(P.d_grids, P.grids.data(), P.grids.size() * sizeof(GridDev),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(P.d_items, P.items.data(), P.items.size() * sizeof(Item),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(WD_ERR_HIP, "plan upload failed");
    (void)ctx;
    return WD_OK;
}

// ---------------------------------------------------------------------
// graphs of K iterations, cached per plan
static bool same_plan(const Plan &a, const CachedGraph &c)
{
    if (a.grids.size() * sizeof(GridDev) != c.grids_bytes.size()) return false;
    if (a.items.size() * sizeof(Item) != c.items_bytes.size()) return false;
    if (std::memcmp(a.grids.data(), c.grids_bytes.data(), c.grids_bytes.size()) != 0) return false;
    if (std::memcmp(a.items.data(), c.items_bytes.data(), c.items_bytes.size()) != 0) return false;
    return a.d_grids == c.d_grids && a.d_items == c.d_items;
}

static void drop_graph(wd_ctx *ctx, CachedGraph &c)
{
    (void)hipGraphExecDestroy(c.exec);
    for (auto e : c.ev) ctx->ev_pool.push_back(e);
    c.ev.clear();
}

CachedGraph *graph_for(wd_ctx *ctx, const Plan &P, int K)
{
    for (auto &c : ctx->graphs)
        if (c.K == K && c.profile == ctx->profile && same_plan(P, c)) {
            c.stamp = ++ctx->clock;
            return &c;
        }
    prof_collect(ctx);
    hipStream_t s = ctx->stream;
    // relaxed: other threads (the caller's, a server's) keep full use of
    // the runtime while this context's stream is being captured
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
        fail(WD_ERR_HIP, "hipStreamBeginCapture failed");
        return nullptr;
    }
    for (int k = 0; k < K; ++k) issue_iteration(ctx, P, s);
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(s, &graph) != hipSuccess || !graph) {
        fail(WD_ERR_HIP, "hipStreamEndCapture failed");
        return nullptr;
    }
    std::vector<PendingLaunch> captured;
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        fail(WD_ERR_HIP, "hipGraphInstantiate failed");
        return nullptr;
    }
    (void)hipGraphDestroy(graph);
    if (ctx->graphs.size() >= 16) {
        auto oldest = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                       [](const CachedGraph &a, const CachedGraph &b) { return a.stamp < b.stamp; });
        drop_graph(ctx, *oldest);
        ctx->graphs.erase(oldest);
    }
    CachedGraph c;
    c.K = K;
    c.profile = ctx->profile;
    c.exec = exec;
    for (auto &pl : captured) {
        c.ev.push_back(pl.a);
        c.ev.push_back(pl.b);
        c.ev_name.push_back(pl.name);
        c.ev_bytes.push_back(pl.bytes);
    }
    c.d_grids = P.d_grids;
    c.d_items = P.d_items;
    c.grids_bytes.assign(reinterpret_cast<const unsigned char *>(P.grids.data()),
                         reinterpret_cast<const unsigned char *>(P.grids.data()) + P.grids.size() * sizeof(GridDev));
    c.items_bytes.assign(reinterpret_cast<const unsigned char *>(P.items.data()),
                         reinterpret_cast<const unsigned char *>(P.items.data()) + P.items.size() * sizeof(Item));
    c.stamp = ++ctx->clock;
    ctx->graphs.push_back(std::move(c));
    return &ctx->graphs.back();
}

void ctx_drop_graphs(wd_ctx *ctx)
{
    for (auto &c : ctx->graphs) drop_graph(ctx, c);
    ctx->graphs.clear();
}

// Iterate until every grid of the plan has stopped.  States are read back
// after each graph replay of K iterations.
int run_plan(wd_ctx *ctx, Plan &P, int K, std::vector<GridState> &states)
{
    hipStream_t s = ctx->stream;
    int maxit = 0;
    for (int i = 0; i < P.n; ++i) maxit = std::max(maxit, P.grids[i].max_iter);
    // profiling mode launches directly, each kernel bracketed by events
    const int use_graph = ctx->use_graphs && !ctx->profile && !P.arena;
    CachedGraph *cg = use_graph ? graph_for(ctx, P, K) : nullptr;
    if (use_graph && !cg) return WD_ERR_HIP;
    states.resize(P.n);
    // points the current work lists cover: once the grids still running
    // hold half of them or less, the lists are rebuilt over those grids
    // alone (a stopped grid's items only test its flag, but every pass of
    // every iteration still launches over them)
    long long plan_pts = 0;
    for (int i = 0; i < P.n; ++i) plan_pts += P.grids[i].N;
    const long long max_rounds = (maxit + K - 1) / K + 1;
    int prev_iter = 0;
    for (long long r = 0; r < max_rounds; ++r) {
        if (cg) {
            if (hipGraphLaunch(cg->exec, s) != hipSuccess) return fail(WD_ERR_HIP, "hipGraphLaunch failed");
        } else {
            for (int k = 0; k < K; ++k) issue_iteration(ctx, P, s);
        }
        if (hipMemcpyAsync(ctx->pinned_states, P.d_states, P.n * sizeof(GridState),
                           hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(WD_ERR_HIP, "state read-back failed: %s", hipGetErrorString(hipGetLastError()));
        bool all = true;
        int max_iter_now = 0;
        for (int i = 0; i < P.n; ++i) {
            states[i] = ctx->pinned_states[i];
            all &= states[i].done != 0;
            max_iter_now = std::max(max_iter_now, states[i].iter);
        }
        if (ctx->profile) {
            // keep only launches of iterations in which some grid was active
            const int active = std::min(K, max_iter_now - prev_iter);
            const size_t per_iter = ctx->pending.size() / K;
            const size_t keep = (size_t)active * per_iter;
            for (size_t i = keep; i < ctx->pending.size(); ++i) {
                ctx->ev_pool.push_back(ctx->pending[i].a);
                ctx->ev_pool.push_back(ctx->pending[i].b);
            }
            if (ctx->pending.size() > keep) ctx->pending.resize(keep);
            prof_collect(ctx);
        }
        prev_iter = max_iter_now;
        if (all) return WD_OK;
        long long live_pts = 0;
        for (int i = 0; i < P.n; ++i)
            if (!states[i].done) live_pts += P.grids[i].N;
        if (P.n > 1 && 2 * live_pts <= plan_pts) {
            P.live.assign(P.n, 0);
            for (int i = 0; i < P.n; ++i) P.live[i] = states[i].done ? 0 : 1;
            build_items(P);
            if (hipMemcpyAsync(P.d_items, P.items.data(), P.items.size() * sizeof(Item),
                               hipMemcpyHostToDevice, s) != hipSuccess)
                return fail(WD_ERR_HIP, "item upload failed");
            plan_pts = live_pts;
            if (use_graph) {
                cg = graph_for(ctx, P, K);
                if (!cg) return WD_ERR_HIP;
            }
        }
    }
    return fail(WD_ERR_HIP, "grids did not stop within max_iter");
}

// FP64 Poisson conversion of grid i of a plan (after the march): phi' is in
// g.phi (solve precision); the distance replaces it, phi' goes to aux.
int poisson_convert(wd_ctx *ctx, const Plan &P, int i, void *aux, hipStream_t s)
{
    const GridDev &g = P.grids[i];
    const GridHost &gh = P.host[i];
    const size_t S = P.fp64 ? 8 : 4;
    if (aux && hipMemcpyAsync(aux, g.phi, (size_t)g.N * S, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(WD_ERR_HIP, "copy of phi' failed");
    double *phip = static_cast<double *>(gh.pois_phip);
    launch_convert(P.fp64, 1, g.phi, phip, g.N, s);
    // FP64 first derivatives of phi' with a one-grid FP64 view
    GridDev v = g;
    v.phi = phip;
    v.lad = 0;
    for (int l = 0; l < g.ndim; ++l) {
        v.F[l] = gh.pois_F[l];
        const LineOpDev *dop = ctx_lineop(ctx, OP_DERIV, g.n[l], g.periodic[l], g.scheme, 0.0, 1,
                                          P.arena);
        if (!dop) return WD_ERR_NO_MEMORY;
        v.dop[l] = *dop;
    }
    v.state = P.d_states + P.n;  // scratch state, never done
    GridState zero{};
    std::vector<Item> items;
    if (hipMemcpyAsync(v.state, &zero, sizeof zero, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(P.d_aux, &v, sizeof v, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(WD_ERR_HIP, "poisson view upload failed");
    (void)items;
    for (int l = 0; l < g.ndim; ++l) {
        const int nt = g.ntiles[l];
        std::vector<Item> it(nt);
        for (int t = 0; t < nt; ++t) it[t] = Item{0, t};
        Item *d_it = P.d_items + P.items.size();  // spare item space after the plan's lists
        if ((long long)(P.items.size() + nt) > P.items_cap)
            return fail(WD_ERR_INVALID_ARG, "internal: no item space for the Poisson passes");
        if (hipMemcpyAsync(d_it, it.data(), nt * sizeof(Item), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(WD_ERR_HIP, "poisson items upload failed");
        launch_pass(PASS_D1, 1, tile_np(g, l), P.d_aux, d_it, nt, l, 0,
                    nwg_for(ctx, 1, PASS_D1, tile_np(g, l), nt), s);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(WD_ERR_HIP, "poisson pass failed");
    }
    GridDev w = g;  // metrics in the solve precision, F in FP64
    for (int l = 0; l < g.ndim; ++l) w.F[l] = v.F[l];
    if (hipMemcpyAsync(P.d_aux2, &w, sizeof w, hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(WD_ERR_HIP, "poisson view upload failed");
    launch_poisson_dist(P.d_aux2, P.fp64, g.N, phip, g.phi, s);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(WD_ERR_HIP, "poisson conversion failed");
    return WD_OK;
}

// one batch from start to finish on the context stream
int solve_plan(wd_ctx *ctx, Plan &P, void *const *aux, double *const *hists, int hist_cap,
               int *iters, int *status)
{
    hipStream_t s = ctx->stream;
    int rc = upload_plan(ctx, P, s);
    if (rc) return rc;
    issue_init(ctx, P, s);
    std::vector<GridState> states;
    // iterations per graph: at most graph_iters, spread evenly over the
    // rounds the longest grid may need, so a run to max_iter issues few
    // no-op iterations after the last grid stops
    int maxit = 1;
    for (int i = 0; i < P.n; ++i) maxit = std::max(maxit, P.grids[i].max_iter);
    const int gi = std::max(1, ctx->graph_iters);
    const int rounds = (maxit + gi - 1) / gi;
    rc = run_plan(ctx, P, (maxit + rounds - 1) / rounds, states);
    if (rc) return rc;
    int worst = WD_OK;
    for (int i = 0; i < P.n; ++i) {
        const GridDev &g = P.grids[i];
        int st = states[i].status;
        if (g.eq == 2) {
            int r2 = poisson_convert(ctx, P, i, aux ? aux[i] : nullptr, s);
            if (r2) return r2;
        }
        if (iters) iters[i] = states[i].iter;
        if (status) status[i] = st;
        if (hists && hists[i] && hist_cap > 0) {
            const int nh = std::min(std::min(states[i].iter, hist_cap), g.hist_cap);
            if (nh > 0 &&
                hipMemcpyAsync(hists[i], g.hist, (size_t)nh * 16, hipMemcpyDeviceToHost, s) != hipSuccess)
                return fail(WD_ERR_HIP, "history copy failed");
        }
        if (st < 0 && (worst >= 0 || st < worst)) worst = st;
        else if (worst >= 0 && st > worst) worst = st;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(WD_ERR_HIP, "final sync failed");
    if (worst == WD_ERR_DIVERGED) fail(WD_ERR_DIVERGED, "a pseudo-step change was not finite");
    if (worst == WD_ERR_WARM_RUNAWAY) fail(WD_ERR_WARM_RUNAWAY, "warm start stopped by the runaway check");
    return worst;
}

}  // namespace wd

// =====================================================================
// C ABI
using namespace wd;

struct StreamJoin {
    wd_ctx *ctx;
    hipStream_t user;
    StreamJoin(wd_ctx *c, void *stream) : ctx(c), user(static_cast<hipStream_t>(stream))
    {
        (void)hipEventRecord(ctx->ev_in, user);
        (void)hipStreamWaitEvent(ctx->stream, ctx->ev_in, 0);
    }
    ~StreamJoin()
    {
        (void)hipEventRecord(ctx->ev_out, ctx->stream);
        (void)hipStreamWaitEvent(user, ctx->ev_out, 0);
    }
};

extern "C" {

const char *wd_version(void) { return "wd 1.0 gfx950"; }

const char *wd_last_error(void) { return g_last_error.c_str(); }

int wd_method_default(wd_method *m)
{
    if (!m) return fail(WD_ERR_INVALID_ARG, "null method");
    std::memset(m, 0, sizeof *m);
    m->equation = WD_EQ_HJ;
    m->gamma = WD_GAMMA_LAD;
    m->curvature = 0;
    m->eps = 0.2;
    m->c_lad = 0.1;
    m->nu0 = 1e-3;
    m->eps0 = 1e-6;
    m->scheme = WD_C6;
    m->filter = 1;
    m->alpha_f = 0.48;   // strong end of Sec. 3.4's 0.48-0.495: stable with corners
    m->rk = WD_RK4;
    m->sigma = 1.0;
    m->tol = 1e-10;
    m->max_iter = 100000;
    m->stall_window = 0;
    m->precision = WD_FP64;
    m->warm_start = 0;
    m->warm_probe = 300;
    return WD_OK;
}

int wd_ctx_create(int device, wd_ctx **out)
{
    if (!out) return fail(WD_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(WD_ERR_INVALID_ARG, "no HIP device %d (found %d)", device, count);
    if (hipSetDevice(device) != hipSuccess) return fail(WD_ERR_HIP, "hipSetDevice(%d) failed", device);
    wd_ctx *c = new wd_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return fail(WD_ERR_HIP, "hipGetDeviceProperties failed");
    }
    c->cus = prop.multiProcessorCount;
    std::snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
    // occupancy of every line kernel, queried now rather than on a first
    // launch that may sit inside a graph capture
    for (int fp64 = 0; fp64 < 2; ++fp64)
        for (int np = 1; np <= 8; np *= 2)
            for (int kind : {PASS_CART, PASS_D1, PASS_D2, PASS_D12, PASS_FILTER, PASS_LAD})
                (void)line_blocks_per_cu(kind, fp64, np);
    for (int fp64 = 0; fp64 < 2; ++fp64)
        for (int kind : {PASS_SCART, PASS_SCART_LAST, PASS_SFILTER, PASS_SLAD})
            for (int M : {16, 24, 32}) (void)seg_blocks_per_cu_regs(kind, fp64, M);
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&c->pinned_states, sizeof(GridState) * 4096, 0) != hipSuccess) {
        delete c;
        return fail(WD_ERR_HIP, "stream/event/pinned allocation failed");
    }
    c->pinned_cap = 4096;
    // the device's static scratch for calls that allocate nothing
    if (noalloc_scratch(device, &c->noalloc) != 0) {
        (void)hipStreamDestroy(c->stream);
        (void)hipEventDestroy(c->ev_in);
        (void)hipEventDestroy(c->ev_out);
        (void)hipHostFree(c->pinned_states);
        delete c;
        return fail(WD_ERR_HIP, "hipGetSymbolAddress of the scratch array failed on device %d",
                    device);
    }
    c->noalloc_bytes = kNoAllocBytes;
    const char *g = std::getenv("WD_NO_GRAPHS");
    c->use_graphs = !(g && g[0] == '1');
    c->graph_iters = 32;
    *out = c;
    return WD_OK;
}

int wd_ctx_destroy(wd_ctx *ctx)
{
    if (!ctx) return WD_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx_drop_graphs(ctx);
    prof_collect(ctx);
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto &kv : ctx->ops) (void)hipFree(kv.second.mem);
    for (auto &kv : ctx->segops)
        if (kv.second.mem) (void)hipFree(kv.second.mem);
    if (ctx->pinned_states) (void)hipHostFree(ctx->pinned_states);
    (void)hipEventDestroy(ctx->ev_in);
    (void)hipEventDestroy(ctx->ev_out);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return WD_OK;
}

int wd_workspace_bytes(wd_ctx *ctx, int n, const wd_grid_desc *descs,
                       const wd_method *methods, size_t *bytes)
{
    (void)ctx;
    if (!bytes || n < 1 || !descs || !methods) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < n; ++i) {
        int rc = check_desc(&descs[i]);
        if (!rc) rc = check_walls(&descs[i]);
        if (!rc) rc = check_method(&methods[i]);
        if (rc) return rc;
    }
    *bytes = batch_bytes(n, descs, methods);
    return WD_OK;
}

int wd_solve_batched(wd_ctx *ctx, int n, const wd_grid_desc *descs, const wd_method *methods,
                     void *const *phis, void *const *aux, double *const *hists, int hist_cap,
                     int *iters, int *status, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx || n < 1 || !descs || !methods || !phis) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    for (int i = 0; i < n; ++i) {
        int rc = check_desc(&descs[i]);
        if (!rc) rc = check_walls(&descs[i]);
        if (!rc) rc = check_method(&methods[i]);
        if (rc) return rc;
        if (!phis[i]) return fail(WD_ERR_INVALID_ARG, "phi[%d] is null", i);
        if (methods[i].precision != methods[0].precision || methods[i].rk != methods[0].rk)
            return fail(WD_ERR_UNSUPPORTED, "a batch needs one precision and one RK scheme");
    }
    if (n + 1 > ctx->pinned_cap) return fail(WD_ERR_UNSUPPORTED, "batch of %d grids is too large", n);
    (void)hipSetDevice(ctx->device);
    StreamJoin join(ctx, stream);
    Plan P;
    int rc = plan_batch(ctx, n, descs, methods, phis, ws, ws_bytes, P);
    if (rc) return rc;
    return solve_plan(ctx, P, aux, hists, hist_cap, iters, status);
}

int wd_solve(wd_ctx *ctx, const wd_grid_desc *desc, const wd_method *method, void *phi,
             void *phi_aux, double *hist, int hist_cap, int *iters, void *ws, size_t ws_bytes,
             void *stream)
{
    void *phis[1] = {phi};
    void *auxs[1] = {phi_aux};
    double *hs[1] = {hist};
    int st = 0;
    int rc = wd_solve_batched(ctx, 1, desc, method, phis, auxs, hs, hist_cap, iters, &st, ws,
                              ws_bytes, stream);
    return rc;
}

int wd_solve_noalloc(wd_ctx *ctx, const wd_grid_desc *desc, const wd_method *method, void *phi,
                     void *phi_aux, double *hist, int hist_cap, int *iters, void *stream)
{
    if (!ctx || !desc || !method || !phi) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    int rc = check_desc(desc);
    if (!rc) rc = check_walls(desc);
    if (!rc) rc = check_method(method);
    if (rc) return rc;
    if (!ctx->noalloc) return fail(WD_ERR_HIP, "no scratch on this context");
    // workspace first, the line-operator tables after it
    const size_t ws = batch_bytes(1, desc, method);
    if (ws > ctx->noalloc_bytes)
        return fail(WD_ERR_NO_MEMORY,
                    "the grid needs a %zu-byte workspace; the scratch of calls that allocate "
                    "nothing holds %zu bytes", ws, ctx->noalloc_bytes);
    (void)hipSetDevice(ctx->device);
    StreamJoin join(ctx, stream);
    TableArena ar;
    ar.base = static_cast<unsigned char *>(ctx->noalloc) + ((ws + 255) & ~(size_t)255);
    ar.cap = ctx->noalloc_bytes - ((ws + 255) & ~(size_t)255);
    ar.stream = ctx->stream;
    Plan P;
    void *phis[1] = {phi};
    void *auxs[1] = {phi_aux};
    double *hs[1] = {hist};
    int st = 0;
    rc = plan_batch(ctx, 1, desc, method, phis, ctx->noalloc, ws, P, &ar);
    if (rc) {
        (void)hipStreamSynchronize(ctx->stream);   // table uploads read host memory held here
        return rc;
    }
    rc = solve_plan(ctx, P, auxs, hs, hist_cap, iters, &st);
    (void)hipStreamSynchronize(ctx->stream);
    return rc;
}

int wd_compute_metrics_form(wd_ctx *ctx, const wd_grid_desc *desc, int scheme, int form,
                            const double *coords, const double *period, void *out,
                            int out_precision, void *stream)
{
    if (!ctx || !desc || !coords || !out) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    if (form != WD_METRICS_INVERSE && form != WD_METRICS_CONSERVATIVE)
        return fail(WD_ERR_INVALID_ARG, "bad metric form");
    wd_grid_desc d = *desc;
    d.metric_mode = WD_METRIC_UNIFORM;
    for (int l = 0; l < 3; ++l) d.h[l] = 1.0;
    d.metrics = nullptr;
    int rc = check_desc(&d);
    if (rc) return rc;
    if (scheme < WD_E2 || scheme > WD_UW) return fail(WD_ERR_INVALID_ARG, "bad scheme");
    if (scheme == WD_UW) scheme = WD_E2;   // the upwind baseline's metrics are central E2
    const int dim = d.ndim;
    // the conservative form differs from the inverse in 3D only (in 2D both
    // are the adjugate of the coordinate derivatives)
    const bool gcl = form == WD_METRICS_CONSERVATIVE && dim == 3;
    if (gcl && period)
        for (int k = 0; k < 9; ++k)
            if (period[k] != 0.0)
                return fail(WD_ERR_UNSUPPORTED, "conservative metrics: coordinates jump across a seam");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    StreamJoin join(ctx, stream);
    hipStream_t s = ctx->stream;
    const long long N = npoints(d);
    // scratch: J (dim*dim*N doubles), for the conservative form the products
    // Q (9N) and their derivatives (18N), one grid view, items, state
    void *scratch = nullptr;
    long long maxt = 0;
    for (int l = 0; l < dim; ++l) maxt = std::max(maxt, N / d.n[l]);
    const size_t jb = al256((size_t)dim * dim * N * 8);
    const size_t qb = gcl ? al256((size_t)9 * N * 8) : 0, db = gcl ? al256((size_t)18 * N * 8) : 0;
    const size_t bytes = jb + qb + db + al256(sizeof(GridDev)) +
                         al256((size_t)maxt * sizeof(Item)) + al256(sizeof(GridState));
    if (hipMalloc(&scratch, bytes) != hipSuccess) return fail(WD_ERR_NO_MEMORY, "metric scratch allocation failed");
    unsigned char *b = static_cast<unsigned char *>(scratch);
    double *J = reinterpret_cast<double *>(b);
    double *Q = reinterpret_cast<double *>(b + jb);
    double *D = reinterpret_cast<double *>(b + jb + qb);
    GridDev *dg = reinterpret_cast<GridDev *>(b + jb + qb + db);
    Item *ditems = reinterpret_cast<Item *>(reinterpret_cast<unsigned char *>(dg) + al256(sizeof(GridDev)));
    GridState *dst = reinterpret_cast<GridState *>(reinterpret_cast<unsigned char *>(ditems) +
                                                   al256((size_t)maxt * sizeof(Item)));
    GridState zero{};
    rc = WD_OK;
    if (hipMemcpyAsync(dst, &zero, sizeof zero, hipMemcpyHostToDevice, s) != hipSuccess)
        rc = fail(WD_ERR_HIP, "state upload failed");
    GridDev g;
    std::memset(&g, 0, sizeof g);
    g.ndim = dim;
    g.mode = MODE_GENERAL;
    g.N = N;
    long long st = 1;
    for (int l = 0; l < 3; ++l) {
        g.n[l] = l < dim ? d.n[l] : 1;
        g.stride[l] = st;
        st *= g.n[l];
    }
    for (int l = 0; l < dim; ++l) g.periodic[l] = d.bc[l][0] == WD_BC_PERIODIC;
    g.uniform = 1;
    g.scheme = scheme;
    switch (scheme) {
    case WD_E2: g.da = 1.0; g.dradius = 1; break;
    case WD_E4: g.da = 4.0 / 3.0; g.db = -1.0 / 3.0; g.dradius = 2; break;
    case WD_E6: g.da = 1.5; g.db = -0.6; g.dc = 0.1; g.dradius = 3; break;
    case WD_C4: g.da = 1.5; g.dradius = 1; g.compact = 1; break;
    default: g.da = 14.0 / 9.0; g.db = 1.0 / 9.0; g.dradius = 2; g.compact = 1; break;
    }
    g.state = dst;
    for (int l = 0; l < dim && !rc; ++l) {
        const LineOpDev *op = ctx_lineop(ctx, OP_DERIV, d.n[l], g.periodic[l], scheme, 0.0, 1);
        if (!op) rc = WD_ERR_NO_MEMORY;
        else g.dop[l] = *op;
        g.tw[l] = pick_tile(ctx, d, l, 1);
        g.ntiles[l] = l == 0 ? (int)((N / d.n[0] + g.tw[0] - 1) / g.tw[0])
                             : (int)((N / ((long long)d.n[0] * d.n[l])) * ((d.n[0] + g.tw[l] - 1) / g.tw[l]));
    }
    // dst = D_l src (FP64, index space), `jump` added across a periodic seam
    auto deriv = [&](const double *src, int l, double *out_l, double jump) {
        GridDev v = g;
        v.phi = const_cast<double *>(src);
        v.F[l] = out_l;
        v.jump[l] = jump;
        std::vector<Item> it(g.ntiles[l]);
        for (int t = 0; t < g.ntiles[l]; ++t) it[t] = Item{0, t};
        if (hipMemcpyAsync(dg, &v, sizeof v, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(ditems, it.data(), it.size() * sizeof(Item), hipMemcpyHostToDevice, s) != hipSuccess)
            return fail(WD_ERR_HIP, "metric view upload failed");
        launch_pass(PASS_D1, 1, tile_np(g, l), dg, ditems, g.ntiles[l], l, 0,
                    nwg_for(ctx, 1, PASS_D1, tile_np(g, l), g.ntiles[l]), s);
        if (hipStreamSynchronize(s) != hipSuccess) return fail(WD_ERR_HIP, "metric pass failed");
        return (int)WD_OK;
    };
    for (int m = 0; m < dim && !rc; ++m)
        for (int l = 0; l < dim && !rc; ++l)
            rc = deriv(coords + (size_t)m * N, l, J + (size_t)(m * dim + l) * N,
                       period ? period[l * 3 + m] : 0.0);
    if (!rc && gcl) {
        // J xi_{l,m} = (D_q Q[p][m] - D_p Q[q][m]) / 2, (l, p, q) cyclic
        launch_gcl_products(coords, J, Q, N, s);
        for (int l = 0; l < 3 && !rc; ++l) {
            const int p = (l + 1) % 3, q = (l + 2) % 3;
            for (int m = 0; m < 3 && !rc; ++m) {
                rc = deriv(Q + (size_t)(p * 3 + m) * N, q, D + (size_t)((l * 3 + m) * 2) * N, 0.0);
                if (!rc)
                    rc = deriv(Q + (size_t)(q * 3 + m) * N, p, D + (size_t)((l * 3 + m) * 2 + 1) * N, 0.0);
            }
        }
        if (!rc) {
            launch_gcl_combine(J, D, out, out_precision == WD_FP64, N, s);
            if (hipStreamSynchronize(s) != hipSuccess) rc = fail(WD_ERR_HIP, "metric combination failed");
        }
    } else if (!rc) {
        launch_invert(J, out, out_precision == WD_FP64, dim, N, s);
        if (hipStreamSynchronize(s) != hipSuccess) rc = fail(WD_ERR_HIP, "metric inversion failed");
    }
    (void)hipFree(scratch);
    return rc;
}

int wd_compute_metrics(wd_ctx *ctx, const wd_grid_desc *desc, int scheme, const double *coords,
                       const double *period, void *out, int out_precision, void *stream)
{
    return wd_compute_metrics_form(ctx, desc, scheme, WD_METRICS_INVERSE, coords, period, out,
                                   out_precision, stream);
}

int wd_autotune(wd_ctx *ctx, const wd_grid_desc *desc, const wd_method *method, void *phi,
                void *ws, size_t ws_bytes, int iters, int *widths, void *stream)
{
    if (!ctx || !desc || !method || !phi || iters < 1) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    int rc = check_desc(desc);
    if (!rc) rc = check_walls(desc);
    if (!rc) rc = check_method(method);
    if (rc) return rc;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    StreamJoin join(ctx, stream);
    hipStream_t s = ctx->stream;
    wd_method m = *method;
    m.tol = 0.0;                 // run exactly `iters` iterations
    m.max_iter = iters;
    m.stall_window = 0;
    m.warm_start = 0;
    const int fp64 = m.precision == WD_FP64;
    const int prof = ctx->profile;
    ctx->profile = 0;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    void *phis[1] = {phi};
    const wd_grid_desc &d = *desc;
    for (int l = 0; l < d.ndim && !rc; ++l) {
        TuneKey key{d.ndim, d.n[0], d.n[1], d.n[2], l, fp64};
        const int n = d.n[l];
        const int wmax = l == 0 ? std::max(1, kTileMax / n) : std::max(1, std::min(64, kTileMax / n));
        int best_w = pick_tile(ctx, d, l, fp64);
        float best_ms = 1e30f;
        for (int w = 1; w <= wmax && !rc; w *= 2) {
            ctx->tune[key] = w;
            Plan P;
            rc = plan_batch(ctx, 1, desc, &m, phis, ws, ws_bytes, P);
            if (rc) break;
            if (P.grids[0].seg) {
                // the segmented passes fix their own tiles (whole lines per
                // wave): nothing to tune along any direction
                for (int k = 0; k < d.ndim; ++k)
                    if (widths) widths[k] = P.grids[0].sgeo[k].W;
                l = d.ndim;
                break;
            }
            rc = upload_plan(ctx, P, s);
            if (rc) break;
            issue_init(ctx, P, s);
            CachedGraph *cg = graph_for(ctx, P, iters);
            if (!cg) { rc = WD_ERR_HIP; break; }
            float ms = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {   // first replay warms caches
                issue_init(ctx, P, s);
                (void)hipEventRecord(e0, s);
                (void)hipGraphLaunch(cg->exec, s);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(WD_ERR_HIP, "autotune run failed"); break; }
                float t = 0.f;
                (void)hipEventElapsedTime(&t, e0, e1);
                ms = std::min(ms, t);
            }
            if (ms < best_ms) {
                best_ms = ms;
                best_w = w;
            }
        }
        if (l >= d.ndim) break;
        ctx->tune[key] = best_w;
        if (widths) widths[l] = best_w;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->profile = prof;
    return rc;
}

int wd_tune_get(wd_ctx *ctx, const wd_grid_desc *desc, int precision, int *widths)
{
    if (!ctx || !desc || !widths) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    int rc = check_desc(desc);
    if (rc) return rc;
    if (precision != WD_FP32 && precision != WD_FP64) return fail(WD_ERR_INVALID_ARG, "bad precision");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    for (int l = 0; l < desc->ndim; ++l) widths[l] = pick_tile(ctx, *desc, l, precision == WD_FP64);
    return WD_OK;
}

int wd_tune_set(wd_ctx *ctx, const wd_grid_desc *desc, int precision, const int *widths)
{
    if (!ctx || !desc || !widths) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    int rc = check_desc(desc);
    if (rc) return rc;
    if (precision != WD_FP32 && precision != WD_FP64) return fail(WD_ERR_INVALID_ARG, "bad precision");
    const wd_grid_desc &d = *desc;
    const long long N = npoints(d);
    for (int l = 0; l < d.ndim; ++l) {
        const long long w = widths[l];
        const long long cap = l == 0 ? N / d.n[0] : d.n[0];
        if (w < 1 || w > cap || w * d.n[l] > kTileMax)
            return fail(WD_ERR_INVALID_ARG, "tile width %lld out of range for direction %d", w, l);
    }
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    for (int l = 0; l < d.ndim; ++l)
        ctx->tune[TuneKey{d.ndim, d.n[0], d.n[1], d.n[2], l, precision == WD_FP64}] = widths[l];
    return WD_OK;
}

int wd_ctx_profile(wd_ctx *ctx, int enable)
{
    if (!ctx) return fail(WD_ERR_INVALID_ARG, "null context");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipStreamSynchronize(ctx->stream);
    prof_collect(ctx);
    ctx->kstats.clear();
    ctx->profile = enable ? 1 : 0;
    return WD_OK;
}

int wd_ctx_profile_read(wd_ctx *ctx, wd_kernel_stat *out, int cap, int *n)
{
    if (!ctx || (cap > 0 && !out)) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipStreamSynchronize(ctx->stream);
    prof_collect(ctx);
    int k = 0;
    for (auto &kv : ctx->kstats) {
        if (k < cap) {
            std::memset(&out[k], 0, sizeof out[k]);
            std::snprintf(out[k].name, sizeof out[k].name, "%s", kv.first.c_str());
            out[k].launches = kv.second.launches;
            out[k].total_ms = kv.second.ms;
            out[k].alg_bytes = kv.second.bytes;
        }
        ++k;
    }
    if (n) *n = k;
    return WD_OK;
}

int wd_line_solve_host(int kind, int n, int periodic, int scheme, double alpha_f, int fp64,
                       const double *rhs, double *x, int *nlev)
{
    if (!rhs || !x || n < 8 || n > kMaxLine || (kind != OP_DERIV && kind != OP_FILTER) ||
        scheme < WD_E2 || scheme > WD_C6)
        return fail(WD_ERR_INVALID_ARG, "bad arguments");
    std::vector<double> d(rhs, rhs + n);
    const bool solve = kind == OP_FILTER || scheme == WD_C4 || scheme == WD_C6;
    int lev = 0;
    if (solve) {
        std::vector<int> smod;
        std::vector<double> left, right, scale;
        lev = build_line_system(kind, n, periodic, scheme, alpha_f, fp64, smod, left, right, scale);
        if (lev < 0) return fail(WD_ERR_UNSUPPORTED, "line system did not reduce");
        auto rnd = [fp64](double v) { return fp64 ? v : (double)(float)v; };
        for (int k = 0; k < lev; ++k) {
            const int s = smod[k];
            std::vector<double> nx(n);
            for (int i = 0; i < n; ++i) {
                int im = i - s, ip = i + s;
                if (periodic) {
                    im += im < 0 ? n : 0;
                    ip -= ip >= n ? n : 0;
                } else {
                    im = std::max(im, 0);
                    ip = std::min(ip, n - 1);
                }
                nx[i] = d[i] + rnd(left[(size_t)k * n + i]) * d[im] + rnd(right[(size_t)k * n + i]) * d[ip];
            }
            d.swap(nx);
        }
        for (int i = 0; i < n; ++i) d[i] *= rnd(scale[i]);
    }
    for (int i = 0; i < n; ++i) x[i] = d[i];
    if (nlev) *nlev = lev;
    return WD_OK;
}

int wd_seg_solve_host(int kind, int n, int periodic, int scheme, double alpha_f, int M,
                      const double *rhs, double *x, int *S_used)
{
    if (!rhs || !x || n < 8 || n > kMaxLine || (kind != OP_DERIV && kind != OP_FILTER) ||
        scheme < WD_E2 || scheme > WD_C6)
        return fail(WD_ERR_INVALID_ARG, "bad arguments");
    SegGeo sg;
    if (!seg_plan(n, 0, sg, M) || (M != 0 && M != sg.M))
        return fail(WD_ERR_UNSUPPORTED, "no segmentation of a %d-point line", n);
    if (S_used) *S_used = sg.S * 100 + sg.M;
    const bool solve = kind == OP_FILTER || scheme == WD_C4 || scheme == WD_C6;
    std::vector<double> r(rhs, rhs + n);
    if (!solve) {
        for (int i = 0; i < n; ++i) x[i] = r[i];
        return WD_OK;
    }
    std::vector<double> t;
    if (build_seg_tables(kind, n, periodic, scheme, alpha_f, sg, t))
        return fail(WD_ERR_UNSUPPORTED, "segmented line system (n=%d) is singular", n);
    const int S = sg.S;
    const double *ell = &t[0], *ib = &t[n], *cb = &t[2 * (size_t)n];
    const double *vv = &t[3 * (size_t)n], *ww = &t[4 * (size_t)n], *red = &t[5 * (size_t)n];
    std::vector<double> xl(n), f0(S), l0(S);
    for (int s = 0; s < S; ++s) {
        int bs, len;
        seg_bounds(sg, s, bs, len);
        const int es = bs + len;
        double y = 0.0;
        for (int j = bs; j < es; ++j) {
            y = r[j] - ell[j] * y;
            xl[j] = y;
        }
        double v = 0.0;
        for (int j = es - 1; j >= bs; --j) {
            v = ib[j] * xl[j] - cb[j] * v;
            xl[j] = v;
        }
        f0[s] = xl[bs];
        l0[s] = xl[es - 1];
    }
    for (int s = 0; s < S; ++s) {
        int bs, len;
        seg_bounds(sg, s, bs, len);
        const double *rs = red + (size_t)s * 4 * S;
        double lp = 0.0, fn = 0.0;
        for (int k = 0; k < S; ++k) {
            lp += rs[k] * f0[k] + rs[S + k] * l0[k];
            fn += rs[2 * S + k] * f0[k] + rs[3 * S + k] * l0[k];
        }
        for (int j = bs; j < bs + len; ++j) x[j] = xl[j] - vv[j] * lp - ww[j] * fn;
    }
    return WD_OK;
}

int wd_ctx_set_segmented(wd_ctx *ctx, int enable)
{
    if (!ctx) return fail(WD_ERR_INVALID_ARG, "null context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->use_seg = enable;
    return WD_OK;
}

int wd_ctx_set_explicit_onepass(wd_ctx *ctx, int enable)
{
    if (!ctx) return fail(WD_ERR_INVALID_ARG, "null context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->use_xstage = enable ? 1 : 0;
    return WD_OK;
}

int wd_ctx_set_lad_tiles(wd_ctx *ctx, int enable)
{
    if (!ctx) return fail(WD_ERR_INVALID_ARG, "null context");
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    ctx->use_xlad = enable ? 1 : 0;
    return WD_OK;
}

int wd_poisson_distance(wd_ctx *ctx, const wd_grid_desc *desc, int scheme, int precision,
                        const void *phip, void *dist, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx || !desc || !phip || !dist) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    wd_method m;
    wd_method_default(&m);
    m.equation = WD_EQ_POISSON;
    m.scheme = scheme;
    m.precision = precision;
    m.filter = 0;
    int rc = check_desc(desc);
    if (!rc) rc = check_method(&m);
    if (rc) return rc;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    StreamJoin join(ctx, stream);
    hipStream_t s = ctx->stream;
    void *phis[1] = {dist};
    Plan P;
    rc = plan_batch(ctx, 1, desc, &m, phis, ws, ws_bytes, P);
    if (rc) return rc;
    rc = upload_plan(ctx, P, s);
    if (rc) return rc;
    const size_t S = precision == WD_FP64 ? 8 : 4;
    if (dist != phip &&
        hipMemcpyAsync(dist, phip, (size_t)P.grids[0].N * S, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(WD_ERR_HIP, "copy failed");
    const GridDev &g = P.grids[0];
    if (!g.uniform)   // no initial pass here: the point-major metrics directly
        launch_met_points(P.fp64, g.met_src, const_cast<void *>(g.met), g.N, g.ndim * g.ndim, s);
    return poisson_convert(ctx, P, 0, nullptr, s);
}

// ---------------------------------------------------------------------
// Level-set burnback (Sec. 5.5).  The march borrows a solve plan of the
// grid for its buffers (stage values in ps and P[0], the RK4 accumulator)
// and its pointwise work items; the length partials sit after the plan.

static wd_method levelset_method(int precision)
{
    wd_method m;
    wd_method_default(&m);
    m.equation = WD_EQ_EIKONAL;
    m.scheme = WD_UW;
    m.filter = 0;
    m.rk = WD_RK4;
    m.precision = precision;
    return m;
}

// the solve plan that lends the march its buffers: no mask, wall faces
// (the march's own kernels give every non-periodic face a zero gradient)
static wd_grid_desc levelset_desc(const wd_grid_desc *desc)
{
    wd_grid_desc d = *desc;
    d.mask = nullptr;
    for (int l = 0; l < d.ndim; ++l)
        if (d.bc[l][0] != WD_BC_PERIODIC) d.bc[l][0] = d.bc[l][1] = WD_BC_WALL;
    return d;
}

static int levelset_check(const wd_grid_desc *desc, int precision)
{
    int rc = check_desc(desc);
    if (rc) return rc;
    if (desc->metric_mode != WD_METRIC_UNIFORM)
        return fail(WD_ERR_UNSUPPORTED, "the level-set march takes uniform grids");
    if (precision != WD_FP32 && precision != WD_FP64)
        return fail(WD_ERR_INVALID_ARG, "precision must be WD_FP32 or WD_FP64");
    return WD_OK;
}

static size_t levelset_part_blocks() { return 1024; }

int wd_levelset_workspace_bytes(wd_ctx *ctx, const wd_grid_desc *desc, int precision,
                                size_t *bytes)
{
    if (!ctx || !bytes) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    int rc = levelset_check(desc, precision);
    if (rc) return rc;
    wd_grid_desc d = levelset_desc(desc);
    wd_method m = levelset_method(precision);
    size_t b = 0;
    rc = wd_workspace_bytes(ctx, 1, &d, &m, &b);
    if (rc) return rc;
    *bytes = b + levelset_part_blocks() * kMaxLevels * sizeof(double) + 256;
    return WD_OK;
}

int wd_levelset_advance(wd_ctx *ctx, const wd_grid_desc *desc, int precision, double speed,
                        double dt, int nsteps, void *phi_s, void *ws, size_t ws_bytes,
                        void *stream)
{
    if (!ctx || !phi_s || nsteps < 0) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    if (!(std::fabs(speed * dt) < 1e300)) return fail(WD_ERR_INVALID_ARG, "speed * dt is not finite");
    int rc = levelset_check(desc, precision);
    if (rc) return rc;
    if (nsteps == 0) return WD_OK;
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    StreamJoin join(ctx, stream);
    hipStream_t s = ctx->stream;
    wd_grid_desc d = levelset_desc(desc);
    wd_method m = levelset_method(precision);
    void *phis[1] = {phi_s};
    Plan P;
    rc = plan_batch(ctx, 1, &d, &m, phis, ws, ws_bytes, P);
    if (rc) return rc;
    rc = upload_plan(ctx, P, s);
    if (rc) return rc;
    // the initial pass's list holds tiles 0 .. nchunks-1 of the grid, in
    // order: a stage launch takes the first ceil(N / chunk) of them, a face
    // launch the first ceil(face points / kChunk)
    const ItemList &L = P.lists[P.init];
    const GridDev &g = P.grids[0];
    const Item *items = P.d_items + L.first;
    const int nwg = std::max(8, ctx->cus * (P.fp64 ? 2 : 4));
    const double fdt = speed * dt;
    // large grids: 4096-point work items (more loads in flight per thread)
    // while there are still 8 per compute unit; else 1024-point ones
    const int chunk = g.N >= 8LL * ctx->cus * kLsChunk ? kLsChunk : kChunk;
    // the row-walking stage kernel (falls back to the work-item one when
    // its launch grid would not fit)
    const int n2 = g.ndim == 3 ? g.n[2] : 1;
    // and both directions' faces in one launch (none when both are periodic)
    const bool faces2d = g.ndim == 2 && g.n[0] >= 4 && g.n[1] >= 4 &&
                         !(g.periodic[0] && g.periodic[1]);
    auto one_step = [&]() {
        for (int st = 0; st < 4; ++st) {
            if (launch_ls_stage_rows(P.fp64, P.d_grids, g.n[0], g.n[1], n2, st, fdt, s))
                launch_ls_stage(P.fp64, P.d_grids, items, (int)((g.N + chunk - 1) / chunk), st,
                                fdt, chunk, nwg, s);
            if (faces2d) {
                launch_ls_face2d(P.fp64, P.d_grids, g.n[0], g.n[1], st, s);
                continue;
            }
            for (int l = 0; l < g.ndim; ++l) {
                if (g.periodic[l]) continue;
                const int nf = (int)((g.N / g.n[l] + kChunk - 1) / kChunk);
                launch_ls_face(P.fp64, P.d_grids, items, nf, l, st, nwg, s);
            }
        }
    };
    // several steps: one step's launches captured in a graph and replayed
    hipGraphExec_t exec = nullptr;
    if (nsteps >= 4 && !ctx->profile) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) == hipSuccess) {
            one_step();
            if (hipStreamEndCapture(s, &graph) == hipSuccess && graph) {
                if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                    exec = nullptr;
                (void)hipGraphDestroy(graph);
            }
        }
        (void)hipGetLastError();
    }
    for (int it = 0; it < nsteps; ++it) {
        if (exec) {
            if (hipGraphLaunch(exec, s) != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return fail(WD_ERR_HIP, "hipGraphLaunch failed");
            }
        } else {
            one_step();
        }
    }
    if (exec) {
        // the executable graph is released once its replays have run
        const hipError_t e = hipStreamSynchronize(s);
        (void)hipGraphExecDestroy(exec);
        if (e != hipSuccess) return fail(WD_ERR_HIP, "level-set march failed");
    }
    if (hipGetLastError() != hipSuccess) return fail(WD_ERR_HIP, "level-set launch failed");
    return WD_OK;
}

int wd_level_lengths(wd_ctx *ctx, const wd_grid_desc *desc, int precision, const void *phi_s,
                     const double *levels, int nlevels, double *lengths, void *ws,
                     size_t ws_bytes, void *stream)
{
    if (!ctx || !phi_s || !levels || !lengths || !ws)
        return fail(WD_ERR_INVALID_ARG, "bad arguments");
    int rc = levelset_check(desc, precision);
    if (rc) return rc;
    if (desc->ndim != 2) return fail(WD_ERR_UNSUPPORTED, "iso-line lengths are 2D");
    if (nlevels < 1 || nlevels > kMaxLevels)
        return fail(WD_ERR_INVALID_ARG, "nlevels must be 1..%d", kMaxLevels);
    const size_t nb = levelset_part_blocks();
    const size_t need = nb * kMaxLevels * sizeof(double);
    if (ws_bytes < need) return fail(WD_ERR_INVALID_ARG, "workspace too small");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    hipStream_t s = ctx->stream;
    std::vector<double> part(nb * kMaxLevels);
    {
        StreamJoin join(ctx, stream);
        launch_ls_length(precision == WD_FP64, phi_s, desc->n[0], desc->n[1], desc->h[0],
                         desc->h[1], levels, nlevels, static_cast<double *>(ws), (int)nb, s);
        if (hipMemcpyAsync(part.data(), ws, need, hipMemcpyDeviceToHost, s) != hipSuccess)
            return fail(WD_ERR_HIP, "length partials copy failed");
    }
    if (hipStreamSynchronize(s) != hipSuccess) return fail(WD_ERR_HIP, "length pass failed");
    for (int k = 0; k < nlevels; ++k) {
        double t = 0.0;
        for (size_t b = 0; b < nb; ++b) t += part[b * kMaxLevels + k];
        lengths[k] = t;
    }
    return WD_OK;
}

int wd_signed_distance(wd_ctx *ctx, long long n, int precision, const unsigned char *solid,
                       const void *d_solid, const void *d_gas, void *phi_s, void *stream)
{
    if (!ctx || !solid || !d_solid || !d_gas || !phi_s || n < 0)
        return fail(WD_ERR_INVALID_ARG, "bad arguments");
    if (precision != WD_FP32 && precision != WD_FP64)
        return fail(WD_ERR_INVALID_ARG, "precision must be WD_FP32 or WD_FP64");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    (void)hipSetDevice(ctx->device);
    StreamJoin join(ctx, stream);
    launch_ls_signed(precision == WD_FP64, n, solid, d_solid, d_gas, phi_s, ctx->stream);
    if (hipGetLastError() != hipSuccess) return fail(WD_ERR_HIP, "signed-distance launch failed");
    return WD_OK;
}

}  // extern "C"
