// wd_host.h -- host-side internals of the wall-distance library.
#pragma once

#include "../../include/wd.h"
#include "wd_common.h"
#include "wd_kernels.h"

#include <list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

namespace wd {

enum { OP_DERIV = 0, OP_FILTER = 1 };
enum { SCHEME_E2 = 0, SCHEME_E4 = 1, SCHEME_E6 = 2, SCHEME_C4 = 3, SCHEME_C6 = 4 };

struct OpKey {
    int kind, n, periodic, scheme, fp64;
    double alpha;
    bool operator<(const OpKey &o) const
    {
        return std::tie(kind, n, periodic, scheme, fp64, alpha) <
               std::tie(o.kind, o.n, o.periodic, o.scheme, o.fp64, o.alpha);
    }
};

struct OpEntry {
    LineOpDev dev;
    void *mem = nullptr;
};

struct SegEntry {
    SegOpDev dev;
    void *mem = nullptr;
};

struct TuneKey {
    int ndim, n0, n1, n2, dir, fp64;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(ndim, n0, n1, n2, dir, fp64) <
               std::tie(o.ndim, o.n0, o.n1, o.n2, o.dir, o.fp64);
    }
};

// Device memory for the line-operator tables of one call that must not
// allocate: carved from a caller-provided region, filled by stream-ordered
// copies whose host sources live here until the call ends.
struct TableArena {
    unsigned char *base = nullptr;
    size_t cap = 0, used = 0;
    hipStream_t stream = nullptr;
    std::list<std::vector<unsigned char>> host;
    std::list<std::pair<OpKey, OpEntry>> ops;
    std::list<std::pair<OpKey, SegEntry>> segops;
    void *carve(size_t bytes)
    {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off + bytes > cap) return nullptr;
        used = off + bytes;
        return base + off;
    }
};

struct PendingLaunch;
struct CachedGraph {
    int K = 0;
    int profile = 0;
    hipGraphExec_t exec = nullptr;
    std::vector<hipEvent_t> ev;          // event pairs captured per launch
    std::vector<std::string> ev_name;
    std::vector<double> ev_bytes;
    GridDev *d_grids = nullptr;
    Item *d_items = nullptr;
    std::vector<unsigned char> grids_bytes, items_bytes;
    unsigned long long stamp = 0;
};

struct ItemList {
    int kind, l, arg, np, first, count;
};

// one line pass: its lists per tile variant (np = 1, 2, 4, 8), -1 if none
struct Slot {
    int list[4] = {-1, -1, -1, -1};
};

// live kernel timing (profiling mode): one record per launch
struct KStat {
    long long launches = 0;
    double ms = 0.0;
    double bytes = 0.0;    // algorithmic (compulsory) bytes
};
struct PendingLaunch {
    hipEvent_t a, b;
    std::string name;
    double bytes;
};

struct GridHost {
    void *pois_phip = nullptr;   // FP64 phi' (Poisson grids)
    void *pois_F[3] = {nullptr, nullptr, nullptr};
    bool init = true;            // issue the initial field for this grid
};

struct Plan {
    int n = 0, fp64 = 0, rk = 1, stages = 4, maxdim = 0;
    std::vector<GridDev> grids;
    std::vector<GridHost> host;
    long long items_cap = 0;
    std::vector<Item> items;
    std::vector<ItemList> lists;
    Slot cart[3], d1[3], d1n[3], d12, d2[3], filt[3], lad0[3], lad1[3];   // d1n: stages > 0
    Slot scart[3], scartl[3], sfilt[3], slad0[3], slad1[3];  // segmented passes, one list per M
    int face[6], face_init[6];
    int fin = 0, resid = 0, init = 0, uwadv = 0, cfin = 0;
    int xstage[3][2] = {};       // one-pass explicit stages per scheme radius:
                                 // general and fast tiles
    int xlad[2] = {0, 0};        // two-pass LAD field: sensor, smoothing
    std::vector<char> live;      // grids the work lists cover (empty: all of
                                 // them); a solve drops grids that stopped
    TableArena *arena = nullptr;   // line-operator tables of a call that allocates nothing
    GridDev *d_grids = nullptr;
    GridDev *d_aux = nullptr, *d_aux2 = nullptr;
    GridState *d_states = nullptr;
    Item *d_items = nullptr;
};

int fail(int code, const char *fmt, ...);
extern thread_local std::string g_last_error;

int check_desc(const wd_grid_desc *d);
int check_walls(const wd_grid_desc *d);
int check_method(const wd_method *m);
int grid_mode(const wd_grid_desc &d, const wd_method &m);
size_t batch_bytes(int n, const wd_grid_desc *d, const wd_method *m);
int pick_tile(wd_ctx *ctx, const wd_grid_desc &d, int l, int fp64);
int pcr_reduce(int n, int periodic, std::vector<double> a, std::vector<double> b,
               std::vector<double> c, double tol, std::vector<int> &smod,
               std::vector<double> &left, std::vector<double> &right,
               std::vector<double> &scale);
int build_line_system(int kind, int n, int periodic, int scheme, double af, int fp64,
                      std::vector<int> &smod, std::vector<double> &left,
                      std::vector<double> &right, std::vector<double> &scale);
bool seg_plan(int n, int fp64, SegGeo &sg, int prefer = 0);
int build_seg_tables(int kind, int n, int periodic, int scheme, double af, const SegGeo &sg,
                     std::vector<double> &out);
const SegOpDev *ctx_segop(wd_ctx *ctx, int kind, int n, int periodic, int scheme, double af,
                          int fp64, const SegGeo &sg, TableArena *ar = nullptr);
size_t seg_lds_bytes(const GridDev &g, int kind, int l, int fp64);
const LineOpDev *ctx_lineop(wd_ctx *ctx, int kind, int n, int periodic, int scheme,
                            double af, int fp64, TableArena *ar = nullptr);
size_t grid_region_bytes(const wd_grid_desc &d, const wd_method &m);
long long grid_items(const wd_grid_desc &d);
size_t table_bytes(int n, long long items);
int layout_grid(wd_ctx *ctx, const wd_grid_desc &d, const wd_method &m, void *phi,
                void *region, GridDev &g, GridHost &h, TableArena *ar = nullptr);
int plan_tables(Plan &P, void *tables, size_t bytes, long long items_cap);
int plan_batch(wd_ctx *ctx, int n, const wd_grid_desc *descs, const wd_method *meths,
               void *const *phis, void *ws, size_t ws_bytes, Plan &P, TableArena *ar = nullptr);
int tile_np(const GridDev &g, int l);
void build_items(Plan &P);
int upload_plan(wd_ctx *ctx, const Plan &P, hipStream_t s);
void issue_init(wd_ctx *ctx, const Plan &P, hipStream_t s);
void issue_iteration(wd_ctx *ctx, const Plan &P, hipStream_t s);
CachedGraph *graph_for(wd_ctx *ctx, const Plan &P, int K);
void prof_collect(wd_ctx *ctx);
void ctx_drop_graphs(wd_ctx *ctx);
int run_plan(wd_ctx *ctx, Plan &P, int K, std::vector<GridState> &states);
int poisson_convert(wd_ctx *ctx, const Plan &P, int i, void *aux, hipStream_t s);
int solve_plan(wd_ctx *ctx, Plan &P, void *const *aux, double *const *hists, int hist_cap,
               int *iters, int *status);

}  // namespace wd

struct wd_ctx {
    int device = 0;
    int cus = 256;
    char arch[64] = {0};
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    wd::GridState *pinned_states = nullptr;
    int pinned_cap = 0;
    int use_graphs = 1;
    int graph_iters = 32;
    std::map<wd::OpKey, wd::OpEntry> ops;
    std::map<wd::OpKey, wd::SegEntry> segops;
    void *noalloc = nullptr;             // the device's static scratch (calls that allocate nothing)
    size_t noalloc_bytes = 0;
    int use_seg = 1;                     // segmented passes on Cartesian grids
                                         // (16, 24, 32: segment length tried first)
    int seg_split_finish = 1;            // 1: a pointwise pass finishes their stages
    int use_xstage = 1;                  // explicit schemes on Cartesian grids: one
    int use_xlad = 1;                    // Cartesian LAD grids: the field in two tile passes
                                         // pointwise pass per RK stage
    std::map<wd::TuneKey, int> tune;
    std::vector<wd::CachedGraph> graphs;
    int profile = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<wd::PendingLaunch> pending;
    std::map<std::string, wd::KStat> kstats;
    unsigned long long clock = 0;
    std::recursive_mutex mu;
};
