// wd_server.cpp -- continuous-batching request loop behind wd_server_*.
//
// A host thread owns a context (its own stream), a device arena of the
// caller's budget and the batch tables.  Each request's footprint is its
// grid region (fields, partial sums, history, stopping state).  Between
// rounds of K pseudo iterations the thread retires grids that stopped,
// admits queued requests (small grids first; larger ones smallest first,
// long waiters first, within a point budget) while a slot is free and their
// region fits in the arena, and re-plans the batch; a grid joining a
// running batch starts at its own iteration 0 and every grid keeps its own
// state, so results do not depend on what else is running.
#include "wd_host.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

namespace wd {

static double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static size_t al256s(size_t x) { return (x + 255) & ~(size_t)255; }

static long long grid_points(const wd_grid_desc &d)
{
    long long N = 1;
    for (int l = 0; l < d.ndim; ++l) N *= d.n[l];
    return N;
}

// first-fit allocator over one device allocation, coalescing on release
struct Arena {
    size_t size = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void reset(size_t n)
    {
        size = n;
        used = peak = 0;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(size_t n, size_t &off)
    {
        n = al256s(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rem = it->second - n;
            free_.erase(it);
            if (rem) free_[off + n] = rem;
            used += n;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = al256s(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Req {
    long long id = 0;
    wd_grid_desc desc;
    wd_method meth;
    void *phi = nullptr;
    long long session = -1;
    int hist_cap = 0;
    int status = WD_PENDING;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int iters = 0;
    int spent = 0;                     // iterations of an abandoned warm attempt
    std::vector<double> hist;
    size_t bytes = 0, off = 0;
    bool running = false, cancel = false, finished = false, fresh = false;
    GridDev g;
    GridHost h;
};

}  // namespace wd

struct wd_server {
    wd_ctx *ctx = nullptr;            // the server's own context and stream
    size_t budget = 0;
    int max_slots = 0;
    void *arena_mem = nullptr;
    wd::Arena arena;
    void *tables = nullptr;
    size_t tables_bytes = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<long long> queue;
    std::map<long long, wd::Req> reqs;
    std::map<long long, std::deque<long long>> sessions;
    std::vector<long long> active;
    long long next_id = 1;
    bool stop = false;
    int error = 0;
    std::thread th;
    long long n_done = 0, n_iters = 0, n_restarts = 0;
    int peak_active = 0;
    int round_iters = 16;
    long long point_budget = 8LL << 20;   // grid points iterated together
    double age_s = 30.0;                  // waiting longer than this: first
    std::vector<long long> last_set;
};

namespace wd {

static void finish_locked(wd_server *srv, Req &r, int status)
{
    r.status = status;
    r.finished = true;
    r.running = false;
    r.t_done = now_s();
    if (r.session >= 0) {
        auto &q = srv->sessions[r.session];
        for (auto it = q.begin(); it != q.end(); ++it)
            if (*it == r.id) {
                q.erase(it);
                break;
            }
        if (q.empty()) srv->sessions.erase(r.session);
    }
    ++srv->n_done;
    srv->cv_done.notify_all();
}

static bool session_head(wd_server *srv, const Req &r)
{
    if (r.session < 0) return true;
    auto it = srv->sessions.find(r.session);
    return it == srv->sessions.end() || it->second.empty() || it->second.front() == r.id;
}

// admission under the lock: arrival order, a free slot, room in the arena
// Admission: cancelled requests leave the queue; then, while a slot is
// free and the arena has room, requests join the running set.  Small ones
// (at most 1/16 of the point budget) go first, smallest first, and do not
// count against the budget: they cost little per iteration and finish
// quickly.  Among the larger ones, any that has waited longer than age_s
// goes first (in arrival order), otherwise the smallest, as long as the
// larger grids iterated together stay within point_budget (a lone request
// always runs).  A session's requests run in submission order.
static void admit_locked(wd_server *srv)
{
    for (auto it = srv->queue.begin(); it != srv->queue.end();) {
        Req &r = srv->reqs[*it];
        if (r.cancel) {
            finish_locked(srv, r, WD_ERR_CANCELLED);
            it = srv->queue.erase(it);
            continue;
        }
        if (r.bytes > srv->arena.size) {
            finish_locked(srv, r, WD_ERR_NO_MEMORY);
            it = srv->queue.erase(it);
            continue;
        }
        ++it;
    }
    const long long small = std::max(1LL, srv->point_budget / 16);
    long long big_pts = 0;
    for (long long id : srv->active) {
        const long long n = grid_points(srv->reqs[id].desc);
        if (n > small) big_pts += n;
    }
    const double t = now_s();
    while ((int)srv->active.size() < srv->max_slots && !srv->queue.empty()) {
        auto pick_small = srv->queue.end(), pick_aged = srv->queue.end(),
             pick_big = srv->queue.end();
        long long best_small = -1, best_big = -1;
        for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it) {
            Req &r = srv->reqs[*it];
            if (!session_head(srv, r)) continue;
            const long long pts = grid_points(r.desc);
            if (pts <= small) {
                if (best_small < 0 || pts < best_small) {
                    best_small = pts;
                    pick_small = it;
                }
            } else if (t - r.t_submit > srv->age_s) {
                if (pick_aged == srv->queue.end()) pick_aged = it;   // the earliest
            } else if (best_big < 0 || pts < best_big) {
                best_big = pts;
                pick_big = it;
            }
        }
        auto pick = pick_small;
        if (pick == srv->queue.end()) {
            pick = pick_aged != srv->queue.end() ? pick_aged : pick_big;
            if (pick == srv->queue.end()) break;
            const long long pts = grid_points(srv->reqs[*pick].desc);
            if (!srv->active.empty() && big_pts + pts > srv->point_budget) break;
        }
        Req &r = srv->reqs[*pick];
        const long long pts = grid_points(r.desc);
        size_t off = 0;
        if (!srv->arena.alloc(r.bytes, off)) break;   // wait for memory
        r.off = off;
        int rc = layout_grid(srv->ctx, r.desc, r.meth, r.phi,
                             static_cast<unsigned char *>(srv->arena_mem) + off, r.g, r.h);
        if (rc) {
            srv->arena.release(off, r.bytes);
            finish_locked(srv, r, rc);
            srv->queue.erase(pick);
            continue;
        }
        r.running = true;
        r.fresh = true;
        r.t_admit = now_s();
        srv->active.push_back(r.id);
        if (pts > small) big_pts += pts;
        srv->peak_active = std::max(srv->peak_active, (int)srv->active.size());
        srv->queue.erase(pick);
    }
}

// one round for the grids of one (precision, rk) group
static int run_group(wd_server *srv, const std::vector<long long> &ids, bool same_set)
{
    wd_ctx *ctx = srv->ctx;
    hipStream_t s = ctx->stream;
    Plan P;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        const Req &r0 = srv->reqs[ids[0]];
        P.fp64 = r0.meth.precision == WD_FP64;
        P.rk = r0.meth.rk;
        P.stages = P.rk == WD_RK4 ? 4 : 3;
        for (long long id : ids) {
            Req &r = srv->reqs[id];
            GridHost h = r.h;
            h.init = r.fresh;
            P.grids.push_back(r.g);
            P.host.push_back(h);
        }
    }
    long long items = 0;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (long long id : ids) items += grid_items(srv->reqs[id].desc);
    }
    const size_t tb = table_bytes((int)ids.size(), items);
    if (tb > srv->tables_bytes) {
        if (srv->tables) (void)hipFree(srv->tables);
        srv->tables = nullptr;
        srv->tables_bytes = 0;
        if (hipMalloc(&srv->tables, tb * 2) != hipSuccess)
            return fail(WD_ERR_NO_MEMORY, "server tables allocation failed");
        srv->tables_bytes = tb * 2;
        same_set = false;
    }
    int rc = plan_tables(P, srv->tables, srv->tables_bytes, items);
    if (rc) return rc;
    rc = upload_plan(ctx, P, s);
    if (rc) return rc;
    launch_mirror(P.d_grids, P.n, s);
    issue_init(ctx, P, s);
    // a set unchanged since the last round replays the graph of its K
    // iterations (captured in relaxed mode, so the clients' runtime calls go
    // on meanwhile; cached by the plan's contents); a new set launches
    // directly, since it may last a single round
    const int K = srv->round_iters;
    CachedGraph *cg = nullptr;
    if (same_set && ctx->use_graphs && !ctx->profile) cg = graph_for(ctx, P, K);
    if (cg) {
        if (hipGraphLaunch(cg->exec, s) != hipSuccess)
            return fail(WD_ERR_HIP, "server round graph launch failed");
    } else {
        for (int k = 0; k < K; ++k) issue_iteration(ctx, P, s);
    }
    if (hipMemcpyAsync(ctx->pinned_states, P.d_states, P.n * sizeof(GridState),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(WD_ERR_HIP, "server round failed: %s", hipGetErrorString(hipGetLastError()));
    std::vector<GridState> st(ctx->pinned_states, ctx->pinned_states + P.n);
    // retire grids that stopped (or were cancelled)
    for (int i = 0; i < P.n; ++i) {
        bool cancel;
        int hist_cap;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            Req &r = srv->reqs[ids[i]];
            r.fresh = false;
            r.iters = r.spent + st[i].iter;
            cancel = r.cancel;
            hist_cap = r.hist_cap;
            if (st[i].done && !cancel && st[i].status == WD_ERR_WARM_RUNAWAY) {
                // the runaway check stopped a warm start: solve it again
                // from zero in the same slot (the next round initialises it)
                r.spent += st[i].iter;
                r.g.warm = 0;
                r.g.warm_probe = 0;
                r.meth.warm_start = 0;
                r.fresh = true;
                ++srv->n_restarts;
                continue;
            }
        }
        if (!st[i].done && !cancel) continue;
        int status = cancel && !st[i].done ? WD_ERR_CANCELLED : st[i].status;
        if (!cancel && P.grids[i].eq == 2) {
            int r2 = poisson_convert(ctx, P, i, nullptr, s);
            if (r2) status = r2;
        }
        std::vector<double> h;
        const int nh = std::min(std::min(st[i].iter, hist_cap), P.grids[i].hist_cap);
        if (nh > 0) {
            h.resize((size_t)nh * 2);
            if (hipMemcpy(h.data(), P.grids[i].hist, (size_t)nh * 16, hipMemcpyDeviceToHost) != hipSuccess)
                status = WD_ERR_HIP;
        }
        std::lock_guard<std::mutex> lk(srv->mu);
        Req &r = srv->reqs[ids[i]];
        r.hist.swap(h);
        srv->arena.release(r.off, r.bytes);
        srv->active.erase(std::find(srv->active.begin(), srv->active.end(), r.id));
        finish_locked(srv, r, status);
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->n_iters += K;
    }
    return WD_OK;
}

static void server_loop(wd_server *srv)
{
    (void)hipSetDevice(srv->ctx->device);
    for (;;) {
        std::vector<long long> ids;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            admit_locked(srv);
            if (srv->active.empty()) {
                if (srv->stop) break;
                srv->cv_work.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
            if (srv->stop) {
                for (long long id : srv->active) {
                    Req &r = srv->reqs[id];
                    srv->arena.release(r.off, r.bytes);
                    finish_locked(srv, r, WD_ERR_CANCELLED);
                }
                srv->active.clear();
                break;
            }
            ids = srv->active;
        }
        // group by (precision, rk)
        std::map<std::pair<int, int>, std::vector<long long>> groups;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            for (long long id : ids) {
                const Req &r = srv->reqs[id];
                groups[{r.meth.precision, r.meth.rk}].push_back(id);
            }
        }
        const bool same = ids == srv->last_set && groups.size() == 1;
        srv->last_set = ids;
        for (auto &kv : groups) {
            int rc = run_group(srv, kv.second, same);
            if (rc) {
                std::lock_guard<std::mutex> lk(srv->mu);
                srv->error = rc;
                for (long long id : kv.second) {
                    Req &r = srv->reqs[id];
                    if (r.finished) continue;
                    srv->arena.release(r.off, r.bytes);
                    srv->active.erase(std::find(srv->active.begin(), srv->active.end(), id));
                    finish_locked(srv, r, rc);
                }
            }
        }
    }
}

}  // namespace wd

using namespace wd;

extern "C" {

int wd_server_create(wd_ctx *ctx, size_t budget_bytes, int max_slots, wd_server **out)
{
    if (!ctx || !out || max_slots < 1 || budget_bytes < 4096)
        return fail(WD_ERR_INVALID_ARG, "bad arguments");
    *out = nullptr;
    wd_server *srv = new wd_server();
    int rc = wd_ctx_create(ctx->device, &srv->ctx);
    if (rc) {
        delete srv;
        return rc;
    }
    srv->budget = budget_bytes;
    srv->max_slots = std::min(max_slots, 4000);
    if (hipMalloc(&srv->arena_mem, budget_bytes) != hipSuccess) {
        wd_ctx_destroy(srv->ctx);
        delete srv;
        return fail(WD_ERR_NO_MEMORY, "arena of %zu bytes could not be allocated", budget_bytes);
    }
    srv->arena.reset(budget_bytes);
    const char *k = std::getenv("WD_SERVER_ROUND");
    if (k) srv->round_iters = std::max(1, std::atoi(k));
    const char *pb = std::getenv("WD_SERVER_POINTS");
    if (pb) srv->point_budget = std::max(1LL, std::atoll(pb));
    const char *ag = std::getenv("WD_SERVER_AGE");
    if (ag) srv->age_s = std::max(0.0, std::atof(ag));
    srv->th = std::thread(server_loop, srv);
    *out = srv;
    return WD_OK;
}

int wd_server_submit(wd_server *srv, const wd_grid_desc *desc, const wd_method *method, void *phi,
                     long long session, int hist_cap, long long *req_id)
{
    if (!srv || !desc || !method || !phi || !req_id || hist_cap < 0)
        return fail(WD_ERR_INVALID_ARG, "bad arguments");
    int rc = check_desc(desc);
    if (!rc) rc = check_walls(desc);
    if (!rc) rc = check_method(method);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(WD_ERR_INVALID_ARG, "server is shutting down");
    if (srv->error) return fail(srv->error, "server stopped after an error");
    Req r;
    r.id = srv->next_id++;
    r.desc = *desc;
    r.meth = *method;
    r.phi = phi;
    r.session = session;
    r.hist_cap = hist_cap;
    r.t_submit = now_s();
    r.bytes = grid_region_bytes(*desc, *method);
    if (session >= 0) srv->sessions[session].push_back(r.id);
    srv->reqs[r.id] = r;
    srv->queue.push_back(r.id);
    *req_id = r.id;
    srv->cv_work.notify_one();
    return WD_OK;
}

int wd_server_poll(wd_server *srv, long long req_id, int *status, double *t_submit, double *t_admit,
                   double *t_done, int *iters)
{
    if (!srv) return fail(WD_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return fail(WD_ERR_NOT_FOUND, "no request %lld", req_id);
    const Req &r = it->second;
    if (status) *status = r.finished ? r.status : WD_PENDING;
    if (t_submit) *t_submit = r.t_submit;
    if (t_admit) *t_admit = r.t_admit;
    if (t_done) *t_done = r.t_done;
    if (iters) *iters = r.iters;
    return WD_OK;
}

int wd_server_wait(wd_server *srv, long long req_id, double timeout_s)
{
    if (!srv) return fail(WD_ERR_INVALID_ARG, "null server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return fail(WD_ERR_NOT_FOUND, "no request %lld", req_id);
    auto pred = [&] { return srv->reqs[req_id].finished; };
    if (timeout_s < 0)
        srv->cv_done.wait(lk, pred);
    else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
        return WD_PENDING;
    return srv->reqs[req_id].status;
}

int wd_server_history(wd_server *srv, long long req_id, double *hist, int cap, int *n)
{
    if (!srv || (cap > 0 && !hist)) return fail(WD_ERR_INVALID_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return fail(WD_ERR_NOT_FOUND, "no request %lld", req_id);
    const Req &r = it->second;
    if (!r.finished) return fail(WD_PENDING, "request %lld is not finished", req_id);
    const int m = std::min(cap, (int)(r.hist.size() / 2));
    if (m > 0) std::memcpy(hist, r.hist.data(), (size_t)m * 16);
    if (n) *n = m;
    return WD_OK;
}

int wd_server_cancel(wd_server *srv, long long req_id)
{
    if (!srv) return fail(WD_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(req_id);
    if (it == srv->reqs.end()) return fail(WD_ERR_NOT_FOUND, "no request %lld", req_id);
    it->second.cancel = true;
    srv->cv_work.notify_one();
    return WD_OK;
}

int wd_server_stats(wd_server *srv, long long *done, long long *iterations, size_t *peak_bytes,
                    int *peak_active, long long *restarts)
{
    if (!srv) return fail(WD_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (restarts) *restarts = srv->n_restarts;
    if (done) *done = srv->n_done;
    if (iterations) *iterations = srv->n_iters;
    if (peak_bytes) *peak_bytes = srv->arena.peak;
    if (peak_active) *peak_active = srv->peak_active;
    return WD_OK;
}

int wd_server_destroy(wd_server *srv)
{
    if (!srv) return WD_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        for (long long id : srv->queue) {
            Req &r = srv->reqs[id];
            if (!r.finished) finish_locked(srv, r, WD_ERR_CANCELLED);
        }
        srv->queue.clear();
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable()) srv->th.join();
    (void)hipSetDevice(srv->ctx->device);
    if (srv->tables) (void)hipFree(srv->tables);
    if (srv->arena_mem) (void)hipFree(srv->arena_mem);
    wd_ctx_destroy(srv->ctx);
    delete srv;
    return WD_OK;
}

}  // extern "C"
