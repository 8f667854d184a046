// pms_serve.cpp -- continuous-batching request engine.
//
// pms_submit copies a request into a waiting queue. An engine thread owned
// by the context admits waiting requests, first come first served, while a
// slot and device memory (a sub-allocation of one pool, sized for the
// request's index, tile arrays and output) are free. Admitted requests are
// indexed on the device and then advance together: every launch of the
// tiled kernel drains a work list that holds a slice of tiles from every
// admitted request, sized so that one launch is short. Requests that arrive
// meanwhile join at the next launch; a request whose tiles are all done is
// compacted into its ascending motif set, copied out, and leaves, freeing
// its slot and memory. No kernel waits on host-written memory: each launch
// ends when its work list is drained.
#include "pms_host.h"

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

using namespace pms;

namespace pms {

namespace {

// default device time aimed at per launch: every launch ends in a host
// synchronisation, so longer launches waste less of the GPU between them
// (at the cost of a longer wait for the smallest requests)
constexpr double kLaunchTargetMs = 16.0;
constexpr int kMaxOrder = 4096;          // strings per request (serving)

// First-fit sub-allocator over one device allocation (host bookkeeping).
struct Pool {
    size_t bytes = 0;
    std::map<size_t, size_t> free_;   // offset -> size
    size_t used = 0;

    void reset(size_t b)
    {
        bytes = b;
        free_.clear();
        free_[0] = b;
        used = 0;
    }
    bool take(size_t want, size_t &off)
    {
        want = align_up(want, 4096);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= want) {
                off = it->first;
                const size_t rest = it->second - want;
                free_.erase(it);
                if (rest)
                    free_[off + want] = rest;
                used += want;
                return true;
            }
        }
        return false;
    }
    void give(size_t off, size_t want)
    {
        want = align_up(want, 4096);
        used -= want;
        auto it = free_.emplace(off, want).first;
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
    uint64_t ticket = 0;
    int n = 0, m = 0, l = 0, d = 0, s = 0, surv_t = 0;
    uint64_t ntiles = 0, next_tile = 0, heap_cap = 0;
    double cost_per_tile = 0;
    std::vector<char> seqs;
    int state = 0;   // 0 waiting, 1 admitted, 2 done
    int status = PMS_OK;
    int slot = -1;
    size_t pool_off = 0, pool_bytes = 0;
    InstLayout lay;
    InstDev desc;
    std::vector<uint64_t> result;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct Server {
    pms_ctx *c = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    bool stop = false;
    std::deque<Req *> queue;
    std::vector<Req *> active;
    std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    int max_slots = 64, max_queue = 4096;
    double launch_ms = kLaunchTargetMs;   // device time aimed at per launch
    std::vector<int> free_slots;
    Pool pool;
    void *pool_mem = nullptr;
    size_t pool_bytes = 0;
    void *ctl_mem = nullptr;   // slots, items, counter, stats
    InstDev *d_slots = nullptr;
    WorkItem *d_items = nullptr;
    unsigned int *d_next = nullptr;
    TileStats *d_stats = nullptr;
    size_t max_items = 0;
    WorkItem *h_items = nullptr;     // pinned
    InstDev *h_desc = nullptr;       // pinned
    unsigned long long *h_small = nullptr;   // pinned
    int *h_order = nullptr;          // pinned
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double ops_per_ms = 5.0e9;       // refined from measured launches
    pms_serve_stats stats{};
    std::string err;

    int start();
    void run();
    int setup(Req *r);
    int finalize(std::vector<Req *> &fin);
};

int Server::start()
{
    hipSetDevice(c->device);
    max_slots = c->opt.serve_slots ? c->opt.serve_slots : 64;
    max_queue = c->opt.serve_queue ? c->opt.serve_queue : 4096;
    launch_ms = c->opt.serve_launch_ms > 0.0 ? c->opt.serve_launch_ms
                                             : kLaunchTargetMs;
    size_t room = c->budget > c->held.load() ? c->budget - c->held.load() : 0;
    pool_bytes = std::min<size_t>(room / 2, (size_t)8 << 30);
    if (pool_bytes < ((size_t)64 << 20))
        return c->fail(PMS_ENOMEM, "serving pool: only %zu bytes of budget "
                       "left", room);
    if (hipMalloc(&pool_mem, pool_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(PMS_ENOMEM, "serving pool allocation failed");
    }
    c->held += pool_bytes;
    pool.reset(pool_bytes);
    max_items = 1 << 16;
    const size_t o_items = align_up(sizeof(InstDev) * max_slots);
    const size_t o_next = o_items + align_up(sizeof(WorkItem) * max_items);
    const size_t o_stats = o_next + 256;
    const size_t ctl = o_stats + align_up(sizeof(TileStats));
    if (hipMalloc(&ctl_mem, ctl) != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(PMS_ENOMEM, "serving control allocation failed");
    }
    c->held += ctl;
    d_slots = (InstDev *)ctl_mem;
    d_items = (WorkItem *)((char *)ctl_mem + o_items);
    d_next = (unsigned int *)((char *)ctl_mem + o_next);
    d_stats = (TileStats *)((char *)ctl_mem + o_stats);
    if (hipHostMalloc((void **)&h_items, sizeof(WorkItem) * max_items) !=
            hipSuccess ||
        hipHostMalloc((void **)&h_desc, sizeof(InstDev) * max_slots) !=
            hipSuccess ||
        hipHostMalloc((void **)&h_small, 8 * 3 * (size_t)max_slots + 64) !=
            hipSuccess ||
        hipHostMalloc((void **)&h_order, 4 * kMaxOrder * (size_t)max_slots) !=
            hipSuccess)
        return c->fail(PMS_EDEVICE, "serving pinned staging failed");
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return c->fail(PMS_EDEVICE, "serving stream/events failed");
    for (int i = max_slots - 1; i >= 0; i--)
        free_slots.push_back(i);
    th = std::thread([this] { run(); });
    return PMS_OK;
}

// Copy a newly admitted request in and index it (engine thread).
int Server::setup(Req *r)
{
    char *base = (char *)pool_mem + r->pool_off;
    r->desc = make_desc(base, r->lay, nullptr, r->n, r->m, r->l, r->d, r->s,
                        r->surv_t, r->ntiles, r->heap_cap);
    InstDev *slot = d_slots + r->slot;
    memcpy(h_desc + r->slot, &r->desc, sizeof(InstDev));
    int *ord = h_order + (size_t)kMaxOrder * r->slot;
    for (int i = 0; i < r->n; i++)
        ord[i] = i;
    // the slot's pinned staging is not reused before this request leaves,
    // so the copies need no wait here; the request's seqs vector lives
    // until release
    if (hipMemcpyAsync((void *)r->desc.seqs, r->seqs.data(),
                       (size_t)r->n * r->m, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync((void *)r->desc.order, ord, 4 * (size_t)r->n,
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(slot, h_desc + r->slot, sizeof(InstDev),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_fill_u64(r->desc.bad, 1, ~0ull, st) != hipSuccess ||
        launch_fill_u64(r->desc.heap_top, 1, 0, st) != hipSuccess ||
        launch_index(slot, 1, r->n * r->desc.wpr, r->n * r->desc.L, st) !=
            hipSuccess)
        return PMS_EDEVICE;
    return PMS_OK;
}

// Compact finished requests and copy their results out (engine thread).
int Server::finalize(std::vector<Req *> &fin)
{
    for (size_t i = 0; i < fin.size(); i++) {
        Req *r = fin[i];
        char *base = (char *)pool_mem + r->pool_off;
        uint64_t *tile_pos = (uint64_t *)(base + r->lay.tile_pos);
        uint64_t *out = (uint64_t *)(base + r->lay.out);
        if (launch_scan_u32(r->desc.tile_cnt, r->ntiles, tile_pos,
                            base + r->lay.scan, st) != hipSuccess ||
            launch_gather(r->desc.tile_cnt, r->desc.tile_heap_off, tile_pos,
                          r->desc.heap, r->ntiles, out, r->heap_cap,
                          r->heap_cap, st) !=
                hipSuccess ||
            hipMemcpyAsync(h_small + 3 * i, tile_pos + r->ntiles, 8,
                           hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(h_small + 3 * i + 1, r->desc.heap_top, 8,
                           hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(h_small + 3 * i + 2, r->desc.bad, 8,
                           hipMemcpyDeviceToHost, st) != hipSuccess)
            return PMS_EDEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess)
        return PMS_EDEVICE;
    for (size_t i = 0; i < fin.size(); i++) {
        Req *r = fin[i];
        const unsigned long long total = h_small[3 * i],
                                 top = h_small[3 * i + 1],
                                 bad = h_small[3 * i + 2];
        if (bad != ~0ull) {
            r->status = PMS_EBASE;
            continue;
        }
        if (top > r->heap_cap) {
            // output heap overflowed: run the request again with room
            r->status = PMS_PENDING;
            r->heap_cap = top + top / 4 + 1024;
            continue;
        }
        char *base = (char *)pool_mem + r->pool_off;
        r->result.resize(total);
        if (total &&
            hipMemcpyAsync(r->result.data(), base + r->lay.out, total * 8,
                           hipMemcpyDeviceToHost, st) != hipSuccess)
            return PMS_EDEVICE;
        r->status = PMS_OK;
    }
    if (hipStreamSynchronize(st) != hipSuccess)
        return PMS_EDEVICE;
    return PMS_OK;
}

void Server::run()
{
    hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // ---- admission: first come first served, by slot and memory ----
        std::vector<Req *> fresh;
        while (!queue.empty() && !free_slots.empty()) {
            Req *r = queue.front();
            size_t off = 0;
            if (!pool.take(r->pool_bytes, off)) {
                if (active.empty() && fresh.empty()) {
                    // cannot fit even alone
                    queue.pop_front();
                    r->status = PMS_ENOMEM;
                    r->state = 2;
                    r->t_done = now_ms();
                    done_cv.notify_all();
                    continue;
                }
                break;
            }
            queue.pop_front();
            r->pool_off = off;
            r->slot = free_slots.back();
            free_slots.pop_back();
            r->state = 1;
            r->t_admit = now_ms();
            fresh.push_back(r);
            active.push_back(r);
        }
        if (active.empty()) {
            if (stop)
                break;
            cv.wait(lk);
            continue;
        }
        stats.max_inflight = std::max<uint64_t>(stats.max_inflight,
                                                active.size());
        std::vector<Req *> act = active;
        lk.unlock();

        int rc = PMS_OK;
        for (Req *r : fresh)
            if (rc == PMS_OK)
                rc = setup(r);

        // ---- one launch: a slice of every admitted request's tiles ------
        const double t0 = now_ms();
        const double budget = launch_ms * ops_per_ms;
        const double share = budget / (double)act.size();
        size_t ni = 0;
        double planned = 0, planned_wide = 0;
        std::vector<uint64_t> took(act.size(), 0);
        for (size_t a = 0; a < act.size() && rc == PMS_OK; a++) {
            Req *r = act[a];
            const uint64_t left = r->ntiles - r->next_tile;
            if (!left)
                continue;
            uint64_t q = (uint64_t)std::max(1.0, share / r->cost_per_tile);
            q = std::min(q, left);
            const uint64_t chunk =
                std::max<uint64_t>(1, std::min<uint64_t>(16, q / 64));
            uint64_t t = r->next_tile;
            const uint64_t end = r->next_tile + q;
            while (t < end && ni < max_items) {
                WorkItem w;
                w.inst = r->slot;
                w.pad = 0;
                w.t0 = t;
                w.t1 = std::min(t + chunk, end);
                h_items[ni++] = w;
                t = w.t1;
            }
            took[a] = t - r->next_tile;
            planned += (double)took[a] * r->cost_per_tile;
            if (r->s >= kWideMinSuffix)
                planned_wide += (double)took[a] * r->cost_per_tile;
        }
        if (rc == PMS_OK && ni > 0) {
            // the 512-thread tile kernel when most of this launch's work is
            // in tiles of at least 4^8 codes
            const bool wide = pick_wide(c, planned_wide >= 0.5 * planned);
            const int tbpc = wide ? c->tiled_wide_bpc : c->tiled_bpc;
            if (hipMemcpyAsync(d_items, h_items, sizeof(WorkItem) * ni,
                               hipMemcpyHostToDevice, st) != hipSuccess ||
                launch_fill_u32(d_next, 1, 0, st) != hipSuccess ||
                hipEventRecord(e0, st) != hipSuccess ||
                launch_tiled(d_slots, d_items, (int)ni, 0, d_next, c->tb,
                             nullptr, std::max(1, c->n_cu * tbpc), st,
                             wide) != hipSuccess ||
                hipEventRecord(e1, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = PMS_EDEVICE;
            float ms = 0;
            if (rc == PMS_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
                ms > 0.05)
                ops_per_ms = 0.7 * ops_per_ms + 0.3 * (planned / ms);
        }
        std::vector<Req *> fin;
        for (size_t a = 0; a < act.size(); a++) {
            act[a]->next_tile += took[a];
            if (act[a]->next_tile >= act[a]->ntiles)
                fin.push_back(act[a]);
        }
        if (rc == PMS_OK && !fin.empty())
            rc = finalize(fin);
        const double t1 = now_ms();

        lk.lock();
        stats.launches++;
        stats.busy_ms += t1 - t0;
        if (rc != PMS_OK) {
            // device failure: fail every admitted request
            err = "serving engine: HIP error";
            fin = active;
            for (Req *r : fin)
                r->status = PMS_EDEVICE;
        }
        for (Req *r : fin) {
            if (r->status == PMS_PENDING) {
                // overflowed heap: give the memory back and queue again
                pool.give(r->pool_off, r->pool_bytes);
                free_slots.push_back(r->slot);
                active.erase(std::find(active.begin(), active.end(), r));
                r->lay = layout_instance(r->n, r->m, r->l, r->ntiles,
                                         r->heap_cap, true, true, true);
                r->pool_bytes = r->lay.total;
                r->next_tile = 0;
                r->state = 0;
                r->status = PMS_OK;
                queue.push_front(r);
                continue;
            }
            pool.give(r->pool_off, r->pool_bytes);
            free_slots.push_back(r->slot);
            active.erase(std::find(active.begin(), active.end(), r));
            r->state = 2;
            r->t_done = now_ms();
            stats.completed++;
        }
        if (!fin.empty())
            done_cv.notify_all();
    }
}

void serve_shutdown(pms_ctx *c)
{
    Server *s = c->srv;
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        // requests still waiting are dropped
        for (Req *r : s->queue) {
            r->state = 2;
            r->status = PMS_EINVAL;
        }
        s->queue.clear();
    }
    s->cv.notify_all();
    if (s->th.joinable())
        s->th.join();
    if (s->st)
        hipStreamSynchronize(s->st);
    if (s->pool_mem) {
        hipFree(s->pool_mem);
        c->held -= s->pool_bytes;
    }
    if (s->ctl_mem)
        hipFree(s->ctl_mem);
    if (s->h_items)
        hipHostFree(s->h_items);
    if (s->h_desc)
        hipHostFree(s->h_desc);
    if (s->h_small)
        hipHostFree(s->h_small);
    if (s->h_order)
        hipHostFree(s->h_order);
    if (s->e0)
        hipEventDestroy(s->e0);
    if (s->e1)
        hipEventDestroy(s->e1);
    if (s->st)
        hipStreamDestroy(s->st);
    delete s;
    c->srv = nullptr;
}

}  // namespace pms

extern "C" {

int pms_submit(pms_ctx *c, const pms_instance *in, uint64_t *ticket)
{
    if (!c)
        return PMS_EINVAL;
    if (!in || !in->seqs || !ticket)
        return c->fail(PMS_EINVAL, "NULL argument");
    int rc = check_shape(in->n, in->m, in->l, in->d);
    if (rc)
        return c->fail(rc, "bad shape n=%d m=%d l=%d d=%d", in->n, in->m,
                       in->l, in->d);
    if (in->n > kMaxOrder)
        return c->fail(PMS_EINVAL, "serving: n=%d above %d", in->n, kMaxOrder);
    Plan P = c->plan(in->n, in->m, in->l, in->d, PMS_PATH_TILED);
    if (P.path != PMS_PATH_TILED)
        return c->fail(PMS_EINVAL, "serving runs the tiled path, which does "
                       "not suit l=%d d=%d; use pms_solve", in->l, in->d);
    if (!c->srv) {
        hipSetDevice(c->device);
        Server *s = new Server();
        s->c = c;
        c->srv = s;
        rc = s->start();
        if (rc) {
            serve_shutdown(c);
            return rc;
        }
    }
    Server *s = c->srv;
    std::unique_ptr<Req> r(new Req());
    r->n = in->n;
    r->m = in->m;
    r->l = in->l;
    r->d = in->d;
    r->s = P.s;
    r->surv_t = P.surv_t;
    r->ntiles = P.ntiles;
    r->cost_per_tile = std::max(1.0, P.cost_tiled / (double)P.ntiles);
    r->heap_cap = std::max<uint64_t>(4096, P.ntiles / 16);
    r->lay = layout_instance(r->n, r->m, r->l, r->ntiles, r->heap_cap, true,
                             true, true);
    r->pool_bytes = r->lay.total;
    if (align_up(r->pool_bytes, 4096) > s->pool_bytes)
        return c->fail(PMS_ENOMEM, "request needs %zu bytes, serving pool "
                       "holds %zu", r->pool_bytes, s->pool_bytes);
    r->seqs.assign(in->seqs, in->seqs + (size_t)in->n * in->m);
    std::lock_guard<std::mutex> g(s->mu);
    if ((int)s->queue.size() >= s->max_queue)
        return c->fail(PMS_EBUSY, "serving queue full (%d waiting)",
                       (int)s->queue.size());
    r->ticket = s->next_ticket++;
    r->t_submit = now_ms();
    *ticket = r->ticket;
    s->queue.push_back(r.get());
    s->reqs[r->ticket] = std::move(r);
    s->stats.submitted++;
    s->cv.notify_all();
    return PMS_OK;
}

static int fill_result(Req *r, pms_result *out)
{
    if (out) {
        out->status = r->status;
        out->count = r->status == PMS_OK ? r->result.size() : 0;
        out->motifs = out->count ? r->result.data() : nullptr;
    }
    return r->status;
}

int pms_poll(pms_ctx *c, uint64_t ticket, pms_result *out)
{
    if (!c || !c->srv)
        return c ? c->fail(PMS_EINVAL, "no request submitted") : PMS_EINVAL;
    Server *s = c->srv;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return c->fail(PMS_EINVAL, "unknown ticket %llu",
                       (unsigned long long)ticket);
    Req *r = it->second.get();
    if (r->state != 2)
        return PMS_PENDING;
    return fill_result(r, out);
}

int pms_wait(pms_ctx *c, uint64_t ticket, int timeout_ms, pms_result *out)
{
    if (!c || !c->srv)
        return c ? c->fail(PMS_EINVAL, "no request submitted") : PMS_EINVAL;
    Server *s = c->srv;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return c->fail(PMS_EINVAL, "unknown ticket %llu",
                       (unsigned long long)ticket);
    Req *r = it->second.get();
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::milliseconds(timeout_ms < 0 ? 0
                                                                : timeout_ms);
    while (r->state != 2) {
        if (timeout_ms >= 0) {
            if (s->done_cv.wait_until(lk, until) == std::cv_status::timeout &&
                r->state != 2)
                return PMS_PENDING;
        } else {
            s->done_cv.wait(lk);
        }
    }
    return fill_result(r, out);
}

int pms_release(pms_ctx *c, uint64_t ticket)
{
    if (!c || !c->srv)
        return c ? c->fail(PMS_EINVAL, "no request submitted") : PMS_EINVAL;
    Server *s = c->srv;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return c->fail(PMS_EINVAL, "unknown ticket %llu",
                       (unsigned long long)ticket);
    if (it->second->state != 2)
        return c->fail(PMS_EINVAL, "ticket %llu still running",
                       (unsigned long long)ticket);
    s->reqs.erase(it);
    return PMS_OK;
}

int pms_ticket_times(pms_ctx *c, uint64_t ticket, double *t_submit,
                     double *t_admit, double *t_done)
{
    if (!c || !c->srv)
        return c ? c->fail(PMS_EINVAL, "no request submitted") : PMS_EINVAL;
    Server *s = c->srv;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return c->fail(PMS_EINVAL, "unknown ticket %llu",
                       (unsigned long long)ticket);
    if (t_submit)
        *t_submit = it->second->t_submit;
    if (t_admit)
        *t_admit = it->second->t_admit;
    if (t_done)
        *t_done = it->second->t_done;
    return PMS_OK;
}

double pms_clock_ms(void) { return now_ms(); }

int pms_serve_stats_get(const pms_ctx *c, pms_serve_stats *out)
{
    if (!c || !out)
        return PMS_EINVAL;
    memset(out, 0, sizeof(*out));
    if (!c->srv)
        return PMS_OK;
    std::lock_guard<std::mutex> g(c->srv->mu);
    *out = c->srv->stats;
    return PMS_OK;
}

}  // extern "C"
