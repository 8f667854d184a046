// pms_serve.cpp -- continuous-batching request engine.
//
// pms_submit copies a request into a waiting queue. An engine thread owned
// by the context admits waiting requests, first come first served, while a
// slot and device memory (a sub-allocation of one pool, sized for the
// request's index, tile arrays and output) are free. Admitted requests are
// indexed on the device and then advance together: every launch of the
// tiled kernel drains a work list that holds a slice of tiles from every
// admitted request, sized so that one launch is short. Requests that arrive
// meanwhile join at a later launch; a request whose tiles are all done is
// compacted into its ascending motif set, copied out, and leaves, freeing
// its slot and memory. No kernel waits on host-written memory: each launch
// ends when its work list is drained.
//
// Two launches are in flight: while launch k runs, the engine keeps
// admitting requests; shortly before k's predicted end it plans launch k+1
// (its work list in the other of two buffers) and queues it behind k on the
// same stream, then waits for k. The requests whose last tiles ran in k are
// compacted and copied out on a second stream while k+1 runs, so the device
// does not idle through the host's work between launches, and a request
// that arrives during a launch still joins the next one.
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

// default device time aimed at per launch: shorter launches finish the
// smallest requests sooner, longer ones cost less per launch (a work list
// copy, a counter fill, a kernel's ramp-up and tail)
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
    int n = 0, m = 0, l = 0, d = 0, s = 0, surv_t = 0, tpb = 0;
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

// One launch of the tile kernel that the engine has queued.
struct Launch {
    bool queued = false;
    std::vector<Req *> last;   // requests whose last tiles are in it
    double planned = 0;        // its planned work (cost model units)
};

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
    WorkItem *d_items[2] = {nullptr, nullptr};   // per launch buffer
    unsigned int *d_next[2] = {nullptr, nullptr};
    TileStats *d_stats = nullptr;
    size_t max_items = 0;
    WorkItem *h_items[2] = {nullptr, nullptr};   // pinned
    InstDev *h_desc = nullptr;       // pinned
    unsigned long long *h_small = nullptr;   // pinned
    int *h_order = nullptr;          // pinned
    hipStream_t st = nullptr;        // index kernels and launches
    hipStream_t st_out = nullptr;    // compaction and copies of results
    hipEvent_t e0[2] = {nullptr, nullptr}, e1[2] = {nullptr, nullptr};
    Launch L[2];
    double ops_per_ms = 5.0e9;       // refined from measured launches
    pms_serve_stats stats{};
    std::string err;

    int start();
    void run();
    int setup(Req *r);
    int plan_launch(int b, const std::vector<Req *> &act);
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
    const size_t items_bytes = align_up(sizeof(WorkItem) * max_items);
    const size_t o_next = o_items + 2 * items_bytes;
    const size_t o_stats = o_next + 2 * 256;
    const size_t ctl = o_stats + align_up(sizeof(TileStats));
    if (hipMalloc(&ctl_mem, ctl) != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(PMS_ENOMEM, "serving control allocation failed");
    }
    c->held += ctl;
    d_slots = (InstDev *)ctl_mem;
    for (int b = 0; b < 2; b++) {
        d_items[b] = (WorkItem *)((char *)ctl_mem + o_items + b * items_bytes);
        d_next[b] = (unsigned int *)((char *)ctl_mem + o_next + b * 256);
    }
    d_stats = (TileStats *)((char *)ctl_mem + o_stats);
    if (hipHostMalloc((void **)&h_items[0], sizeof(WorkItem) * max_items) !=
            hipSuccess ||
        hipHostMalloc((void **)&h_items[1], sizeof(WorkItem) * max_items) !=
            hipSuccess ||
        hipHostMalloc((void **)&h_desc, sizeof(InstDev) * max_slots) !=
            hipSuccess ||
        hipHostMalloc((void **)&h_small, 8 * 3 * (size_t)max_slots + 64) !=
            hipSuccess ||
        hipHostMalloc((void **)&h_order, 4 * kMaxOrder * (size_t)max_slots) !=
            hipSuccess)
        return c->fail(PMS_EDEVICE, "serving pinned staging failed");
    // both streams at the default priority
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&st_out, hipStreamNonBlocking) !=
            hipSuccess)
        return c->fail(PMS_EDEVICE, "serving streams failed");
    for (int b = 0; b < 2; b++)
        if (hipEventCreate(&e0[b]) != hipSuccess ||
            hipEventCreate(&e1[b]) != hipSuccess)
            return c->fail(PMS_EDEVICE, "serving events failed");
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
// Their last launch has completed; the work runs on st_out, beside the
// launch that is running on st.
int Server::finalize(std::vector<Req *> &fin)
{
    for (size_t i = 0; i < fin.size(); i++) {
        Req *r = fin[i];
        char *base = (char *)pool_mem + r->pool_off;
        uint64_t *tile_pos = (uint64_t *)(base + r->lay.tile_pos);
        uint64_t *out = (uint64_t *)(base + r->lay.out);
        if (launch_scan_u32(r->desc.tile_cnt, r->ntiles, tile_pos,
                            base + r->lay.scan, st_out) != hipSuccess ||
            launch_gather(r->desc.tile_cnt, r->desc.tile_heap_off, tile_pos,
                          r->desc.heap, r->ntiles, out, r->heap_cap,
                          r->heap_cap, st_out) != hipSuccess ||
            hipMemcpyAsync(h_small + 3 * i, tile_pos + r->ntiles, 8,
                           hipMemcpyDeviceToHost, st_out) != hipSuccess ||
            hipMemcpyAsync(h_small + 3 * i + 1, r->desc.heap_top, 8,
                           hipMemcpyDeviceToHost, st_out) != hipSuccess ||
            hipMemcpyAsync(h_small + 3 * i + 2, r->desc.bad, 8,
                           hipMemcpyDeviceToHost, st_out) != hipSuccess)
            return PMS_EDEVICE;
    }
    if (hipStreamSynchronize(st_out) != hipSuccess)
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
                           hipMemcpyDeviceToHost, st_out) != hipSuccess)
            return PMS_EDEVICE;
        r->status = PMS_OK;
    }
    if (hipStreamSynchronize(st_out) != hipSuccess)
        return PMS_EDEVICE;
    return PMS_OK;
}

// Plan launch buffer b: a slice of every admitted request's remaining
// tiles, sized by processor sharing, queued on st behind whatever runs.
// Requests whose last tiles go into it are noted in L[b].last.
int Server::plan_launch(int b, const std::vector<Req *> &act)
{
    Launch &Lb = L[b];
    Lb.last.clear();
    Lb.planned = 0;
    Lb.queued = false;
    const double budget = launch_ms * ops_per_ms;
    size_t nleft = 0;
    for (Req *r : act)
        nleft += r->next_tile < r->ntiles;
    if (nleft == 0)
        return PMS_OK;
    const double share = budget / (double)nleft;
    size_t ni = 0;
    double planned_wide = 0;
    WorkItem *hi = h_items[b];
    for (Req *r : act) {
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
            hi[ni++] = w;
            t = w.t1;
        }
        const uint64_t took = t - r->next_tile;
        r->next_tile = t;
        Lb.planned += (double)took * r->cost_per_tile;
        if (r->tpb ? r->tpb == 512 : r->s >= kWideMinSuffix)
            planned_wide += (double)took * r->cost_per_tile;
        if (r->next_tile >= r->ntiles)
            Lb.last.push_back(r);
    }
    if (ni == 0)
        return PMS_OK;
    // the 512-thread tile kernel when most of this launch's work wants it
    // (tuned so, or untuned with tiles of at least 4^8 codes)
    const bool wide = pick_wide(c, planned_wide >= 0.5 * Lb.planned);
    const int tbpc = wide ? c->tiled_wide_bpc : c->tiled_bpc;
    if (hipMemcpyAsync(d_items[b], hi, sizeof(WorkItem) * ni,
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_fill_u32(d_next[b], 1, 0, st) != hipSuccess ||
        hipEventRecord(e0[b], st) != hipSuccess ||
        launch_tiled(d_slots, d_items[b], (int)ni, 0, d_next[b], c->tb,
                     nullptr, std::max(1, c->n_cu * tbpc), st,
                     wide) != hipSuccess ||
        hipEventRecord(e1[b], st) != hipSuccess)
        return PMS_EDEVICE;
    Lb.queued = true;
    return PMS_OK;
}

void Server::run()
{
    hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(mu);
    int b = 0;   // launch buffer to plan next; b ^ 1 may be in flight
    // predicted end of the launch in flight (steady clock, ms): the next
    // launch is queued shortly before it, so that requests arriving until
    // then still join the next launch
    double inflight_end = 0;
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
        const int pb = b ^ 1;
        if (active.empty() && !L[pb].queued) {
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

        // ---- not yet time to queue the next launch: admit more ----------
        if (rc == PMS_OK && L[pb].queued) {
            const double margin = std::max(0.5, 0.25 * launch_ms);
            const hipError_t q = hipEventQuery(e1[pb]);
            (void)hipGetLastError();   // "not ready" is no error here
            const double wait = inflight_end - margin - now_ms();
            if (q == hipErrorNotReady && wait > 0.05) {
                lk.lock();
                cv.wait_for(lk, std::chrono::microseconds(
                                    (long long)(std::min(wait, 0.25) * 1e3)));
                continue;
            }
        }

        // ---- queue launch b behind the one in flight --------------------
        const double t_queue = now_ms();
        if (rc == PMS_OK)
            rc = plan_launch(b, act);
        double b_end = 0;
        if (L[b].queued)
            b_end = (L[pb].queued ? std::max(t_queue, inflight_end)
                                  : t_queue) +
                    L[b].planned / ops_per_ms;

        // ---- wait for the launch in flight, finish its requests ---------
        std::vector<Req *> fin;
        double kms = 0;
        if (rc == PMS_OK && L[pb].queued) {
            if (hipEventSynchronize(e1[pb]) != hipSuccess) {
                rc = PMS_EDEVICE;
            } else {
                float ms = 0;
                if (hipEventElapsedTime(&ms, e0[pb], e1[pb]) == hipSuccess) {
                    kms = ms;
                    if (ms > 0.05)
                        ops_per_ms = 0.7 * ops_per_ms +
                                     0.3 * (L[pb].planned / ms);
                }
                fin = L[pb].last;
                if (!fin.empty())
                    rc = finalize(fin);
            }
            L[pb].queued = false;
            L[pb].last.clear();
            // launch b started when pb ended
            if (L[b].queued)
                b_end = now_ms() + L[b].planned / ops_per_ms;
        } else if (rc == PMS_OK && !L[b].queued && !fresh.empty()) {
            // nothing to launch yet: let the new requests' index kernels
            // finish before they are planned
            if (hipStreamSynchronize(st) != hipSuccess)
                rc = PMS_EDEVICE;
        }
        inflight_end = b_end;

        lk.lock();
        if (kms > 0) {
            stats.launches++;
            stats.busy_ms += kms;
        }
        if (rc != PMS_OK) {
            // device failure: fail every admitted request
            err = "serving engine: HIP error";
            hipStreamSynchronize(st);
            hipStreamSynchronize(st_out);
            L[0] = Launch();
            L[1] = Launch();
            fin = active;
            for (Req *r : fin)
                r->status = PMS_EDEVICE;
        }
        for (Req *r : fin) {
            pool.give(r->pool_off, r->pool_bytes);
            free_slots.push_back(r->slot);
            active.erase(std::find(active.begin(), active.end(), r));
            if (r->status == PMS_PENDING) {
                // overflowed heap: queue again, at the head, with room
                stats.retries++;
                r->lay = layout_instance(r->n, r->m, r->l, r->ntiles,
                                         r->heap_cap, true, true, true);
                r->pool_bytes = r->lay.total;
                r->next_tile = 0;
                r->state = 0;
                r->status = PMS_OK;
                queue.push_front(r);
                continue;
            }
            r->state = 2;
            r->t_done = now_ms();
            stats.completed++;
        }
        if (!fin.empty())
            done_cv.notify_all();
        b ^= 1;
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
    if (s->st_out)
        hipStreamSynchronize(s->st_out);
    if (s->pool_mem) {
        hipFree(s->pool_mem);
        c->held -= s->pool_bytes;
    }
    if (s->ctl_mem)
        hipFree(s->ctl_mem);
    for (int b = 0; b < 2; b++)
        if (s->h_items[b])
            hipHostFree(s->h_items[b]);
    if (s->h_desc)
        hipHostFree(s->h_desc);
    if (s->h_small)
        hipHostFree(s->h_small);
    if (s->h_order)
        hipHostFree(s->h_order);
    for (int b = 0; b < 2; b++) {
        if (s->e0[b])
            hipEventDestroy(s->e0[b]);
        if (s->e1[b])
            hipEventDestroy(s->e1[b]);
    }
    if (s->st)
        hipStreamDestroy(s->st);
    if (s->st_out)
        hipStreamDestroy(s->st_out);
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
    if (in->q != 0 && in->q != in->n)
        return c->fail(PMS_EINVAL, "serving runs plain (l,d) requests (q=%d "
                       "of n=%d); use pms_solve_quorum or pms_solve_batch",
                       in->q, in->n);
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
    r->tpb = P.tpb;
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
