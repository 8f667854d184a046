// pms_batch.cpp -- many independent instances in one persistent launch.
//
// Every instance of a batch is indexed, then all their tiles go into one
// work list that a single launch of the tiled kernel drains (instances of
// different (l, d, n, m) mix freely: l, d, n, m and the tile shape are
// per-instance values in the descriptors). The tile-count arrays of all
// instances are laid end to end, so one scan and one ordered gather give
// every instance its ascending motif set in one output array. The device
// part (fills, index, tiled kernel, scan, gather, ranges) is captured once
// as a HIP graph and replayed while the batch shape stays the same; only the
// input bytes are copied in per call.
#include "pms_host.h"

#include <algorithm>
#include <cstring>

using namespace pms;

namespace {

struct Member {
    int idx;
    int n, m, l, d, s, surv_t, tpb;
    uint64_t ntiles, tile_base;
    double cost;
    InstLayout lay;
    size_t arena_off, seq_off;
};

uint64_t batch_shape_key(const std::vector<Member> &mem)
{
    uint64_t key = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
    mix(mem.size());
    for (auto &b : mem) {
        mix(b.n);
        mix(b.m);
        mix(b.l);
        mix(b.d);
    }
    return key;
}

}  // namespace

namespace pms {

int batch_core(pms_ctx *c, const pms_instance *in, int k, pms_result *out)
{
    const double t0 = now_ms();
    hipStream_t st = c->stream;
    std::vector<Member> mem;
    std::vector<int> solo;
    int first_bad = PMS_OK;
    for (int i = 0; i < k; i++) {
        out[i].motifs = nullptr;
        out[i].count = 0;
        out[i].status = PMS_OK;
        const pms_instance &x = in[i];
        int rc = x.seqs ? check_shape(x.n, x.m, x.l, x.d) : PMS_EINVAL;
        if (!rc && (x.q < 0 || x.q > x.n))
            rc = PMS_EINVAL;
        if (rc) {
            out[i].status = rc;
            if (!first_bad)
                first_bad = rc;
            continue;
        }
        // quorum instances run one by one on their own kernels
        if (x.q > 0 && x.q < x.n) {
            solo.push_back(i);
            continue;
        }
        Plan P = c->plan(x.n, x.m, x.l, x.d, PMS_PATH_AUTO);
        if (P.path != PMS_PATH_TILED) {
            solo.push_back(i);
            continue;
        }
        Member b{};
        b.idx = i;
        b.n = x.n;
        b.m = x.m;
        b.l = x.l;
        b.d = x.d;
        b.s = P.s;
        b.surv_t = P.surv_t;
        b.tpb = P.tpb;
        b.ntiles = P.ntiles;
        b.cost = P.cost_tiled;
        mem.push_back(b);
    }
    const int ninst = (int)mem.size();
    pms_stats S{};
    S.path = PMS_PATH_TILED;
    uint64_t heap_cap = 0;
    for (auto &b : mem)
        heap_cap += std::max<uint64_t>(256, b.ntiles / 16);
    heap_cap = std::max<uint64_t>(heap_cap, 1 << 16);
    // a batch of the same shape needed this much last time: start there, so
    // that repeated batches run once and keep their captured graph
    if (c->b_heap_key == batch_shape_key(mem))
        heap_cap = std::max<uint64_t>(heap_cap, c->b_heap_need);
    c->b_host.clear();

    for (int attempt = 0; attempt < 5 && ninst > 0; attempt++) {
        // ---- layout -------------------------------------------------------
        size_t seq_bytes = 0, off = 0;
        uint64_t tile_total = 0;
        for (auto &b : mem) {
            b.seq_off = seq_bytes;
            seq_bytes += align_up((size_t)b.n * b.m, 64);
        }
        off = align_up(seq_bytes);
        for (auto &b : mem) {
            b.lay = layout_instance(b.n, b.m, b.l, b.ntiles, 0, false, false,
                                    false);
            b.arena_off = off;
            off += align_up(b.lay.total);
            b.tile_base = tile_total;
            tile_total += b.ntiles;
        }
        // work items: chunks of tiles sized so that one item costs about
        // 1/8 of a persistent workgroup's share, most expensive first (a
        // long item at the end would leave the rest of the chip idle)
        double total_cost = 0, wide_cost = 0;
        for (auto &b : mem) {
            total_cost += b.cost;
            if (b.tpb ? b.tpb == 512 : b.s >= kWideMinSuffix)
                wide_cost += b.cost;
        }
        // the 512-thread tile kernel when most of the work is in instances
        // that want it: tuned so, or untuned with tiles of at least 4^8
        // codes (faster there, slower on smaller tiles)
        const bool wide = pick_wide(c, wide_cost >= 0.5 * total_cost);
        const int tbpc = wide ? c->tiled_wide_bpc : c->tiled_bpc;
        const double slots = (double)std::max(1, c->n_cu * tbpc);
        const double target = total_cost / (slots * 8.0);
        std::vector<WorkItem> items;
        std::vector<double> icost;
        for (int j = 0; j < ninst; j++) {
            const Member &b = mem[j];
            const double per_tile = b.cost / (double)b.ntiles;
            const uint64_t chunk = std::min<uint64_t>(
                64, std::max<uint64_t>(1, (uint64_t)(target / per_tile)));
            for (uint64_t t = 0; t < b.ntiles; t += chunk) {
                WorkItem w;
                w.inst = j;
                w.pad = 0;
                w.t0 = t;
                w.t1 = std::min(t + chunk, b.ntiles);
                items.push_back(w);
                icost.push_back(b.cost * (double)(w.t1 - w.t0) /
                                (double)b.ntiles);
            }
        }
        std::vector<size_t> ord(items.size());
        for (size_t i = 0; i < ord.size(); i++)
            ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) {
            return icost[a] > icost[b];
        });
        std::vector<WorkItem> witems(items.size());
        for (size_t i = 0; i < ord.size(); i++)
            witems[i] = items[ord[i]];

        const size_t o_desc = off;
        const size_t o_items = o_desc + align_up(sizeof(InstDev) * ninst);
        const size_t o_next = o_items + align_up(sizeof(WorkItem) *
                                                 witems.size());
        const size_t o_stats = o_next + 256;
        const size_t o_cnt = o_stats + align_up(sizeof(TileStats));
        const size_t o_hoff = o_cnt + align_up(tile_total * 4);
        const size_t o_pos = o_hoff + align_up(tile_total * 8);
        const size_t o_scan = o_pos + align_up((tile_total + 1) * 8);
        const size_t o_top = o_scan + align_up(scan_scratch_bytes(tile_total));
        const size_t o_bad = o_top + 256;
        const size_t o_ranges = o_bad + align_up(8 * (size_t)ninst);
        const size_t o_order = o_ranges + align_up(16 * (size_t)ninst);
        size_t order_words = 0;
        for (auto &b : mem)
            order_words += b.n;
        const size_t o_heap = o_order + align_up(order_words * 4);
        const size_t o_out = o_heap + align_up(heap_cap * 8);
        const size_t need = o_out + align_up(heap_cap * 8);
        int rc = c->alloc(c->b_arena, need);
        if (rc)
            return rc;
        char *base = (char *)c->b_arena.p;

        std::vector<InstDev> descs(ninst);
        {
            size_t ow = 0;
            for (int j = 0; j < ninst; j++) {
                Member &b = mem[j];
                InstDev I = make_desc(base + b.arena_off, b.lay,
                                      (const uint8_t *)(base + b.seq_off),
                                      b.n, b.m, b.l, b.d, b.s, b.surv_t,
                                      b.ntiles, heap_cap);
                I.order = (const int *)(base + o_order) + ow;
                ow += b.n;
                I.bad = (unsigned long long *)(base + o_bad) + j;
                I.tile_cnt = (uint32_t *)(base + o_cnt) + b.tile_base;
                I.tile_heap_off = (uint64_t *)(base + o_hoff) + b.tile_base;
                I.heap = (uint64_t *)(base + o_heap);
                I.heap_top = (unsigned long long *)(base + o_top);
                I.tile_base = b.tile_base;
                descs[j] = I;
            }
        }
        // ---- pinned staging: inputs | descs | items | orders | results ---
        const size_t s_desc = align_up(seq_bytes);
        const size_t s_items = s_desc + align_up(sizeof(InstDev) * ninst);
        const size_t s_order = s_items + align_up(sizeof(WorkItem) *
                                                  witems.size());
        const size_t s_res = s_order + align_up(order_words * 4);
        const size_t stage = s_res + align_up(8 * (size_t)(3 * ninst + 2));
        if (c->b_pinned_bytes < stage) {
            if (c->b_pinned)
                hipHostFree(c->b_pinned);
            c->b_pinned = nullptr;
            c->b_pinned_bytes = 0;
            HIPCHK(c, hipHostMalloc((void **)&c->b_pinned, stage));
            c->b_pinned_bytes = stage;
        }
        char *P = c->b_pinned;
        for (auto &b : mem)
            memcpy(P + b.seq_off, in[b.idx].seqs, (size_t)b.n * b.m);

        uint64_t key = 1469598103934665603ull;
        auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
        mix((uint64_t)(uintptr_t)base);
        mix(c->b_arena.bytes);
        mix(heap_cap);
        mix(ninst);
        for (auto &b : mem) {
            mix(b.n);
            mix(b.m);
            mix(b.l);
            mix(b.d);
            mix(b.s);
            mix(b.surv_t);
        }
        InstDev *d_desc = (InstDev *)(base + o_desc);
        WorkItem *d_items = (WorkItem *)(base + o_items);
        uint64_t *tile_pos = (uint64_t *)(base + o_pos);
        uint64_t *ranges = (uint64_t *)(base + o_ranges);
        TileStats *d_stats = (TileStats *)(base + o_stats);
        uint64_t *d_out = (uint64_t *)(base + o_out);

        HIPCHK(c, hipEventRecord(c->ev[0], st));
        HIPCHK(c, hipMemcpyAsync(base, P, seq_bytes, hipMemcpyHostToDevice,
                                 st));
        const bool replay = key == c->b_graph_key && c->b_graph;
        if (!replay) {
            if (c->b_graph) {
                hipGraphExecDestroy(c->b_graph);
                hipGraphDestroy(c->b_graph_def);
                c->b_graph = nullptr;
                c->b_graph_def = nullptr;
                c->b_graph_key = 0;
            }
            memcpy(P + s_desc, descs.data(), sizeof(InstDev) * ninst);
            memcpy(P + s_items, witems.data(), sizeof(WorkItem) * witems.size());
            {
                int *o = (int *)(P + s_order);
                for (auto &b : mem)
                    for (int i = 0; i < b.n; i++)
                        *o++ = i;
            }
            HIPCHK(c, hipMemcpyAsync(d_desc, P + s_desc,
                                     sizeof(InstDev) * ninst,
                                     hipMemcpyHostToDevice, st));
            HIPCHK(c, hipMemcpyAsync(d_items, P + s_items,
                                     sizeof(WorkItem) * witems.size(),
                                     hipMemcpyHostToDevice, st));
            HIPCHK(c, hipMemcpyAsync(base + o_order, P + s_order,
                                     order_words * 4, hipMemcpyHostToDevice,
                                     st));
            HIPCHK(c, hipStreamSynchronize(st));
            int max_rw = 0, max_lm = 0;
            for (auto &I : descs) {
                max_rw = std::max(max_rw, I.n * I.wpr);
                max_lm = std::max(max_lm, I.n * I.L);
            }
            HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            hipError_t ce = launch_fill_u64(
                (unsigned long long *)(base + o_bad), ninst, ~0ull, st);
            if (ce == hipSuccess)
                ce = launch_fill_u64((unsigned long long *)(base + o_top), 1,
                                     0, st);
            if (ce == hipSuccess)
                ce = launch_fill_u64((unsigned long long *)(base + o_next), 1,
                                     0, st);
            if (ce == hipSuccess)
                ce = launch_fill_u64((unsigned long long *)d_stats,
                                     sizeof(TileStats) / 8, 0, st);
            if (ce == hipSuccess)
                ce = launch_index(d_desc, ninst, max_rw, max_lm, st);
            if (ce == hipSuccess)
                ce = launch_tiled(d_desc, d_items, (int)witems.size(), 0,
                                  (unsigned int *)(base + o_next), c->tb,
                                  d_stats, std::max(1, c->n_cu * tbpc), st,
                                  wide);
            if (ce == hipSuccess)
                ce = launch_scan_u32((uint32_t *)(base + o_cnt), tile_total,
                                     tile_pos, base + o_scan, st);
            if (ce == hipSuccess)
                ce = launch_gather((uint32_t *)(base + o_cnt),
                                   (uint64_t *)(base + o_hoff), tile_pos,
                                   (uint64_t *)(base + o_heap), tile_total,
                                   d_out, heap_cap, heap_cap, st);
            if (ce == hipSuccess)
                ce = launch_ranges(d_desc, ninst, tile_pos, ranges, st);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(st, &g);
            if (ce != hipSuccess || ee != hipSuccess) {
                if (g)
                    hipGraphDestroy(g);
                return c->fail(PMS_EDEVICE, "batch graph capture failed: %s",
                               hipGetErrorString(ce != hipSuccess ? ce : ee));
            }
            hipGraphExec_t ge = nullptr;
            hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                hipGraphDestroy(g);
                return c->fail(PMS_EDEVICE, "hipGraphInstantiate: %s",
                               hipGetErrorString(ie));
            }
            c->b_graph = ge;
            c->b_graph_def = g;
            c->b_graph_key = key;
        } else {
            c->b_graph_replays++;
        }
        HIPCHK(c, hipEventRecord(c->ev[1], st));
        HIPCHK(c, hipGraphLaunch(c->b_graph, st));
        HIPCHK(c, hipEventRecord(c->ev[2], st));
        unsigned long long *R = (unsigned long long *)(P + s_res);
        HIPCHK(c, hipMemcpyAsync(R, ranges, 16 * (size_t)ninst,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(R + 2 * ninst, base + o_bad, 8 * (size_t)ninst,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(R + 3 * ninst, base + o_top, 8,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(R + 3 * ninst + 1, tile_pos + tile_total, 8,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        const unsigned long long top = R[3 * ninst];
        c->b_heap_key = batch_shape_key(mem);
        c->b_heap_need = std::max<uint64_t>(c->b_heap_need, top + top / 8 + 1024);
        if (top > heap_cap) {
            heap_cap = top + top / 8 + 1024;
            S.retries++;
            continue;
        }
        const uint64_t total = R[3 * ninst + 1];
        c->b_host.resize(total);
        if (total) {
            HIPCHK(c, hipMemcpyAsync(c->b_host.data(), d_out, total * 8,
                                     hipMemcpyDeviceToHost, st));
        }
        TileStats ts{};
        HIPCHK(c, hipMemcpyAsync(c->pinned + 8, d_stats, sizeof(ts),
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipEventRecord(c->ev[3], st));
        HIPCHK(c, hipStreamSynchronize(st));
        memcpy(&ts, c->pinned + 8, sizeof(ts));
        for (int j = 0; j < ninst; j++) {
            pms_result &o = out[mem[j].idx];
            if (R[2 * ninst + j] != ~0ull) {
                o.status = PMS_EBASE;
                if (!first_bad) {
                    first_bad = PMS_EBASE;
                    c->fail(PMS_EBASE, "batch instance %d: bad base in string "
                            "%llu at offset %llu", mem[j].idx,
                            R[2 * ninst + j] / mem[j].m,
                            R[2 * ninst + j] % mem[j].m);
                }
                continue;
            }
            o.count = R[2 * j + 1];
            o.motifs = o.count ? c->b_host.data() + R[2 * j] : nullptr;
        }
        float a = 0, b = 0, e = 0;
        hipEventElapsedTime(&a, c->ev[0], c->ev[1]);
        hipEventElapsedTime(&b, c->ev[1], c->ev[2]);
        hipEventElapsedTime(&e, c->ev[2], c->ev[3]);
        S.ms_index = a;
        S.ms_main = b;
        S.ms_output = e;
        S.main_launches = 1;
        S.tiles = ts.tiles;
        S.tile_passes = ts.passes;
        S.marks = ts.marks;
        S.filter_tests = ts.ftests;
        S.tile_threads = wide ? 512 : 256;
        S.graph_replayed = replay ? 1 : 0;
        break;
    }
    // instances the tiled kernel does not suit, and quorum instances, run
    // one by one
    c->b_solo.assign(solo.size(), {});
    for (size_t q = 0; q < solo.size(); q++) {
        const int i = solo[q];
        SolveOut r{};
        const int qi = (in[i].q > 0 && in[i].q < in[i].n) ? in[i].q : 0;
        int rc = solve_core(c, in[i].seqs, nullptr, in[i].n, in[i].m, in[i].l,
                            in[i].d, st, nullptr, 0, PMS_PATH_AUTO, &r, qi);
        if (rc) {
            out[i].status = rc;
            if (!first_bad)
                first_bad = rc;
            continue;
        }
        c->b_solo[q].resize(r.count);
        if (r.count) {
            HIPCHK(c, hipMemcpyAsync(c->b_solo[q].data(), r.d_out, r.count * 8,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
        }
        out[i].count = r.count;
        out[i].motifs = r.count ? c->b_solo[q].data() : nullptr;
    }
    S.ms_total = now_ms() - t0;
    c->last = S;
    return first_bad;
}

}  // namespace pms

extern "C" int pms_solve_batch(pms_ctx *c, const pms_instance *in, int k,
                               pms_result *out)
{
    if (!c)
        return PMS_EINVAL;
    if (k < 0 || (k > 0 && (!in || !out)))
        return c->fail(PMS_EINVAL, "bad batch arguments");
    hipSetDevice(c->device);
    return batch_core(c, in, k, out);
}
