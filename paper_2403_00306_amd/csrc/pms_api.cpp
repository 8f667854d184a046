// pms_api.cpp -- host side of libpms: context, planner, C ABI.
//
// The planner picks, per instance, the sample-driven filter path or the
// tiled pattern-driven path from a cost model (both are exact; the kernel
// files state what each computes), sizes the device buffers, launches the
// kernels on the context's stream and brings the ascending motif set back.
// pms_serve.cpp holds the serving engine, pms_tune.cpp the autotuner.
#include "pms_host.h"
#include "pms_wide.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

using namespace pms;

namespace pms {

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(
               steady_clock::now().time_since_epoch())
        .count();
}

double nb_real(int l, int d)
{
    double t = 0, c = 1;
    for (int k = 0; k <= d && k <= l; k++) {
        if (k > 0)
            c = c * (l - k + 1) / k;
        t += c * std::pow(3.0, k);
    }
    return t;
}

uint64_t nb_exact(int l, int d)
{
    unsigned __int128 t = 0, c = 1, p = 1;
    for (int k = 0; k <= d && k <= l; k++) {
        if (k > 0) {
            c = c * (unsigned)(l - k + 1) / (unsigned)k;
            p *= 3;
        }
        t += c * p;
    }
    return t > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (uint64_t)t;
}

InstLayout layout_instance(int n, int m, int l, uint64_t ntiles,
                           uint64_t heap_cap, bool own_seqs, bool own_tiles,
                           bool own_out)
{
    InstLayout o;
    const int L = m - l + 1;
    const int wpr = (m + 31) / 32;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        size_t at = p;
        p += align_up(bytes ? bytes : 1);
        return at;
    };
    o.seqs = own_seqs ? take((size_t)n * m) : 0;
    o.packed = take((size_t)n * wpr * 8);
    o.phi = take((size_t)n * wpr * 4);
    o.plo = take((size_t)n * wpr * 4);
    o.planes = take((size_t)n * L * 8);
    o.codes = take((size_t)n * L * 8);
    o.order = take((size_t)n * 4);
    o.bad = take(8);
    if (own_tiles) {
        o.tile_cnt = take(ntiles * 4);
        o.tile_heap_off = take(ntiles * 8);
        o.tile_pos = take((ntiles + 1) * 8);
        o.scan = take(scan_scratch_bytes(ntiles));
        o.heap_top = take(8);
        o.heap = take(heap_cap * 8);
    }
    if (own_out)
        o.out = take(heap_cap * 8);
    o.total = p;
    return o;
}

InstDev make_desc(char *base, const InstLayout &o, const uint8_t *seqs,
                  int n, int m, int l, int d, int s, int surv_t,
                  uint64_t ntiles, uint64_t heap_cap)
{
    InstDev I;
    memset(&I, 0, sizeof(I));
    I.seqs = seqs ? seqs : (const uint8_t *)(base + o.seqs);
    I.packed = (uint64_t *)(base + o.packed);
    I.phi = (uint32_t *)(base + o.phi);
    I.plo = (uint32_t *)(base + o.plo);
    I.planes = (uint2 *)(base + o.planes);
    I.codes = (uint64_t *)(base + o.codes);
    I.order = (const int *)(base + o.order);
    I.bad = (unsigned long long *)(base + o.bad);
    if (o.heap_top) {
        I.tile_cnt = (uint32_t *)(base + o.tile_cnt);
        I.tile_heap_off = (uint64_t *)(base + o.tile_heap_off);
        I.heap = (uint64_t *)(base + o.heap);
        I.heap_top = (unsigned long long *)(base + o.heap_top);
    }
    I.heap_cap = heap_cap;
    I.tile_base = 0;
    I.ntiles = ntiles;
    I.n = n;
    I.m = m;
    I.l = l;
    I.d = d;
    I.L = m - l + 1;
    I.s = s;
    I.surv_t = surv_t;
    I.wpr = (m + 31) / 32;
    I.q = n;
    // per-tile string order (tiled path): worth its n*L prefix tests per
    // tile (shared by sibling tiles) where a pass's expected word marks,
    // L * n_B(l-3, d) / 4^(l-s), are above half of them
    if (n <= kOrderMax && s >= 3 && l >= s) {
        const double L = (double)(m - l + 1);
        const double marks = L * nb_real(l - 3, d) / std::pow(4.0, l - s);
        I.tile_order = marks >= 0.5 * (double)n * L ? 1 : 0;
    } else {
        I.tile_order = 0;
    }
    return I;
}

int check_shape(int n, int m, int l, int d)
{
    if (n < 1 || l < 1 || l > kMaxL || m < l || d < 0 || d >= l)
        return PMS_EINVAL;
    if ((double)n * (double)m > 4.0e9)
        return PMS_EINVAL;
    return PMS_OK;
}

// Expected work (VALU lane operations) of the two exact paths.
//  p: probability that a random l-mer lies within d of one of the L l-mers
//     of a string (independent uniform background).
//  filter: every candidate of s_1 meets ~1/(1-p) strings of L l-mers at
//          ~3.5 operations per Hamming test.
//  tiled: every live tile pays L prefix tests and its share of the
//         word-level sphere marks per string; a tile stays live while it
//         still holds codes (Poisson estimate) and switches to the filter
//         once at most surv_t remain.
void cost_model(int n, int m, int l, int d, int s, int surv_t, double &cf,
                double &ct)
{
    const double L = m - l + 1;
    const double nb = nb_real(l, d);
    const double space = std::pow(4.0, l);
    const double p = 1.0 - std::pow(std::max(0.0, 1.0 - nb / space), L);
    const double exam = std::min((double)std::max(n - 1, 0),
                                 1.0 / std::max(1e-9, 1.0 - p));
    cf = L * nb * L * exam * 3.5 + L * nb;
    if (l < 3 || s < 3 || s > l) {
        ct = INFINITY;
        return;
    }
    const double ntiles = std::pow(4.0, l - s);
    const double words_per_y = nb_real(l - 3, d);
    const double per_pass = L * 6.0 + L * words_per_y / ntiles * 12.0 +
                            std::pow(4.0, s - 3) * 4.0 / 64.0 + 400.0;
    double tiles_live = ntiles, total = 0, left = std::pow(4.0, s);
    for (int k = 0; k < n; k++) {
        total += tiles_live * per_pass;
        left *= p;
        if (left <= surv_t) {
            total += ntiles * left * L *
                     std::min(1.0 / (1.0 - p), (double)(n - k - 1)) * 3.5;
            break;
        }
        tiles_live = ntiles * (1.0 - std::exp(-left));
    }
    ct = total;
}

int default_suffix(int l)
{
    // enough tiles to fill the chip, at most 4^9 codes per tile
    int s = l - 5;
    if (s > kMaxSuffix)
        s = kMaxSuffix;
    if (s < kMinSuffix)
        s = kMinSuffix;
    if (s > l)
        s = l;
    return s;
}

int bucket(int v)
{
    int b = 0;
    while ((1 << (b + 1)) <= v)
        b++;
    return b;
}

uint64_t tune_key(int l, int d, int n, int m)
{
    return ((uint64_t)l << 48) | ((uint64_t)d << 40) |
           ((uint64_t)bucket(n) << 20) | (uint64_t)bucket(m);
}

}  // namespace pms

thread_local std::string g_create_error;

int pms_ctx::fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return status;
}

int pms_ctx::alloc(DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes && b.p)
        return PMS_OK;
    size_t want = align_up(std::max(bytes, b.bytes + b.bytes / 4), 1 << 16);
    if (held.load() - b.bytes + want > budget) {
        want = align_up(bytes, 1 << 16);
        if (held.load() - b.bytes + want > budget)
            return fail(PMS_ENOMEM,
                        "device memory budget exceeded: need %zu bytes, "
                        "holding %zu of %zu",
                        want, held.load(), budget);
    }
    if (b.p) {
        hipStreamSynchronize(stream);
        hipFree(b.p);
        held -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PMS_ENOMEM, "hipMalloc(%zu): %s", want,
                    hipGetErrorString(e));
    }
    b.p = p;
    b.bytes = want;
    held += want;
    return PMS_OK;
}

void pms_ctx::release(DevBuf &b)
{
    if (b.p) {
        hipFree(b.p);
        held -= b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

TileCfg pms_ctx::tile_config(int n, int m, int l, int d)
{
    std::lock_guard<std::mutex> g(tune_mu);
    auto o = override_cfg.find({l, d});
    if (o != override_cfg.end())
        return o->second;
    auto t = tune.find(tune_key(l, d, n, m));
    if (t != tune.end())
        return t->second;
    return {default_suffix(l), kDefaultSurv, 0};
}

Plan pms_ctx::plan(int n, int m, int l, int d, int forced)
{
    Plan p{};
    const TileCfg cfg = tile_config(n, m, l, d);
    p.s = std::min(cfg.s, l);
    p.surv_t = std::max(1, std::min(cfg.surv_t, kSurvMax));
    p.tpb = cfg.tpb;
    p.ntiles = (l >= 3 && p.s >= 3) ? pow4(l - p.s) : 0;
    cost_model(n, m, l, d, p.s, p.surv_t, p.cost_filter, p.cost_tiled);
    if (forced == PMS_PATH_FILTER || forced == PMS_PATH_TILED ||
        forced == PMS_PATH_BITSET || forced == PMS_PATH_PAIR)
        p.path = forced;
    else
        p.path = (p.cost_tiled < p.cost_filter) ? PMS_PATH_TILED
                                                : PMS_PATH_FILTER;
    // beyond 4^14 tiles the pattern-driven paths are out of reach (every
    // tile pays at least one pass of prefix tests)
    if ((p.path == PMS_PATH_TILED || p.path == PMS_PATH_BITSET) &&
        (l < 3 || p.s < 3 || l - p.s > kMaxTilePrefix))
        p.path = PMS_PATH_FILTER;
    if (p.path == PMS_PATH_FILTER || p.path == PMS_PATH_PAIR)
        p.ntiles = 0;
    return p;
}

namespace {

void build_tables(std::vector<uint16_t> &ball, std::vector<int> &base,
                  std::vector<int> &off, std::vector<uint32_t> &ball32,
                  std::vector<uint32_t> &grp,
                  std::vector<unsigned long long> &m3)
{
    ball.clear();
    base.assign(8, 0);
    off.assign(7 * 8, 0);
    for (int q = 0; q <= kBallDigits; q++) {
        base[q] = (int)ball.size();
        std::vector<std::pair<int, int>> v;
        for (int mask = 0; mask < (1 << (2 * q)); mask++) {
            int w = 0;
            for (int i = 0; i < q; i++)
                w += ((mask >> (2 * i)) & 3) != 0;
            v.push_back({w, mask});
        }
        std::sort(v.begin(), v.end());
        for (int w = 0; w <= q + 1; w++) {
            int c = 0;
            for (auto &e : v)
                c += e.first < w;
            off[q * 8 + w] = c;
        }
        // Within each weight, deal the masks out round-robin by the bank
        // bits of their word position, wpos(mask) & 31: consecutive entries
        // (the lanes of one LDS instruction) then fall in distinct banks as
        // far as the weight's masks allow, and XOR with the l-mer's word
        // position, the same in every lane, keeps them distinct.
        for (int w = 0; w <= q; w++) {
            std::vector<std::vector<int>> byres(32);
            for (int i = off[q * 8 + w]; i < off[q * 8 + w + 1]; i++)
                byres[wpos((uint32_t)v[i].second) & 31u].push_back(
                    v[i].second);
            for (size_t k = 0;; k++) {
                bool any = false;
                for (int r = 0; r < 32; r++)
                    if (k < byres[r].size()) {
                        ball.push_back((uint16_t)(byres[r][k] | (w << 12)));
                        any = true;
                    }
                if (!any)
                    break;
            }
        }
    }
    ball32.resize(ball.size());
    for (size_t i = 0; i < ball.size(); i++)
        ball32[i] = 8u * wpos(ball[i] & 0xfffu) | (uint32_t)(ball[i] >> 12)
                                                      << 16;
    grp.assign(2 * kGrpStride, 0);
    for (int set = 0; set < 2; set++) {
        const uint32_t tpb = set ? 512u : 256u;
        for (int q = 0; q <= kBallDigits; q++)
            for (int rw = 0; rw <= q; rw++) {
                const uint32_t bs = (uint32_t)off[q * 8 + rw + 1];
                const uint32_t mg = ((1u << kGrpShift) + bs - 1) / bs;
                for (uint32_t v = 0; v < 1024; v++)
                    if ((v * mg) >> kGrpShift != v / bs)
                        abort();   // the multiplier must divide exactly
                uint32_t *g = &grp[set * kGrpStride + (q * 8 + rw) * 2];
                g[0] = tpb / bs;
                g[1] = mg;
            }
    }
    m3.assign(256, 0);
    for (int b = 0; b < 64; b++)
        for (int t = 0; t < 4; t++) {
            unsigned long long mk = 0;
            for (int z = 0; z < 64; z++) {
                int dist = 0;
                for (int i = 0; i < 3; i++)
                    dist += ((b >> (2 * i)) & 3) != ((z >> (2 * i)) & 3);
                if (dist <= t)
                    mk |= 1ull << z;
            }
            m3[b * 4 + t] = mk;
        }
}

int grid_for(pms_ctx *c, int bpc) { return std::max(1, c->n_cu * bpc); }

}  // namespace

// ---------------------------------------------------------------------------
// plain solve
// ---------------------------------------------------------------------------

namespace pms {

// Core of pms_solve / pms_solve_device. `d_seqs` is device input owned by
// the caller, or nullptr when host_seqs must be copied in. Results end in
// d_out_ext (cap_ext codes) if given, else in ctx-owned memory.
int solve_core(pms_ctx *c, const char *host_seqs, const uint8_t *d_seqs,
               int n, int m, int l, int d, hipStream_t st, uint64_t *d_out_ext,
               size_t cap_ext, int forced_path, SolveOut *res, int q,
               const FixedArena *fixed)
{
    const double t0 = now_ms();
    res->d_out = nullptr;
    res->count = 0;
    int rc = check_shape(n, m, l, d);
    if (rc)
        return c->fail(rc, "bad shape n=%d m=%d l=%d d=%d (need n>=1, "
                           "1<=l<=32, l<=m, 0<=d<l)", n, m, l, d);
    if (q < 0 || q > n)
        return c->fail(PMS_EINVAL, "quorum q=%d outside 1..n=%d", q, n);
    const bool quorum = q > 0 && q < n;
    bool quorum_filter = false;
    if (quorum) {
        if (n - q > kQuorumMaxMiss)
            return c->fail(PMS_EINVAL, "quorum: n-q=%d above %d", n - q,
                           kQuorumMaxMiss);
        if (forced_path == PMS_PATH_BITSET || forced_path == PMS_PATH_PAIR)
            return c->fail(PMS_EINVAL, "quorum (q<n) runs the tiled or the "
                           "filter path");
        quorum_filter = forced_path == PMS_PATH_FILTER;
        forced_path = quorum_filter ? PMS_PATH_FILTER : PMS_PATH_TILED;
    }
    if (fixed) {
        if (quorum || !d_out_ext)
            return c->fail(PMS_EINVAL, "fixed scratch: plain solves into a "
                           "caller buffer only");
        forced_path = PMS_PATH_TILED;
    }
    Plan P = c->plan(n, m, l, d, forced_path);
    if (fixed && P.path != PMS_PATH_TILED)
        return c->fail(PMS_EINVAL, "fixed scratch: l=%d is outside the tiled "
                       "path (3 <= l, at most 4^%d tiles)", l, kMaxTilePrefix);
    if (quorum) {
        // the tiled path while its tiles fit, else the sample-driven
        // filter with miss counts (Observation 3.1: references from the
        // first n-q+1 strings)
        P.s = std::min(P.s, kQuorumMaxSuffix);
        if (quorum_filter || l < 3 || P.s < 3 || l - P.s > kMaxTilePrefix) {
            quorum_filter = true;
            P.path = PMS_PATH_FILTER;
            P.ntiles = 0;
            const uint64_t refs = (uint64_t)(n - q + 1) * (uint64_t)(m - l + 1);
            if (refs >= filter_quorum_max_refs())
                return c->fail(PMS_EINVAL, "quorum filter: %llu reference "
                               "l-mers above %u", (unsigned long long)refs,
                               filter_quorum_max_refs());
        } else {
            P.path = PMS_PATH_TILED;
            P.ntiles = pow4(l - P.s);
        }
    }
    pms_stats S{};
    S.path = P.path;
    S.tile_suffix = (P.path == PMS_PATH_FILTER) ? 0 : P.s;
    const int L = m - l + 1;
    const uint64_t ntiles = P.ntiles;
    uint64_t heap_cap = std::max<uint64_t>(1 << 16, ntiles / 8);
    if (P.path == PMS_PATH_BITSET)
        heap_cap = 1;
    if (P.path == PMS_PATH_BITSET && (l - 3 > 28 || pow4(l - 3) * 8 >
                                                        c->budget))
        return c->fail(PMS_ENOMEM, "bitset path needs 4^%d/8 bytes", l);
    const auto shape_key =
        std::make_tuple(n, m, l, d, (quorum ? q : n) * 8 + P.path);
    if (P.path != PMS_PATH_BITSET) {
        auto hn = c->heap_need.find(shape_key);
        if (hn != c->heap_need.end())
            heap_cap = std::max(heap_cap, hn->second);
    }
    if (fixed) {
        // the heap takes every byte of the scratch that the rest leaves
        const InstLayout l0 = layout_instance(n, m, l, ntiles, 1, false, true,
                                              false);
        const size_t fixed_part = align_up(l0.total) +
                                  align_up(sizeof(InstDev)) +
                                  align_up(sizeof(TileStats)) + 256 + 512;
        if (fixed_part >= fixed->bytes)
            return c->fail(PMS_ENOMEM, "fixed scratch: the instance needs "
                           "%zu bytes beside its output heap; the scratch "
                           "holds %zu", fixed_part, fixed->bytes);
        heap_cap = 1 + (fixed->bytes - fixed_part) / 8;
    }

    for (int attempt = 0; attempt < 5; attempt++) {
        const bool own_out = (d_out_ext == nullptr) &&
                             P.path != PMS_PATH_BITSET;
        InstLayout lay = layout_instance(n, m, l, ntiles, heap_cap,
                                         d_seqs == nullptr, true, own_out);
        const size_t desc_off = align_up(lay.total);
        const size_t stats_off = desc_off + align_up(sizeof(InstDev));
        const size_t next_off = stats_off + align_up(sizeof(TileStats));
        const size_t need = next_off + 256;
        char *base;
        if (fixed) {
            if (need > fixed->bytes)
                return c->fail(PMS_ENOMEM, "fixed scratch: need %zu bytes, "
                               "the scratch holds %zu", need, fixed->bytes);
            base = fixed->base;
        } else {
            if ((rc = c->alloc(c->arena, need)))
                return rc;
            base = (char *)c->arena.p;
        }
        InstDev I = make_desc(base, lay, d_seqs, n, m, l, d, P.s, P.surv_t,
                              ntiles, heap_cap);
        if (quorum)
            I.q = q;
        InstDev *d_inst = (InstDev *)(base + desc_off);
        TileStats *d_stats = (TileStats *)(base + stats_off);
        unsigned long long *d_next = (unsigned long long *)(base + next_off);
        uint64_t *tile_pos = (uint64_t *)(base + lay.tile_pos);
        uint64_t *dst = d_out_ext ? d_out_ext : (uint64_t *)(base + lay.out);
        const uint64_t dst_cap = d_out_ext ? cap_ext : heap_cap;

        // host side of the descriptor and string order, via pinned staging
        memcpy(c->pinned_desc, &I, sizeof(I));
        int *ord = (int *)(c->pinned_desc + align_up(sizeof(InstDev)));
        if ((size_t)n * 4 + align_up(sizeof(InstDev)) > kPinnedDescBytes)
            return c->fail(PMS_EINVAL, "n=%d too large", n);
        for (int i = 0; i < n; i++)
            ord[i] = i;

        HIPCHK(c, hipEventRecord(c->ev[0], st));
        if (!d_seqs)
            HIPCHK(c, hipMemcpyAsync((void *)I.seqs, host_seqs, (size_t)n * m,
                                     hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync((void *)I.order, ord, 4 * (size_t)n,
                                 hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(d_inst, c->pinned_desc, sizeof(I),
                                 hipMemcpyHostToDevice, st));
        HIPCHK(c, launch_fill_u64(I.bad, 1, ~0ull, st));
        HIPCHK(c, launch_index(d_inst, 1, n * I.wpr, n * L, st));
        HIPCHK(c, launch_fill_u64((unsigned long long *)d_stats,
                                  sizeof(TileStats) / 8, 0, st));
        HIPCHK(c, launch_fill_u64(I.heap_top, 1, 0, st));
        HIPCHK(c, launch_fill_u64(d_next, 1, 0, st));
        HIPCHK(c, hipEventRecord(c->ev[1], st));

        unsigned long long *hp = c->pinned;   // [0] total [1] top [2] bad
        if (P.path == PMS_PATH_FILTER) {
            const uint64_t nb = nb_exact(l, d);
            if (nb > (1ull << 31))
                return c->fail(PMS_EINVAL, "filter path: n_B(%d,%d)=%llu too "
                               "large", l, d, (unsigned long long)nb);
            if (c->masks_l != l || c->masks_d != d) {
                if ((rc = c->alloc(c->masks, nb * 8)))
                    return rc;
                HIPCHK(c, launch_masks(l, d, (uint2 *)c->masks.p, nb, st));
                c->masks_l = l;
                c->masks_d = d;
                c->masks_nb = nb;
            }
            if ((rc = c->alloc(c->hc_ref, (size_t)L * 8)))
                return rc;
            HIPCHK(c, launch_fill_u64((unsigned long long *)c->hc_ref.p, L, 0,
                                      st));
            HIPCHK(c, hipEventRecord(c->ev[1], st));
            if (quorum_filter)
                HIPCHK(c, launch_filter_quorum(d_inst,
                                               (const uint2 *)c->masks.p, nb,
                                               n - q + 1, d_next, I.heap,
                                               I.heap_top, heap_cap,
                                               grid_for(c, c->filter_bpc),
                                               st));
            else
                HIPCHK(c, launch_filter(d_inst, (const uint2 *)c->masks.p, nb,
                                        d_next, I.heap, I.heap_top, heap_cap,
                                        (unsigned long long *)c->hc_ref.p,
                                        &d_stats->ftests,
                                        grid_for(c, c->filter_bpc), st));
            S.main_launches = 1;
            HIPCHK(c, hipEventRecord(c->ev[2], st));
            HIPCHK(c, hipMemcpyAsync(hp + 1, I.heap_top, 8,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipMemcpyAsync(hp + 2, I.bad, 8, hipMemcpyDeviceToHost,
                                     st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (hp[2] != ~0ull)
                return c->fail(PMS_EBASE, "bad base in string %llu at offset "
                               "%llu", hp[2] / m, hp[2] % m);
            if (hp[1] > heap_cap) {
                heap_cap = hp[1] + 1024;
                S.retries++;
                continue;
            }
            c->heap_need[shape_key] = hp[1] + 1024;
            const uint64_t total = hp[1];
            if (total > dst_cap) {
                res->count = total;
                return c->fail(PMS_ENOMEM, "output capacity %llu < %llu",
                               (unsigned long long)dst_cap,
                               (unsigned long long)total);
            }
            if (total) {
                if ((rc = c->alloc(c->sort_scr, sort_scratch_bytes(total))))
                    return rc;
                HIPCHK(c, hipMemcpyAsync(dst, I.heap, total * 8,
                                         hipMemcpyDeviceToDevice, st));
                HIPCHK(c, launch_sort_u64(dst, total, 2 * l, c->sort_scr.p,
                                          st));
            }
            HIPCHK(c, hipEventRecord(c->ev[3], st));
            res->count = total;
        } else if (P.path == PMS_PATH_PAIR) {
            uint64_t found = 0;
            if ((rc = pair_run(c, I, st, &found, S)))
                return rc;
            HIPCHK(c, hipEventRecord(c->ev[2], st));
            HIPCHK(c, hipMemcpyAsync(hp + 2, I.bad, 8, hipMemcpyDeviceToHost,
                                     st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (hp[2] != ~0ull)
                return c->fail(PMS_EBASE, "bad base in string %llu at offset "
                               "%llu", hp[2] / m, hp[2] % m);
            if (found > heap_cap) {
                heap_cap = found + 1024;
                S.retries++;
                continue;
            }
            c->heap_need[shape_key] = found + 1024;
            // sort, then drop repeats (one motif from several pairs)
            uint64_t total = 0;
            if (found) {
                if ((rc = c->alloc(c->sort_scr, sort_scratch_bytes(found))))
                    return rc;
                HIPCHK(c, launch_sort_u64(I.heap, found, 2 * l, c->sort_scr.p,
                                          st));
                const size_t o_pos = align_up(found * 4);
                const size_t o_scan = o_pos + align_up((found + 1) * 8);
                if ((rc = c->alloc(c->aux, o_scan +
                                               scan_scratch_bytes(found))))
                    return rc;
                char *ab = (char *)c->aux.p;
                HIPCHK(c, launch_unique_count(I.heap, found, (uint32_t *)ab,
                                              (uint64_t *)(ab + o_pos),
                                              ab + o_scan, st));
                HIPCHK(c, hipMemcpyAsync(hp, (uint64_t *)(ab + o_pos) + found,
                                         8, hipMemcpyDeviceToHost, st));
                HIPCHK(c, hipStreamSynchronize(st));
                total = hp[0];
                if (total > dst_cap) {
                    res->count = total;
                    return c->fail(PMS_ENOMEM, "output capacity %llu < %llu",
                                   (unsigned long long)dst_cap,
                                   (unsigned long long)total);
                }
                HIPCHK(c, launch_unique_scatter(I.heap, found,
                                                (const uint32_t *)ab,
                                                (const uint64_t *)(ab + o_pos),
                                                dst, st));
            }
            HIPCHK(c, hipEventRecord(c->ev[3], st));
            res->count = total;
        } else if (P.path == PMS_PATH_TILED) {
            const uint64_t max_items = 1u << 20;
            uint64_t chunk = (ntiles + max_items - 1) / max_items;
            // tiles of 4^8 or 4^9 codes on the plain path: the 512-thread
            // kernel (twice the waves per CU in flight); it loses on the
            // smaller tiles (fewer words per thread than lanes can hide)
            const bool wide = !quorum && pick_wide(c, P);
            const int tgrid =
                grid_for(c, wide ? c->tiled_wide_bpc : c->tiled_bpc);
            // sibling tiles share one string order: items of kOrderReuse
            // tiles where that still leaves every workgroup many items
            const uint64_t grid_tiles = (uint64_t)tgrid * kOrderReuse * 4;
            if (!quorum && I.tile_order && ntiles >= grid_tiles)
                chunk = std::max<uint64_t>(chunk, kOrderReuse);
            const uint64_t nitems = (ntiles + chunk - 1) / chunk;
            if (quorum)
                HIPCHK(c, launch_tiled_quorum(d_inst, nullptr, (int)nitems,
                                              chunk, (unsigned int *)d_next,
                                              c->tb, d_stats,
                                              grid_for(c, c->tiled_q_bpc), st));
            else
                HIPCHK(c, launch_tiled(d_inst, nullptr, (int)nitems, chunk,
                                       (unsigned int *)d_next, c->tb, d_stats,
                                       tgrid, st, wide));
            S.main_launches = 1;
            S.tile_threads = wide ? 512 : 256;
            HIPCHK(c, hipEventRecord(c->ev[2], st));
            HIPCHK(c, launch_scan_u32(I.tile_cnt, ntiles, tile_pos,
                                      base + lay.scan, st));
            HIPCHK(c, launch_gather(I.tile_cnt, I.tile_heap_off, tile_pos,
                                    I.heap, ntiles, dst, dst_cap, heap_cap,
                                    st));
            HIPCHK(c, hipEventRecord(c->ev[3], st));
            HIPCHK(c, hipMemcpyAsync(hp, tile_pos + ntiles, 8,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipMemcpyAsync(hp + 1, I.heap_top, 8,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipMemcpyAsync(hp + 2, I.bad, 8, hipMemcpyDeviceToHost,
                                     st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (hp[2] != ~0ull)
                return c->fail(PMS_EBASE, "bad base in string %llu at offset "
                               "%llu", hp[2] / m, hp[2] % m);
            if (hp[1] > heap_cap && fixed) {
                res->count = hp[1];
                return c->fail(PMS_ENOMEM, "fixed scratch: %llu motifs do not "
                               "fit its output heap of %llu",
                               (unsigned long long)hp[1],
                               (unsigned long long)heap_cap);
            }
            if (hp[1] > heap_cap) {
                heap_cap = hp[1] + 1024;
                S.retries++;
                continue;
            }
            if (!fixed)
                c->heap_need[shape_key] = hp[1] + 1024;
            if (hp[0] > dst_cap) {
                res->count = hp[0];
                return c->fail(PMS_ENOMEM, "output capacity %llu < %llu",
                               (unsigned long long)dst_cap,
                               (unsigned long long)hp[0]);
            }
            res->count = hp[0];
        } else {
            // memory-heavy bitset path: 4^l bits in device memory
            const uint64_t words = pow4(l - 3);
            if ((rc = c->alloc(c->bitset, words * 8)))
                return rc;
            // one buffer: the alive flags; (n <= kOrderMax) each tile's
            // string order; 2n pass counters; two lists of live tiles; the
            // per-tile string masses the order is made from. The bytes are
            // read by 32-bit words, so the counters start on a whole word
            // past them.
            if (ntiles >= ((uint64_t)1 << 32))
                return c->fail(PMS_ENOMEM, "bitset path: 4^%d tiles", l - P.s);
            const bool border = n <= kOrderMax;
            const uint64_t cnt_off =
                (ntiles * (border ? 1 + n : 1) + 4 + 15) & ~(uint64_t)15;
            const uint64_t list_off = cnt_off + (uint64_t)8 * n;
            const uint64_t mass_off = list_off + ntiles * 8;
            if ((rc = c->alloc(c->alive, mass_off + (border ? ntiles * 4 * n
                                                             : 0))))
                return rc;
            uint8_t *d_alive = (uint8_t *)c->alive.p;
            uint8_t *d_ord = border ? d_alive + ntiles : nullptr;
            unsigned int *d_cnt = (unsigned int *)(d_alive + cnt_off);
            uint32_t *d_list0 = (uint32_t *)(d_alive + list_off);
            uint32_t *d_list1 = d_list0 + ntiles;
            base = (char *)c->arena.p;
            const int grid = grid_for(c, c->tiled_bpc);
            if (border)
                HIPCHK(c, launch_bitset_order(d_inst, c->tb,
                                              (uint32_t *)(d_alive + mass_off),
                                              d_ord, ntiles, n, st));
            HIPCHK(c, launch_fill_u64((unsigned long long *)d_cnt, n, 0, st));
            // ms_main covers the passes alone; the order counts as index
            HIPCHK(c, hipEventRecord(c->ev[1], st));
            // pass 0: tiles in chunks of up to 8, at least 8 chunks per
            // workgroup (later passes size theirs on the device)
            const int bgrid = grid_for(c, c->bitset_bpc);
            const int bchunk = (int)std::max<uint64_t>(
                1, std::min<uint64_t>(8, ntiles / ((uint64_t)bgrid * 8)));
            for (int pass = 0; pass < n; pass++)
                HIPCHK(c, launch_bitset_pass(d_inst, pass, c->tb,
                                             (unsigned long long *)c->bitset.p,
                                             d_alive, d_ord, d_cnt, d_list0,
                                             d_list1, bchunk, d_stats, bgrid,
                                             st));
            S.main_launches = n;
            HIPCHK(c, hipEventRecord(c->ev[2], st));
            HIPCHK(c, launch_bitset_count(d_inst,
                                          (unsigned long long *)c->bitset.p,
                                          (uint8_t *)c->alive.p, I.tile_cnt,
                                          grid, st));
            HIPCHK(c, launch_scan_u32(I.tile_cnt, ntiles, tile_pos,
                                      base + lay.scan, st));
            HIPCHK(c, hipMemcpyAsync(hp, tile_pos + ntiles, 8,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipMemcpyAsync(hp + 2, I.bad, 8, hipMemcpyDeviceToHost,
                                     st));
            HIPCHK(c, hipStreamSynchronize(st));
            if (hp[2] != ~0ull)
                return c->fail(PMS_EBASE, "bad base in string %llu at offset "
                               "%llu", hp[2] / m, hp[2] % m);
            const uint64_t total = hp[0];
            if (!d_out_ext) {
                if ((rc = c->alloc(c->out, std::max<uint64_t>(total, 1) * 8)))
                    return rc;
                dst = (uint64_t *)c->out.p;
            } else if (total > cap_ext) {
                res->count = total;
                return c->fail(PMS_ENOMEM, "output capacity %zu < %llu",
                               cap_ext, (unsigned long long)total);
            }
            HIPCHK(c, launch_bitset_emit(d_inst,
                                         (unsigned long long *)c->bitset.p,
                                         I.tile_cnt, tile_pos, dst, total, grid,
                                         st));
            HIPCHK(c, hipEventRecord(c->ev[3], st));
            res->count = total;
        }
        res->d_out = dst;
        // statistics
        HIPCHK(c, hipMemcpyAsync(c->pinned + 8, d_stats, sizeof(TileStats),
                                 hipMemcpyDeviceToHost, st));
        if (P.path == PMS_PATH_FILTER && L <= (int)kPinnedHcEntries)
            HIPCHK(c, hipMemcpyAsync(c->pinned_hc, c->hc_ref.p,
                                     (size_t)L * 8, hipMemcpyDeviceToHost,
                                     st));
        HIPCHK(c, hipStreamSynchronize(st));
        TileStats ts;
        memcpy(&ts, c->pinned + 8, sizeof(ts));
        float a = 0, b = 0, e = 0;
        hipEventElapsedTime(&a, c->ev[0], c->ev[1]);
        hipEventElapsedTime(&b, c->ev[1], c->ev[2]);
        hipEventElapsedTime(&e, c->ev[2], c->ev[3]);
        S.ms_index = a;
        S.ms_main = b;
        S.ms_output = e;
        if (P.path == PMS_PATH_FILTER) {
            uint64_t h = 0;
            if (L <= (int)kPinnedHcEntries) {
                for (int j = 0; j < L; j++)
                    h += c->pinned_hc[j];
            } else {
                std::vector<unsigned long long> per(L);
                HIPCHK(c, hipMemcpy(per.data(), c->hc_ref.p, (size_t)L * 8,
                                    hipMemcpyDeviceToHost));
                for (auto v : per)
                    h += v;
            }
            S.hcanon = h;
            S.filter_tests = ts.ftests;   // executed, whole waves
        } else if (P.path != PMS_PATH_PAIR) {
            S.tiles = (P.path == PMS_PATH_TILED) ? ts.tiles : ntiles;
            S.tile_passes = ts.passes;
            S.marks = ts.marks;
            S.filter_tests = ts.ftests;
            if (P.path == PMS_PATH_BITSET) {
                // pass 0 writes 4^s bits per tile; later live passes read
                // and write them
                const uint64_t tb = pow4(P.s) / 8;
                S.bytes_main = ntiles * tb + (ts.passes - ntiles) * 2 * tb;
            }
        }
        S.ms_total = now_ms() - t0;
        c->last = S;
        // per-reference counts exist after the plain filter path only
        c->last_L = quorum_filter ? 0 : L;
        return PMS_OK;
    }
    return c->fail(PMS_ENOMEM, "output did not fit after retries");
}

}  // namespace pms

// ---------------------------------------------------------------------------
// C ABI: context and plain solves
// ---------------------------------------------------------------------------

extern "C" {

void pms_default_options(pms_options *opt)
{
    if (!opt)
        return;
    memset(opt, 0, sizeof(*opt));
}

const char *pms_status_string(int s)
{
    switch (s) {
    case PMS_OK: return "PMS_OK";
    case PMS_PENDING: return "PMS_PENDING";
    case PMS_EINVAL: return "PMS_EINVAL";
    case PMS_EBASE: return "PMS_EBASE";
    case PMS_ENOMEM: return "PMS_ENOMEM";
    case PMS_EDEVICE: return "PMS_EDEVICE";
    case PMS_EBUSY: return "PMS_EBUSY";
    default: return "PMS_UNKNOWN";
    }
}

int pms_create(pms_ctx **out, const pms_options *opt)
{
    if (!out) {
        g_create_error = "out is NULL";
        return PMS_EINVAL;
    }
    *out = nullptr;
    pms_options o;
    pms_default_options(&o);
    if (opt)
        o = *opt;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        g_create_error = "no HIP device";
        return PMS_EDEVICE;
    }
    if (o.device < 0 || o.device >= ndev) {
        g_create_error = "bad device ordinal";
        return PMS_EINVAL;
    }
    if (o.path < 0 || o.path > PMS_PATH_PAIR || o.serve_slots < 0 ||
        o.serve_queue < 0 || !(o.serve_launch_ms >= 0.0) ||
        o.serve_launch_ms > 1000.0 || o.pair_partner < 0 ||
        o.pair_partner > 1 ||
        (o.tile_threads != 0 && o.tile_threads != 256 &&
         o.tile_threads != 512)) {
        g_create_error = "bad option value";
        return PMS_EINVAL;
    }
    if (hipSetDevice(o.device) != hipSuccess) {
        g_create_error = "hipSetDevice failed";
        return PMS_EDEVICE;
    }
    std::unique_ptr<pms_ctx> c(new pms_ctx());
    c->opt = o;
    c->device = o.device;
    if (o.tune_cache)
        c->tune_path = o.tune_cache;
    c->opt.tune_cache = nullptr;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) != hipSuccess) {
        g_create_error = "hipGetDeviceProperties failed";
        return PMS_EDEVICE;
    }
    c->n_cu = prop.multiProcessorCount;
    c->tiled_bpc = tiled_blocks_per_cu();
    c->tiled_wide_bpc = tiled_blocks_per_cu(true);
    c->tiled_q_bpc = tiled_quorum_blocks_per_cu();
    c->bitset_bpc = bitset_blocks_per_cu();
    c->alpha_bpc = alpha_blocks_per_cu();
    c->wide_bpc = wide_blocks_per_cu();
    c->pair_bpc = pair_blocks_per_cu();
    c->filter_bpc = filter_blocks_per_cu();
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) != hipSuccess) {
        g_create_error = "hipMemGetInfo failed";
        return PMS_EDEVICE;
    }
    c->budget = o.mem_budget_bytes ? o.mem_budget_bytes
                                   : (size_t)(0.9 * (double)freeb);
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) !=
        hipSuccess) {
        g_create_error = "hipStreamCreate failed";
        return PMS_EDEVICE;
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            g_create_error = "hipEventCreate failed";
            return PMS_EDEVICE;
        }
    if (hipHostMalloc((void **)&c->pinned, 64 * 8) != hipSuccess ||
        hipHostMalloc((void **)&c->pinned_desc, kPinnedDescBytes) !=
            hipSuccess ||
        hipHostMalloc((void **)&c->pinned_hc, kPinnedHcEntries * 8) !=
            hipSuccess) {
        g_create_error = "hipHostMalloc failed";
        return PMS_EDEVICE;
    }
    std::vector<uint16_t> ball;
    std::vector<int> bbase, boff;
    std::vector<uint32_t> ball32, grp;
    std::vector<unsigned long long> m3;
    build_tables(ball, bbase, boff, ball32, grp, m3);
    const size_t o_ball = 0;
    const size_t o_base = align_up(ball.size() * 2);
    const size_t o_off = o_base + align_up(bbase.size() * 4);
    const size_t o_b32 = o_off + align_up(boff.size() * 4);
    const size_t o_grp = o_b32 + align_up(ball32.size() * 4);
    const size_t o_m3 = o_grp + align_up(grp.size() * 4);
    const size_t tbytes = o_m3 + align_up(m3.size() * 8);
    if (hipMalloc(&c->tables_mem, tbytes) != hipSuccess) {
        g_create_error = "hipMalloc(tables) failed";
        return PMS_ENOMEM;
    }
    c->held += tbytes;
    char *tb = (char *)c->tables_mem;
    if (hipMemcpy(tb + o_ball, ball.data(), ball.size() * 2,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(tb + o_base, bbase.data(), bbase.size() * 4,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(tb + o_off, boff.data(), boff.size() * 4,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(tb + o_b32, ball32.data(), ball32.size() * 4,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(tb + o_grp, grp.data(), grp.size() * 4,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(tb + o_m3, m3.data(), m3.size() * 8,
                  hipMemcpyHostToDevice) != hipSuccess) {
        g_create_error = "table upload failed";
        return PMS_EDEVICE;
    }
    c->tb.ball = (const uint16_t *)(tb + o_ball);
    c->tb.ball_base = (const int *)(tb + o_base);
    c->tb.ball_off = (const int *)(tb + o_off);
    c->tb.ball32 = (const uint32_t *)(tb + o_b32);
    c->tb.grp = (const uint32_t *)(tb + o_grp);
    c->tb.m3 = (const unsigned long long *)(tb + o_m3);
    load_tune_cache(c.get());
    // the no-allocation entry point's scratch array on this device (the
    // device is current); a failure here is retried at that entry point
    (void)noalloc_scratch(c->device);
    *out = c.release();
    return PMS_OK;
}

void pms_destroy(pms_ctx *c)
{
    if (!c)
        return;
    hipSetDevice(c->device);
    serve_shutdown(c);
    if (c->stream)
        hipStreamSynchronize(c->stream);
    if (c->b_graph) {
        hipGraphExecDestroy(c->b_graph);
        hipGraphDestroy(c->b_graph_def);
    }
    for (DevBuf *b : {&c->arena, &c->out, &c->masks, &c->hc_ref, &c->sort_scr,
                      &c->bitset, &c->alive, &c->b_arena, &c->aux})
        c->release(*b);
    if (c->tables_mem)
        hipFree(c->tables_mem);
    if (c->pinned)
        hipHostFree(c->pinned);
    if (c->pinned_desc)
        hipHostFree(c->pinned_desc);
    if (c->pinned_hc)
        hipHostFree(c->pinned_hc);
    if (c->b_pinned)
        hipHostFree(c->b_pinned);
    for (auto &e : c->ev)
        if (e)
            hipEventDestroy(e);
    if (c->stream)
        hipStreamDestroy(c->stream);
    delete c;
}

const char *pms_last_error(const pms_ctx *c)
{
    if (!c)
        return g_create_error.c_str();
    return c->err.c_str();
}

int pms_solve(pms_ctx *c, const char *seqs, int n, int m, int l, int d,
              const uint64_t **motifs, size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!seqs || !motifs || !count)
        return c->fail(PMS_EINVAL, "NULL argument");
    *motifs = nullptr;
    *count = 0;
    hipSetDevice(c->device);
    SolveOut r{};
    int rc = solve_core(c, seqs, nullptr, n, m, l, d, c->stream, nullptr, 0,
                        c->opt.path, &r);
    if (rc)
        return rc;
    c->host_out.resize(r.count);
    if (r.count) {
        HIPCHK(c, hipMemcpyAsync(c->host_out.data(), r.d_out, r.count * 8,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *motifs = c->host_out.data();
    }
    *count = r.count;
    return PMS_OK;
}

int pms_solve_device(pms_ctx *c, const uint8_t *d_seqs, int n, int m, int l,
                     int d, void *stream, uint64_t *d_out, size_t cap,
                     size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!d_seqs || !count || !d_out)
        return c->fail(PMS_EINVAL, "NULL argument");
    *count = 0;
    hipSetDevice(c->device);
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    SolveOut r{};
    int rc = solve_core(c, nullptr, d_seqs, n, m, l, d, st, d_out, cap,
                        c->opt.path, &r);
    *count = r.count;
    return rc;
}

int pms_solve_quorum(pms_ctx *c, const char *seqs, int n, int m, int l,
                     int d, int q, const uint64_t **motifs, size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!seqs || !motifs || !count)
        return c->fail(PMS_EINVAL, "NULL argument");
    *motifs = nullptr;
    *count = 0;
    if (q < 1 || q > n)
        return c->fail(PMS_EINVAL, "quorum q=%d outside 1..n=%d", q, n);
    hipSetDevice(c->device);
    SolveOut r{};
    int rc = solve_core(c, seqs, nullptr, n, m, l, d, c->stream, nullptr, 0,
                        c->opt.path, &r, q);
    if (rc)
        return rc;
    c->host_out.resize(r.count);
    if (r.count) {
        HIPCHK(c, hipMemcpyAsync(c->host_out.data(), r.d_out, r.count * 8,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *motifs = c->host_out.data();
    }
    *count = r.count;
    return PMS_OK;
}

int pms_solve_quorum_device(pms_ctx *c, const uint8_t *d_seqs, int n, int m,
                            int l, int d, int q, void *stream, uint64_t *d_out,
                            size_t cap, size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!d_seqs || !count || !d_out)
        return c->fail(PMS_EINVAL, "NULL argument");
    *count = 0;
    if (q < 1 || q > n)
        return c->fail(PMS_EINVAL, "quorum q=%d outside 1..n=%d", q, n);
    hipSetDevice(c->device);
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    SolveOut r{};
    int rc = solve_core(c, nullptr, d_seqs, n, m, l, d, st, d_out, cap,
                        c->opt.path, &r, q);
    *count = r.count;
    return rc;
}

int pms_last_stats(const pms_ctx *c, pms_stats *out)
{
    if (!c || !out)
        return PMS_EINVAL;
    *out = c->last;
    return PMS_OK;
}

int pms_last_hcanon_per_ref(const pms_ctx *c, uint64_t *out, size_t n_refs)
{
    if (!c || !out)
        return PMS_EINVAL;
    pms_ctx *cc = const_cast<pms_ctx *>(c);
    if (c->last.path != PMS_PATH_FILTER || (size_t)c->last_L != n_refs ||
        !c->hc_ref.p)
        return cc->fail(PMS_EINVAL, "no filter-path solve with %zu "
                        "references", n_refs);
    HIPCHK(cc, hipMemcpy(out, c->hc_ref.p, n_refs * 8, hipMemcpyDeviceToHost));
    return PMS_OK;
}

int pms_set_tile_config(pms_ctx *c, int l, int d, int s, int surv_t)
{
    if (!c)
        return PMS_EINVAL;
    std::lock_guard<std::mutex> g(c->tune_mu);
    if (s == 0) {
        c->override_cfg.erase({l, d});
        return PMS_OK;
    }
    if (s < kMinSuffix || s > kMaxSuffix || s > l || surv_t < 1 ||
        surv_t > kSurvMax)
        return c->fail(PMS_EINVAL, "tile config s=%d surv_t=%d out of range "
                       "(3<=s<=min(9,l), 1<=surv_t<=%d)", s, surv_t, kSurvMax);
    c->override_cfg[{l, d}] = {s, surv_t, 0};
    return PMS_OK;
}

}  // extern "C"
