// pms_wide.cpp -- host side of the long-motif path (pms_solve_wide): motifs
// of length up to 64 (Sec. 3.3.1 keeps such l-mers in ceil(l/32) words per
// group), solved by the sample-driven filter of k_wide.hip, then sorted on
// the device. Codes take 128 bits, returned as a high and a low word each.
#include "pms_host.h"
#include "pms_wide.h"

#include <algorithm>
#include <vector>

using namespace pms;

namespace {

constexpr size_t kMaxPosSets = (size_t)1 << 22;

struct WidePlan {
    std::vector<uint64_t> posset;
    uint64_t posoff[kWideMaxL + 2], cum[kWideMaxL + 2], pow3[kWideMaxL + 2];
    uint64_t nb;
};

// Position sets of every weight k <= d (bit masks over l positions, each
// weight in lexicographic order), the first sphere index of each weight and
// 3^k. Fails when the tables or the sphere are too large.
bool plan_wide(int l, int d, WidePlan &P)
{
    P.posset.clear();
    unsigned __int128 acc = 0;
    for (int k = 0; k <= d; k++) {
        P.posoff[k] = P.posset.size();
        std::vector<int> idx(k);
        for (int i = 0; i < k; i++)
            idx[i] = i;
        for (;;) {
            uint64_t msk = 0;
            for (int i = 0; i < k; i++)
                msk |= 1ull << idx[i];
            P.posset.push_back(msk);
            if (P.posset.size() > kMaxPosSets)
                return false;
            int i = k - 1;
            while (i >= 0 && idx[i] == l - k + i)
                i--;
            if (i < 0)
                break;
            idx[i]++;
            for (int j = i + 1; j < k; j++)
                idx[j] = idx[j - 1] + 1;
        }
        unsigned __int128 pw = 1;
        for (int i = 0; i < k; i++)
            pw *= 3u;
        if (pw > (((unsigned __int128)1) << 62))
            return false;
        P.pow3[k] = (uint64_t)pw;
        P.cum[k] = (uint64_t)acc;
        acc += pw * (unsigned __int128)(P.posset.size() - P.posoff[k]);
        if (acc > (((unsigned __int128)1) << 62))
            return false;
    }
    P.cum[d + 1] = (uint64_t)acc;
    P.posoff[d + 1] = P.posset.size();
    P.pow3[d + 1] = 0;
    P.nb = (uint64_t)acc;
    return true;
}

int check_wide(int n, int m, int l, int d)
{
    if (n < 1 || l < 1 || l > kWideMaxL || m < l || d < 0 || d >= l)
        return PMS_EINVAL;
    if ((double)n * (double)m > 4.0e9)
        return PMS_EINVAL;
    return PMS_OK;
}

// d_out_ext (2 words per motif, capacity cap_ext motifs) or, when null, the
// context's output buffer; res->d_out then points at the words and
// res->count counts motifs.
int wide_core(pms_ctx *c, const char *host_seqs, const uint8_t *d_seqs, int n,
              int m, int l, int d, hipStream_t st, uint64_t *d_out_ext,
              size_t cap_ext, SolveOut *res)
{
    const double t0 = now_ms();
    res->d_out = nullptr;
    res->count = 0;
    int rc = check_wide(n, m, l, d);
    if (rc)
        return c->fail(rc, "bad shape n=%d m=%d l=%d d=%d (need n>=1, "
                           "1<=l<=64, l<=m, 0<=d<l)", n, m, l, d);
    WidePlan P;
    if (!plan_wide(l, d, P))
        return c->fail(PMS_EINVAL, "sphere of (%d,%d) too large", l, d);
    const int L = m - l + 1;
    // candidates (sphere x references) must stay countable in 64 bits
    if ((unsigned __int128)P.nb * (unsigned)L > (((unsigned __int128)1) << 62))
        return c->fail(PMS_EINVAL, "%llu candidates per reference x %d "
                       "references: too many", (unsigned long long)P.nb, L);
    const auto shape_key = std::make_tuple(n, m, l, d, -1000);
    uint64_t heap_cap = 1 << 16;
    {
        auto hn = c->heap_need.find(shape_key);
        if (hn != c->heap_need.end())
            heap_cap = std::max(heap_cap, hn->second);
    }
    pms_stats S{};
    S.path = PMS_PATH_FILTER;
    for (int attempt = 0; attempt < 5; attempt++) {
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off = align_up(off + std::max<size_t>(bytes, 1));
            return o;
        };
        const size_t o_seqs = d_seqs ? 0 : take((size_t)n * m);
        const size_t o_pl = take((size_t)n * L * sizeof(ulonglong2));
        const size_t o_bad = take(8);
        const size_t o_pos = take(P.posset.size() * 8);
        const size_t o_tab = take(3 * (kWideMaxL + 2) * 8);
        const size_t o_cnt = take(24);   // next item, heap top, tests
        if ((rc = c->alloc(c->arena, off)))
            return rc;
        size_t aoff = 0;
        auto atake = [&](size_t bytes) {
            const size_t o = aoff;
            aoff = align_up(aoff + std::max<size_t>(bytes, 1));
            return o;
        };
        const size_t a_heap = atake(heap_cap * sizeof(W128));
        if ((rc = c->alloc(c->aux, aoff)))
            return rc;
        char *base = (char *)c->arena.p, *abase = (char *)c->aux.p;
        const uint8_t *seqs =
            d_seqs ? d_seqs : (const uint8_t *)(base + o_seqs);
        unsigned long long *bad = (unsigned long long *)(base + o_bad);
        unsigned long long *next = (unsigned long long *)(base + o_cnt);
        unsigned long long *top = next + 1;
        uint64_t *tab = (uint64_t *)(base + o_tab);
        std::vector<uint64_t> t(3 * (kWideMaxL + 2), 0);
        for (int k = 0; k <= d + 1; k++) {
            t[k] = P.posoff[k];
            t[(kWideMaxL + 2) + k] = P.cum[k];
            t[2 * (kWideMaxL + 2) + k] = P.pow3[k];
        }
        HIPCHK(c, hipEventRecord(c->ev[0], st));
        if (!d_seqs)
            HIPCHK(c, hipMemcpyAsync((void *)seqs, host_seqs, (size_t)n * m,
                                     hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(base + o_pos, P.posset.data(),
                                 P.posset.size() * 8, hipMemcpyHostToDevice,
                                 st));
        HIPCHK(c, hipMemcpyAsync(tab, t.data(), t.size() * 8,
                                 hipMemcpyHostToDevice, st));
        HIPCHK(c, launch_fill_u64(bad, 1, ~0ull, st));
        HIPCHK(c, launch_fill_u64(next, 3, 0, st));
        ulonglong2 *planes = (ulonglong2 *)(base + o_pl);
        HIPCHK(c, launch_wide_index(seqs, n, m, l, planes, bad, st));
        HIPCHK(c, hipEventRecord(c->ev[1], st));
        WideJob J;
        J.planes = planes;
        J.posset = (const uint64_t *)(base + o_pos);
        J.posoff = tab;
        J.cum = tab + (kWideMaxL + 2);
        J.pow3 = tab + 2 * (kWideMaxL + 2);
        J.nb = P.nb;
        J.heap = (W128 *)(abase + a_heap);
        J.heap_top = top;
        J.heap_cap = heap_cap;
        J.hcanon = next + 2;
        J.n = n;
        J.m = m;
        J.l = l;
        J.d = d;
        J.L = L;
        HIPCHK(c, launch_wide_filter(J, next,
                                     std::max(1, c->n_cu * c->wide_bpc), st));
        HIPCHK(c, hipEventRecord(c->ev[2], st));
        unsigned long long *hp = c->pinned;
        HIPCHK(c, hipMemcpyAsync(hp, top, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(hp + 1, bad, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(hp + 2, J.hcanon, 8, hipMemcpyDeviceToHost,
                                 st));
        HIPCHK(c, hipStreamSynchronize(st));
        S.hcanon = hp[2];
        S.filter_tests = hp[2];
        if (hp[1] != ~0ull)
            return c->fail(PMS_EBASE, "bad base in string %llu at offset %llu",
                           hp[1] / m, hp[1] % m);
        const uint64_t found = hp[0];
        if (found > heap_cap) {
            heap_cap = found + 1024;
            S.retries++;
            continue;
        }
        c->heap_need[shape_key] = found + 1024;
        // the survivors hold no repeats: sort them and copy them out
        W128 *heap = J.heap;
        if (found > 1) {
            if ((rc = c->alloc(c->sort_scr, sort_scratch_bytes_w128(found))))
                return rc;
            HIPCHK(c, launch_sort_w128(heap, found, 2 * l, c->sort_scr.p, st));
        }
        uint64_t *dst = d_out_ext;
        if (!dst) {
            if ((rc = c->alloc(c->out, std::max<uint64_t>(found, 1) * 16)))
                return rc;
            dst = (uint64_t *)c->out.p;
        } else if (found > cap_ext) {
            res->count = found;
            return c->fail(PMS_ENOMEM, "output capacity %llu < %llu",
                           (unsigned long long)cap_ext,
                           (unsigned long long)found);
        }
        if (found)
            HIPCHK(c, hipMemcpyAsync(dst, heap, found * sizeof(W128),
                                     hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipEventRecord(c->ev[3], st));
        HIPCHK(c, hipStreamSynchronize(st));
        float a = 0, b = 0, e = 0;
        (void)hipEventElapsedTime(&a, c->ev[0], c->ev[1]);
        (void)hipEventElapsedTime(&b, c->ev[1], c->ev[2]);
        (void)hipEventElapsedTime(&e, c->ev[2], c->ev[3]);
        S.ms_index = a;
        S.ms_main = b;
        S.ms_output = e;
        S.main_launches = 1;
        S.ms_total = now_ms() - t0;
        c->last = S;
        c->last_L = 0;   // no per-reference counts on this path
        res->d_out = dst;
        res->count = found;
        return PMS_OK;
    }
    return c->fail(PMS_ENOMEM, "output did not fit after retries");
}

}  // namespace

extern "C" {

int pms_solve_wide(pms_ctx *c, const char *seqs, int n, int m, int l, int d,
                   const uint64_t **motifs, size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!seqs || !motifs || !count)
        return c->fail(PMS_EINVAL, "NULL argument");
    *motifs = nullptr;
    *count = 0;
    (void)hipSetDevice(c->device);
    SolveOut r{};
    int rc = wide_core(c, seqs, nullptr, n, m, l, d, c->stream, nullptr, 0,
                       &r);
    if (rc)
        return rc;
    c->host_out.resize(2 * r.count);
    if (r.count) {
        HIPCHK(c, hipMemcpyAsync(c->host_out.data(), r.d_out, r.count * 16,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *motifs = c->host_out.data();
    }
    *count = r.count;
    return PMS_OK;
}

int pms_solve_wide_device(pms_ctx *c, const uint8_t *d_seqs, int n, int m,
                          int l, int d, void *stream, uint64_t *d_out,
                          size_t cap, size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!d_seqs || !count || !d_out)
        return c->fail(PMS_EINVAL, "NULL argument");
    *count = 0;
    (void)hipSetDevice(c->device);
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    SolveOut r{};
    int rc = wide_core(c, nullptr, d_seqs, n, m, l, d, st, d_out, cap, &r);
    *count = r.count;
    return rc;
}

}  // extern "C"
