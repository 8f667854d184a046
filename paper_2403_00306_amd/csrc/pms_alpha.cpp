// pms_alpha.cpp -- host side of the any-alphabet path (pms_solve_alphabet).
//
// Motifs over an alphabet of 2..32 letters (Sec. 1.2.5 states the problem
// over any alphabet; Table 3.1 sizes the spheres for any |Sigma|): the
// sample-driven filter of k_alpha.hip, then sort and repeat removal on the
// device. The DNA alphabet "ACGT" in that order is solved by pms_solve's
// paths, whose codes are the same base-4 numbers.
#include "pms_host.h"

#include <algorithm>
#include <cstring>
#include <vector>

using namespace pms;

namespace {

// sigma^l, or 0 if it does not fit in 64 bits
// sigma^l, the size of the code space, exact up to 2^64 (past that only
// known to be above it). Codes 0 .. sigma^l - 1 fit in 64 bits iff
// sigma^l <= 2^64.
constexpr unsigned __int128 kSpace64 = ((unsigned __int128)1) << 64;

unsigned __int128 space_of(int sigma, int l)
{
    unsigned __int128 v = 1;
    for (int j = 0; j < l && v <= kSpace64; j++)
        v *= (unsigned)sigma;
    return v;
}

struct AlphaPlan {
    std::vector<uint32_t> posset;
    uint64_t posoff[kMaxL + 2], cum[kMaxL + 2], powr[kMaxL + 2];
    uint64_t nb;
    int key_bits;
};

// Position sets of every weight k <= d (bitmasks over l positions), the
// first flat sphere index of each weight and (sigma-1)^k. Fails when the
// tables or the sphere are too large.
bool plan_alpha(int sigma, int l, int d, AlphaPlan &P)
{
    P.posset.clear();
    unsigned __int128 acc = 0;
    for (int k = 0; k <= d; k++) {
        P.posoff[k] = P.posset.size();
        // all k-subsets of {0..l-1} in lexicographic order
        std::vector<int> idx(k);
        for (int i = 0; i < k; i++)
            idx[i] = i;
        for (;;) {
            uint32_t msk = 0;
            for (int i = 0; i < k; i++)
                msk |= 1u << idx[i];
            P.posset.push_back(msk);
            if (P.posset.size() > (1u << 22))
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
            pw *= (unsigned)(sigma - 1);
        if (pw > (((unsigned __int128)1) << 62))
            return false;
        P.powr[k] = (uint64_t)pw;
        P.cum[k] = (uint64_t)acc;
        acc += pw * (unsigned __int128)(P.posset.size() - P.posoff[k]);
        if (acc > (((unsigned __int128)1) << 62))
            return false;
    }
    P.cum[d + 1] = (uint64_t)acc;
    P.posoff[d + 1] = P.posset.size();
    P.nb = (uint64_t)acc;
    const unsigned __int128 space = space_of(sigma, l);
    int bits = 0;
    while (bits < 64 && (((unsigned __int128)1) << bits) < space)
        bits++;
    P.key_bits = std::max(bits, 1);
    return true;
}

int alpha_core(pms_ctx *c, const char *alphabet, int sigma,
               const char *host_seqs, const uint8_t *d_seqs, int n, int m,
               int l, int d, hipStream_t st, uint64_t *d_out_ext,
               size_t cap_ext, SolveOut *res)
{
    const double t0 = now_ms();
    res->d_out = nullptr;
    res->count = 0;
    int rc = check_shape(n, m, l, d);
    if (rc)
        return c->fail(rc, "bad shape n=%d m=%d l=%d d=%d (need n>=1, "
                           "1<=l<=32, l<=m, 0<=d<l)", n, m, l, d);
    if (!alphabet || sigma < 2 || sigma > 32)
        return c->fail(PMS_EINVAL, "alphabet: need 2..32 letters");
    uint8_t map[256];
    memset(map, 0xff, sizeof(map));
    for (int i = 0; i < sigma; i++) {
        const uint8_t ch = (uint8_t)alphabet[i];
        if (map[ch] != 0xff)
            return c->fail(PMS_EINVAL, "alphabet: letter '%c' repeated", ch);
        map[ch] = (uint8_t)i;
    }
    if (space_of(sigma, l) > kSpace64)
        return c->fail(PMS_EINVAL, "alphabet: %d^%d codes do not fit in 64 "
                       "bits", sigma, l);
    AlphaPlan P;
    if (!plan_alpha(sigma, l, d, P))
        return c->fail(PMS_EINVAL, "alphabet: sphere of (%d,%d) over %d "
                       "letters too large", l, d, sigma);
    int planes = 1;
    while ((1 << planes) < sigma)
        planes++;
    const int L = m - l + 1;
    // candidates (sphere x references) must stay countable in 64 bits
    if ((unsigned __int128)P.nb * (unsigned)L > (((unsigned __int128)1) << 62))
        return c->fail(PMS_EINVAL, "alphabet: %llu candidates per reference "
                       "x %d references: too many", (unsigned long long)P.nb,
                       L);

    const auto shape_key = std::make_tuple(n, m, l, d, -sigma);
    uint64_t heap_cap = 1 << 16;
    {
        auto hn = c->heap_need.find(shape_key);
        if (hn != c->heap_need.end())
            heap_cap = std::max(heap_cap, hn->second);
    }
    pms_stats S{};
    S.path = PMS_PATH_FILTER;
    for (int attempt = 0; attempt < 5; attempt++) {
        // arena: inputs, index, tables and counters
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off = align_up(off + std::max<size_t>(bytes, 1));
            return o;
        };
        const size_t o_seqs = d_seqs ? 0 : take((size_t)n * m);
        const size_t o_map = take(256);
        const size_t o_let = take((size_t)n * m);
        const size_t o_pl = take((size_t)n * L * 8 * 4);
        const size_t o_bad = take(8);
        const size_t o_pos = take(P.posset.size() * 4);
        const size_t o_tab = take(3 * (kMaxL + 2) * 8);
        const size_t o_cnt = take(24);   // next item, heap top, tests
        if ((rc = c->alloc(c->arena, off)))
            return rc;
        // aux: heap, flags, positions, scan scratch
        size_t aoff = 0;
        auto atake = [&](size_t bytes) {
            const size_t o = aoff;
            aoff = align_up(aoff + std::max<size_t>(bytes, 1));
            return o;
        };
        const size_t a_heap = atake(heap_cap * 8);
        const size_t a_flag = atake(heap_cap * 4);
        const size_t a_posn = atake((heap_cap + 1) * 8);
        const size_t a_scan = atake(scan_scratch_bytes(heap_cap));
        if ((rc = c->alloc(c->aux, aoff)))
            return rc;
        char *base = (char *)c->arena.p, *abase = (char *)c->aux.p;
        const uint8_t *seqs = d_seqs ? d_seqs : (const uint8_t *)(base + o_seqs);
        unsigned long long *bad = (unsigned long long *)(base + o_bad);
        unsigned int *next = (unsigned int *)(base + o_cnt);
        unsigned long long *top = (unsigned long long *)(base + o_cnt + 8);
        uint64_t *tab = (uint64_t *)(base + o_tab);

        // host tables, staged through the pinned buffer
        std::vector<uint64_t> t(3 * (kMaxL + 2), 0);
        for (int k = 0; k <= d + 1; k++) {
            t[k] = P.posoff[k];
            t[(kMaxL + 2) + k] = P.cum[k];
            t[2 * (kMaxL + 2) + k] = k <= d ? P.powr[k] : 0;
        }
        HIPCHK(c, hipEventRecord(c->ev[0], st));
        if (!d_seqs)
            HIPCHK(c, hipMemcpyAsync((void *)seqs, host_seqs, (size_t)n * m,
                                     hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(base + o_map, map, 256,
                                 hipMemcpyHostToDevice, st));
        HIPCHK(c, hipMemcpyAsync(base + o_pos, P.posset.data(),
                                 P.posset.size() * 4, hipMemcpyHostToDevice,
                                 st));
        HIPCHK(c, hipMemcpyAsync(tab, t.data(), t.size() * 8,
                                 hipMemcpyHostToDevice, st));
        HIPCHK(c, launch_fill_u64(bad, 1, ~0ull, st));
        HIPCHK(c, launch_fill_u64((unsigned long long *)next, 3, 0, st));
        HIPCHK(c, launch_alpha_index(seqs, (const uint8_t *)(base + o_map), n,
                                     m, l, planes, (uint8_t *)(base + o_let),
                                     (uint32_t *)(base + o_pl), bad, st));
        HIPCHK(c, hipEventRecord(c->ev[1], st));
        AlphaJob J;
        J.letters = (const uint8_t *)(base + o_let);
        J.planes = (const uint32_t *)(base + o_pl);
        J.posset = (const uint32_t *)(base + o_pos);
        J.posoff = tab;
        J.cum = tab + (kMaxL + 2);
        J.powr = tab + 2 * (kMaxL + 2);
        J.nb = P.nb;
        J.heap = (uint64_t *)(abase + a_heap);
        J.heap_top = top;
        J.heap_cap = heap_cap;
        J.hcanon = (unsigned long long *)(base + o_cnt + 16);
        J.n = n;
        J.m = m;
        J.l = l;
        J.d = d;
        J.L = L;
        J.sigma = sigma;
        HIPCHK(c, launch_alpha_filter(J, next,
                                      std::max(1, c->n_cu * c->alpha_bpc),
                                      st));
        HIPCHK(c, hipEventRecord(c->ev[2], st));
        unsigned long long *hp = c->pinned;
        HIPCHK(c, hipMemcpyAsync(hp, top, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(hp + 1, bad, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(hp + 2, J.hcanon, 8, hipMemcpyDeviceToHost,
                                 st));
        HIPCHK(c, hipStreamSynchronize(st));
        S.hcanon = hp[2];
        if (hp[1] != ~0ull)
            return c->fail(PMS_EBASE, "byte not in the alphabet in string "
                           "%llu at offset %llu", hp[1] / m, hp[1] % m);
        const uint64_t found = hp[0];
        if (found > heap_cap) {
            heap_cap = found + 1024;
            S.retries++;
            continue;
        }
        c->heap_need[shape_key] = found + 1024;
        // sort, then drop repeats into the output
        uint64_t *heap = J.heap;
        uint64_t *posn = (uint64_t *)(abase + a_posn);
        uint64_t total = 0;
        if (found) {
            if ((rc = c->alloc(c->sort_scr, sort_scratch_bytes(found))))
                return rc;
            HIPCHK(c, launch_sort_u64(heap, found, P.key_bits, c->sort_scr.p,
                                      st));
            // repeats sit next to each other: count the distinct values
            HIPCHK(c, launch_unique_count(heap, found,
                                          (uint32_t *)(abase + a_flag), posn,
                                          abase + a_scan, st));
            HIPCHK(c, hipMemcpyAsync(hp, posn + found, 8,
                                     hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            total = hp[0];
        }
        uint64_t *dst = d_out_ext;
        if (!dst) {
            if ((rc = c->alloc(c->out, std::max<uint64_t>(total, 1) * 8)))
                return rc;
            dst = (uint64_t *)c->out.p;
        } else if (total > cap_ext) {
            res->count = total;
            return c->fail(PMS_ENOMEM, "output capacity %llu < %llu",
                           (unsigned long long)cap_ext,
                           (unsigned long long)total);
        }
        HIPCHK(c, launch_unique_scatter(heap, found,
                                        (const uint32_t *)(abase + a_flag),
                                        posn, dst, st));
        HIPCHK(c, hipEventRecord(c->ev[3], st));
        HIPCHK(c, hipStreamSynchronize(st));
        float a = 0, b = 0, e = 0;
        hipEventElapsedTime(&a, c->ev[0], c->ev[1]);
        hipEventElapsedTime(&b, c->ev[1], c->ev[2]);
        hipEventElapsedTime(&e, c->ev[2], c->ev[3]);
        S.ms_index = a;
        S.ms_main = b;
        S.ms_output = e;
        S.main_launches = 1;
        S.ms_total = now_ms() - t0;
        c->last = S;
        c->last_L = 0;   // no per-reference counts on this path
        res->d_out = dst;
        res->count = total;
        return PMS_OK;
    }
    return c->fail(PMS_ENOMEM, "output did not fit after retries");
}

bool is_dna(const char *alphabet, int sigma)
{
    return sigma == 4 && alphabet && memcmp(alphabet, "ACGT", 4) == 0;
}

}  // namespace

extern "C" {

int pms_solve_alphabet(pms_ctx *c, const char *alphabet, int sigma,
                       const char *seqs, int n, int m, int l, int d,
                       const uint64_t **motifs, size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!seqs || !motifs || !count || !alphabet)
        return c->fail(PMS_EINVAL, "NULL argument");
    if (is_dna(alphabet, sigma))
        return pms_solve(c, seqs, n, m, l, d, motifs, count);
    *motifs = nullptr;
    *count = 0;
    hipSetDevice(c->device);
    SolveOut r{};
    int rc = alpha_core(c, alphabet, sigma, seqs, nullptr, n, m, l, d,
                        c->stream, nullptr, 0, &r);
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

int pms_solve_alphabet_device(pms_ctx *c, const char *alphabet, int sigma,
                              const uint8_t *d_seqs, int n, int m, int l,
                              int d, void *stream, uint64_t *d_out, size_t cap,
                              size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!d_seqs || !count || !d_out || !alphabet)
        return c->fail(PMS_EINVAL, "NULL argument");
    if (is_dna(alphabet, sigma))
        return pms_solve_device(c, d_seqs, n, m, l, d, stream, d_out, cap,
                                count);
    *count = 0;
    hipSetDevice(c->device);
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    SolveOut r{};
    int rc = alpha_core(c, alphabet, sigma, nullptr, d_seqs, n, m, l, d, st,
                        d_out, cap, &r);
    *count = r.count;
    return rc;
}

}  // extern "C"
