// pms_pair.cpp -- host side of the pair-based path (PMS_PATH_PAIR).
//
// Observation 3.3 with q = n: every motif lies in B(x,d) ∩ B(y,d) for an
// l-mer x of s_1 and an l-mer y of a partner string s_j with
// d_H(x,y) <= 2d; j is s_2, or (TraverStringRef's string reordering,
// Sec. 3.2.3) for every x the string whose nearest l-mer is farthest from
// x, which gives smaller intersections. The host builds the counting tables
// of those intersections (they depend on D = d_H(x,y) only), then the
// device picks the partners, lists the compatible pairs, scans their
// work-item counts and filters every pair's candidates against the other
// strings.
#include "pms_host.h"

#include <algorithm>
#include <vector>

namespace pms {

int pair_run(pms_ctx *c, const InstDev &I, hipStream_t st, uint64_t *found,
             pms_stats &S)
{
    const int n = I.n, L = I.L, l = I.l, d = I.d;
    if (n < 2)
        return c->fail(PMS_EINVAL, "pair path needs n >= 2 strings");
    if (2 * d > 20)
        return c->fail(PMS_EINVAL, "pair path needs 2d <= 20 (d=%d)", d);
    const uint64_t LL = (uint64_t)L * (uint64_t)L;
    if (LL > (1ull << 28))
        return c->fail(PMS_EINVAL, "pair path: (m-l+1)^2 = %llu pairs above "
                       "2^28", (unsigned long long)LL);

    // counting tables: factorials, powers of 3, binomials, and per D the
    // tuples (a, b, c, e) with their sizes
    std::vector<uint64_t> fact(21, 1), pow3(kMaxL + 1, 1),
        binom((kMaxL + 1) * (kMaxL + 1), 0);
    for (int i = 1; i <= 20; i++)
        fact[i] = fact[i - 1] * (uint64_t)i;
    for (int i = 1; i <= kMaxL; i++)
        pow3[i] = pow3[i - 1] * 3;
    for (int a = 0; a <= kMaxL; a++) {
        binom[a * (kMaxL + 1)] = 1;
        for (int b = 1; b <= a; b++)
            binom[a * (kMaxL + 1) + b] = binom[(a - 1) * (kMaxL + 1) + b - 1] +
                                         (b <= a - 1
                                              ? binom[(a - 1) * (kMaxL + 1) + b]
                                              : 0);
    }
    std::vector<PairTuple> tup;
    std::vector<int> tup_off(2 * d + 2 + 1, 0);
    std::vector<uint64_t> nD(2 * d + 2, 0);
    for (int D = 0; D <= 2 * d && D <= l; D++) {
        tup_off[D] = (int)tup.size();
        uint64_t acc = 0;
        for (int a = 0; a <= D; a++)
            for (int b = 0; a + b <= D; b++) {
                const int cc = D - a - b;
                for (int e = 0; e <= l - D; e++) {
                    if (b + cc + e > d || a + cc + e > d)
                        continue;
                    const unsigned __int128 cnt =
                        (unsigned __int128)(fact[D] /
                                            (fact[a] * fact[b] * fact[cc])) *
                        (1ull << cc) * binom[(l - D) * (kMaxL + 1) + e] *
                        pow3[e];
                    PairTuple t{};
                    t.first = acc;
                    t.a = (uint8_t)a;
                    t.b = (uint8_t)b;
                    t.c = (uint8_t)cc;
                    t.e = (uint8_t)e;
                    t.n3 = (uint32_t)pow3[e];
                    t.ns = (uint32_t)binom[(l - D) * (kMaxL + 1) + e];
                    tup.push_back(t);
                    // work items per pair are 32-bit counts of 1024
                    if (cnt > ((unsigned __int128)1 << 40) ||
                        acc + (uint64_t)cnt > (1ull << 40))
                        return c->fail(PMS_EINVAL, "pair path: intersections "
                                       "of (%d,%d) too large", l, d);
                    acc += (uint64_t)cnt;
                }
            }
        nD[D] = acc;
    }
    for (int D = std::min(2 * d, l) + 1; D <= 2 * d + 2; D++)
        tup_off[D] = (int)tup.size();
    if (tup.size() > (size_t)kPairMaxTuples)
        return c->fail(PMS_EINVAL, "pair path: %zu intersection shapes of "
                       "(%d,%d) above %d", tup.size(), l, d, kPairMaxTuples);
    // multinomials (r; a, b, r-a-b) for r <= 2d <= 20: at most 3^20 < 2^32
    const int MD = kPairMaxD + 1;
    std::vector<uint32_t> multi((size_t)MD * MD * MD, 0);
    for (int r = 0; r <= kPairMaxD; r++)
        for (int a = 0; a <= r; a++)
            for (int b2 = 0; a + b2 <= r; b2++)
                multi[((size_t)r * MD + a) * MD + b2] =
                    (uint32_t)(fact[r] / (fact[a] * fact[b2] *
                                          fact[r - a - b2]));

    // device layout (the aux buffer): tables, counters, pair arrays
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t o_nD = take(nD.size() * 8);
    const size_t o_tup = take(std::max<size_t>(tup.size(), 1) *
                              sizeof(PairTuple));
    const size_t o_toff = take(tup_off.size() * 4);
    const size_t o_multi = take(multi.size() * 4);
    const size_t o_bin = take(binom.size() * 8);
    const size_t o_cnt = take(8 * 8);
    const size_t o_part = take((size_t)L * 4);
    const size_t o_pairs = take(LL * 8);
    const size_t o_chunks = take(LL * 4);
    const size_t o_pos = take((LL + 1) * 8);
    const size_t o_scan = take(scan_scratch_bytes(LL));
    int rc = c->alloc(c->aux, off);
    if (rc)
        return rc;
    char *b = (char *)c->aux.p;
    HIPCHK(c, hipMemcpyAsync(b + o_nD, nD.data(), nD.size() * 8,
                             hipMemcpyHostToDevice, st));
    if (!tup.empty())
        HIPCHK(c, hipMemcpyAsync(b + o_tup, tup.data(),
                                 tup.size() * sizeof(PairTuple),
                                 hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(b + o_toff, tup_off.data(), tup_off.size() * 4,
                             hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(b + o_multi, multi.data(), multi.size() * 4,
                             hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(b + o_bin, binom.data(), binom.size() * 8,
                             hipMemcpyHostToDevice, st));
    unsigned long long *cnt = (unsigned long long *)(b + o_cnt);
    HIPCHK(c, launch_fill_u64(cnt, 8, 0, st));

    PairJob J;
    J.planes = I.planes;
    J.nD = (const uint64_t *)(b + o_nD);
    J.tup = (const PairTuple *)(b + o_tup);
    J.tup_off = (const int *)(b + o_toff);
    J.multi = (const uint32_t *)(b + o_multi);
    J.binom = (const uint64_t *)(b + o_bin);
    J.ntup = (int)tup.size();
    J.partner = (const uint32_t *)(b + o_part);
    J.pairs = (uint2 *)(b + o_pairs);
    J.chunks = (uint32_t *)(b + o_chunks);
    J.npairs = cnt;
    J.ncand = cnt + 1;
    J.next = cnt + 2;
    J.tests = cnt + 3;
    J.qcount = cnt + 4;                 // cnt[4], cnt[5]: the two queues
    J.overflow = (unsigned int *)(cnt + 6);
    J.q[0] = J.q[1] = nullptr;
    J.qp[0] = J.qp[1] = nullptr;
    J.qcap = 0;
    J.pairs_cap = LL;
    J.item_pos = (const uint64_t *)(b + o_pos);
    J.item_pair = nullptr;
    J.heap = I.heap;
    J.heap_top = I.heap_top;
    J.heap_cap = I.heap_cap;
    J.n = n;
    J.L = L;
    J.l = l;
    J.d = d;
    const bool per_x = c->opt.pair_partner == 0 && n > 2 && n <= 65536;
    if (per_x)
        HIPCHK(c, launch_pair_partner(I.planes, n, L, (uint32_t *)(b + o_part),
                                      st));
    else
        HIPCHK(c, launch_fill_u32((unsigned int *)(b + o_part), L, 1u, st));
    HIPCHK(c, launch_pair_list(J, st));
    unsigned long long *hp = c->pinned + 4;
    HIPCHK(c, hipMemcpyAsync(hp, cnt, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const unsigned long long npairs = hp[0], ncand = hp[1];
    if (npairs >= (1ull << 32))   // work items name their pair in 32 bits
        return c->fail(PMS_ENOMEM, "pair path: %llu pairs", npairs);
    unsigned long long nitems = 0;
    if (npairs) {
        HIPCHK(c, launch_scan_u32(J.chunks, npairs, (uint64_t *)J.item_pos,
                                  b + o_scan, st));
        HIPCHK(c, hipMemcpyAsync(hp, J.item_pos + npairs, 8,
                                 hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        nitems = hp[0];
    }
    // Queues between strings: a batch of work items at a time, sized so
    // that even if every candidate passed s_3 the queue holds them; the
    // later strings run on the compacted queue, stage after stage, with no
    // host wait in between.
    const unsigned long long qcap = std::max<unsigned long long>(
        (unsigned long long)pair_chunk(),
        std::min<unsigned long long>(1ull << 26, ncand + pair_chunk()));
    // the two queues, then the pair of every work item
    const size_t q_bytes = 2 * qcap * (sizeof(uint2) + 2);
    if ((rc = c->alloc(c->alive, q_bytes + (nitems + 1) * 4)))
        return rc;
    J.q[0] = (uint2 *)c->alive.p;
    J.q[1] = J.q[0] + qcap;
    J.qp[0] = (uint16_t *)(J.q[1] + qcap);
    J.qp[1] = J.qp[0] + qcap;
    J.qcap = qcap;
    uint32_t *item_pair = (uint32_t *)((char *)c->alive.p + q_bytes);
    J.item_pair = item_pair;
    if (npairs)
        HIPCHK(c, launch_pair_items(J, npairs, item_pair, st));
    const unsigned long long per_batch = qcap / pair_chunk();
    const int grid = std::max(1, c->n_cu * c->pair_bpc);
    for (unsigned long long lo = 0; lo < nitems; lo += per_batch) {
        const unsigned long long hi = std::min(nitems, lo + per_batch);
        HIPCHK(c, launch_fill_u64(J.next, 1, lo, st));
        HIPCHK(c, launch_fill_u64(J.qcount, 1, 0, st));
        HIPCHK(c, launch_pair_filter(J, hi, npairs, grid, st));
        // stages 2..n-1; with s_2 as every partner the filter stage took
        // string 2, so stage 2 would only copy the queue
        int in = 0;
        for (int i = per_x ? 2 : 3; i < n; i++) {
            const int out = in ^ 1;
            HIPCHK(c, launch_fill_u64(J.qcount + out, 1, 0, st));
            HIPCHK(c, launch_pair_queue(J, i, J.q[in], J.qp[in], J.qcount + in,
                                        J.q[out], J.qp[out], J.qcount + out,
                                        grid, st));
            in = out;
        }
    }
    HIPCHK(c, hipMemcpyAsync(hp + 2, J.overflow, 4, hipMemcpyDeviceToHost,
                             st));
    HIPCHK(c, hipMemcpyAsync(hp, I.heap_top, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(hp + 1, J.tests, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if ((uint32_t)hp[2] != 0)
        return c->fail(PMS_EDEVICE, "pair path: candidate queue overflow");
    *found = hp[0];
    S.pairs = npairs;
    S.candidates = ncand;
    S.filter_tests = hp[1];
    S.main_launches = 2;
    return PMS_OK;
}

}  // namespace pms
