// k_pair.hip -- pair-based candidates (Observation 3.3 with q = n).
//
// A motif M has an l-mer x in s_1 and an l-mer y in any other string s_j
// within distance d, so d_H(x,y) <= 2d and M is in B(x,d) ∩ B(y,d). The
// string j may be chosen per x (Observation 3.3 needs only that it is
// fixed before M is known): TraverStringRef takes for every x the string
// whose nearest l-mer is farthest from x, since the intersections shrink as
// d_H(x,y) grows (Sec. 3.2.3, string reordering); s_2 is the plain choice. The candidates of a pair are
// enumerated directly: on the D positions where x and y differ, M takes x's
// letter (a of them), y's letter (b) or one of the 2 other letters (c); on
// the l-D positions where they agree it changes e of them (3 letters each);
// M is in the intersection iff b+c+e <= d and a+c+e <= d. A flat index over
// the intersection is unranked on the device into such a tuple (a,b,c,e),
// the colouring of the differing positions, the other-letter bits, the set
// of changed agreeing positions and their letters. Each candidate already
// has d-neighbours in s_1 and s_j; it is tested against the other strings
// in input order with the XOR/popcount Hamming form of Sec. 3.3.1 and early
// exit. A motif reached from several pairs is reported once per pair; the
// caller sorts and drops repeats.
#include "pms_internal.h"

namespace pms {

constexpr int kPairPer = 4;                    // candidates per thread
constexpr int kPairChunk = kTPB * kPairPer;    // candidates per work item

// One workgroup per l-mer x of s_1: each wave takes strings 1, 1+kWaves,
// ...; the wave's minimum distance to a string comes from a wave
// reduction; the string with the largest minimum (lowest index on ties)
// is x's partner.
__global__ __launch_bounds__(kTPB) void
k_pair_partner(const uint2 *planes, int n, int L, uint32_t *partner)
{
    __shared__ uint32_t best[kWaves];
    const int x = blockIdx.x, lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint2 xv = planes[x];
    uint32_t key = 0;   // (min distance << 24) | (2^24 - 1 - j): max wins
    for (int j = 1 + wid; j < n; j += kWaves) {
        const uint2 *row = planes + (size_t)j * L;
        uint32_t md = 255;
        for (int k = lane; k < L; k += 64)
            md = min(md, (uint32_t)__popc((xv.x ^ row[k].x) | (xv.y ^ row[k].y)));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            md = min(md, (uint32_t)__shfl_xor((int)md, o, 64));
        key = max(key, (md << 24) | (0xFFFFFFu - (uint32_t)j));
    }
    if (lane == 0)
        best[wid] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t k = 0;
        for (int w = 0; w < kWaves; w++)
            k = max(k, best[w]);
        partner[x] = 0xFFFFFFu - (k & 0xFFFFFFu);
    }
}

hipError_t launch_pair_partner(const uint2 *planes, int n, int L,
                               uint32_t *partner, hipStream_t st)
{
    hipLaunchKernelGGL(k_pair_partner, dim3(L), dim3(kTPB), 0, st, planes, n,
                       L, partner);
    return hipGetLastError();
}

__global__ __launch_bounds__(kTPB) void
k_pair_list(PairJob J)
{
    const uint64_t g = (uint64_t)blockIdx.x * kTPB + threadIdx.x;
    const uint64_t L = (uint64_t)J.L;
    if (g >= L * L)
        return;
    const uint32_t j = (uint32_t)(g / L), k = (uint32_t)(g % L);
    const uint2 x = J.planes[j];                               // s_1
    const uint2 y = J.planes[(uint64_t)J.partner[j] * L + k];  // its partner
    const int D = __popc((x.x ^ y.x) | (x.y ^ y.y));
    if (D > 2 * J.d)
        return;
    const uint64_t nD = J.nD[D];
    if (nD == 0)
        return;
    const unsigned long long at = atomicAdd(J.npairs, 1ull);
    if (at >= J.pairs_cap)
        return;
    J.pairs[at] = make_uint2(j, k);
    J.chunks[at] = (uint32_t)((nD + kPairChunk - 1) / kPairChunk);
    atomicAdd(J.ncand, (unsigned long long)nD);
}

typedef __attribute__((address_space(4))) const unsigned long long c_u64;

__device__ __forceinline__ void set_letter(uint32_t &hi, uint32_t &lo, int p,
                                           uint32_t v)
{
    hi = (hi & ~(1u << p)) | (((v >> 1) & 1u) << p);
    lo = (lo & ~(1u << p)) | ((v & 1u) << p);
}

__device__ __forceinline__ uint32_t multi_at(const uint32_t *M, int r, int a,
                                             int b)
{
    return M[(r * (kPairMaxD + 1) + a) * (kPairMaxD + 1) + b];
}

// Test the candidates (planes ch/cl, kPairPer per thread) against one
// string's l-mers; on return live[u] holds "has a d-neighbour there".
// Wave-uniform l-mer reads, exit once every live candidate of the wave has
// one. Adds L per live candidate to hc (canonical test count).
__device__ __forceinline__ void scan_string(const PairJob &J, int i,
                                            const uint32_t *ch,
                                            const uint32_t *cl, bool *live,
                                            unsigned long long &hc)
{
    // vector loads of the wave-uniform l-mers (one address, broadcast):
    // they complete in order, so the compiler waits for each step's l-mers
    // one by one instead of for all of them at once, as it must for scalar
    // loads
    typedef const __attribute__((address_space(1))) unsigned long long g_u64;
    g_u64 *row = (g_u64 *)(const void *)(J.planes + (size_t)i * J.L);
    // running minimum distance per candidate (two l-mers per v_min3); a
    // dead candidate starts at 0 so that it never holds the wave back
    uint32_t mind[kPairPer];
#pragma unroll
    for (int u = 0; u < kPairPer; u++) {
        mind[u] = live[u] ? 255u : 0u;
        hc += live[u] ? (unsigned long long)J.L : 0ull;
    }
    const uint32_t dd = (uint32_t)J.d;
    int y0 = 0;
    // sixteen l-mers a step: enough tests per wait for their scalar loads
    for (; y0 + 16 <= J.L; y0 += 16) {
#pragma unroll
        for (int yy = 0; yy < 16; yy += 2) {
            const unsigned long long v0 = row[y0 + yy], v1 = row[y0 + yy + 1];
            const uint32_t h0 = (uint32_t)v0, l0 = (uint32_t)(v0 >> 32);
            const uint32_t h1 = (uint32_t)v1, l1 = (uint32_t)(v1 >> 32);
#pragma unroll
            for (int u = 0; u < kPairPer; u++)
                mind[u] = min(mind[u],
                              min((uint32_t)__popc((ch[u] ^ h0) | (cl[u] ^ l0)),
                                  (uint32_t)__popc((ch[u] ^ h1) | (cl[u] ^ l1))));
        }
        bool done = true;
#pragma unroll
        for (int u = 0; u < kPairPer; u++)
            done &= mind[u] <= dd;
        if (__all(done))
            break;
    }
    if (y0 + 16 > J.L) {
        for (int yy = y0; yy < J.L; yy++) {
            const unsigned long long v = row[yy];
            const uint32_t vh = (uint32_t)v, vl = (uint32_t)(v >> 32);
#pragma unroll
            for (int u = 0; u < kPairPer; u++)
                mind[u] = min(mind[u],
                              (uint32_t)__popc((ch[u] ^ vh) | (cl[u] ^ vl)));
        }
    }
#pragma unroll
    for (int u = 0; u < kPairPer; u++)
        live[u] &= mind[u] <= dd;
}

// Survivors of the block (live slots of every thread) to the next queue, or
// to the heap after the last string, with one atomic per block call: every
// block appends to the same counter, and one atomic per wave and slot made
// that counter the bottleneck of the whole path. Called by every thread of
// the block (it holds two barriers).
__device__ __forceinline__ void emit(const PairJob &J, bool last,
                                     const uint32_t *ch, const uint32_t *cl,
                                     const bool *live, const uint32_t *prt,
                                     uint2 *qout, uint16_t *qpout,
                                     unsigned long long *qcount)
{
    constexpr int kWaves = kTPB / 64;
    __shared__ unsigned int s_wcnt[kWaves];
    __shared__ unsigned long long s_wbase[kWaves];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned long long m[kPairPer];
    unsigned int cnt = 0;
#pragma unroll
    for (int u = 0; u < kPairPer; u++) {
        m[u] = __ballot(live[u]);
        cnt += (unsigned int)__popcll(m[u]);
    }
    if (lane == 0)
        s_wcnt[wid] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int tot = 0;
        for (int w = 0; w < kWaves; w++)
            tot += s_wcnt[w];
        unsigned long long base =
            tot ? atomicAdd(last ? J.heap_top : qcount,
                            (unsigned long long)tot)
                : 0ull;
        for (int w = 0; w < kWaves; w++) {
            s_wbase[w] = base;
            base += s_wcnt[w];
        }
    }
    __syncthreads();
    const unsigned long long below_mask =
        lane ? (~0ull >> (64 - lane)) : 0ull;
    unsigned long long at0 = s_wbase[wid];
#pragma unroll
    for (int u = 0; u < kPairPer; u++) {
        if (live[u]) {
            const unsigned long long at =
                at0 + (unsigned long long)__popcll(m[u] & below_mask);
            if (last) {
                uint64_t code = 0;
                for (int p = 0; p < J.l; p++)
                    code = (code << 2) | (((ch[u] >> p) & 1u) << 1) |
                           ((cl[u] >> p) & 1u);
                if (at < J.heap_cap)
                    J.heap[at] = code;
            } else if (at < J.qcap) {
                qout[at] = make_uint2(ch[u], cl[u]);
                qpout[at] = (uint16_t)prt[u];
            } else {
                atomicOr(J.overflow, 1u);
            }
        }
        at0 += (unsigned long long)__popcll(m[u]);
    }
}

// Candidates of the items [it0, it1) tested against s_3 (or straight to the
// heap when n = 2); the next item comes from *J.next, which starts at it0.
__global__ __launch_bounds__(kTPB) void
k_pair_filter(PairJob J, unsigned long long it1, unsigned long long npairs)
{
    __shared__ unsigned long long s_item, s_pair, s_hc;
    __shared__ PairTuple s_tup[kPairMaxTuples];
    const int tid = threadIdx.x;
    const uint32_t lmask = (J.l >= 32) ? ~0u : ((1u << J.l) - 1u);
    unsigned long long hc = 0;
    if (tid == 0)
        s_hc = 0;
    for (int i = tid; i < J.ntup; i += kTPB)
        s_tup[i] = J.tup[i];
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const unsigned long long it = atomicAdd(J.next, 1ull);
            s_item = it;
            // the pair whose chunk range holds the item
            s_pair = it < it1 ? J.item_pair[it] : 0ull;
        }
        __syncthreads();
        const unsigned long long it = s_item;
        if (it >= it1)
            break;
        const unsigned long long pi = s_pair;
        const uint2 pr = J.pairs[pi];
        const uint32_t prt = J.partner[pr.x];
        const uint2 x = J.planes[pr.x];
        const uint2 y = J.planes[(uint64_t)prt * J.L + pr.y];
        const uint32_t dm = (x.x ^ y.x) | (x.y ^ y.y);
        const int D = __popc(dm);
        const uint64_t nD = J.nD[D];
        const uint64_t c0 = (it - J.item_pos[pi]) * kPairChunk;
        const int t0 = J.tup_off[D], t1 = J.tup_off[D + 1];
        uint32_t ch[kPairPer], cl[kPairPer];
        bool live[kPairPer];
#pragma unroll
        for (int u = 0; u < kPairPer; u++) {
            ch[u] = x.x;
            cl[u] = x.y;
            const uint64_t r = c0 + (uint64_t)u * kTPB + tid;
            live[u] = r < nD;
            if (!live[u])
                continue;
            // tuple (a, b, c, e): the last one whose first index is <= r
            int lo = t0, hi = t1 - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (s_tup[mid].first <= r)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const PairTuple T = s_tup[lo];
            const uint64_t q64 = r - T.first;
            // index = ((colouring * 2^c + others) * C(l-D,e) + agreeing set)
            //         * 3^e + agreeing letters; every factor is < 2^32
            uint32_t agl, ags, oth, col;
            if (q64 < (1ull << 32)) {
                uint32_t q = (uint32_t)q64;
                agl = q % T.n3;
                q /= T.n3;
                ags = q % T.ns;
                q /= T.ns;
                oth = q & ((1u << T.c) - 1u);
                col = q >> T.c;
            } else {
                uint64_t q = q64;
                agl = (uint32_t)(q % T.n3);
                q /= T.n3;
                ags = (uint32_t)(q % T.ns);
                q /= T.ns;
                oth = (uint32_t)(q & ((1ull << T.c) - 1ull));
                col = (uint32_t)(q >> T.c);
            }
            // colour the differing positions in increasing order
            int ra = T.a, rb = T.b, rc = T.c, rem = D;
            uint32_t m = dm;
            while (m) {
                const int p = __ffs(m) - 1;
                m &= m - 1;
                rem--;
                const uint32_t n0 = ra ? multi_at(J.multi, rem, ra - 1, rb) : 0u;
                if (col < n0) {
                    ra--;                                 // x's letter
                    continue;
                }
                col -= n0;
                const uint32_t n1 = rb ? multi_at(J.multi, rem, ra, rb - 1) : 0u;
                const uint32_t xv = (((x.x >> p) & 1u) << 1) | ((x.y >> p) & 1u);
                const uint32_t yv = (((y.x >> p) & 1u) << 1) | ((y.y >> p) & 1u);
                if (col < n1) {
                    rb--;                                 // y's letter
                    set_letter(ch[u], cl[u], p, yv);
                    continue;
                }
                col -= n1;
                rc--;                                     // one of the others
                const uint32_t z = xv ^ yv;
                const uint32_t w = (oth & 1u) ? (z == 3u ? 2u : 3u)
                                              : (z == 1u ? 2u : 1u);
                oth >>= 1;
                set_letter(ch[u], cl[u], p, xv ^ w);
            }
            // change e of the agreeing positions (lexicographic unranking)
            int re = T.e, after = J.l - D;
            uint32_t am = ~dm & lmask;
            while (re > 0 && am) {
                const int p = __ffs(am) - 1;
                am &= am - 1;
                after--;
                const uint32_t skip =
                    (uint32_t)J.binom[after * (kMaxL + 1) + re];
                if (ags < skip)
                    continue;
                ags -= skip;
                re--;
                const uint32_t xv = (((x.x >> p) & 1u) << 1) | ((x.y >> p) & 1u);
                const uint32_t w = 1u + agl % 3u;
                agl /= 3u;
                set_letter(ch[u], cl[u], p, xv ^ w);
            }
        }
        // the first string other than s_1 and the partner here; the later
        // ones run on the compacted queue
        const int first = prt == 1u ? 2 : 1;
        uint32_t prts[kPairPer];
#pragma unroll
        for (int u = 0; u < kPairPer; u++)
            prts[u] = prt;
        if (J.n > 2)
            scan_string(J, first, ch, cl, live, hc);
        // with three strings or fewer this was the only one left
        emit(J, J.n <= 3, ch, cl, live, prts, J.q[0], J.qp[0], J.qcount);
    }
    if (hc)
        atomicAdd(&s_hc, hc);
    __syncthreads();
    if (tid == 0 && s_hc)
        atomicAdd(J.tests, s_hc);
}

// Queue stage i (2 <= i < n): the candidates that passed the earlier
// stages (qin, partners in qpin, count in *qin_count) against string i;
// survivors to qout (or the heap after the last string).
__global__ __launch_bounds__(kTPB) void
k_pair_queue(PairJob J, int i, const uint2 *qin, const uint16_t *qpin,
             const unsigned long long *qin_count, uint2 *qout,
             uint16_t *qpout, unsigned long long *qout_count)
{
    __shared__ unsigned long long s_hc;
    const int tid = threadIdx.x;
    unsigned long long hc = 0;
    if (tid == 0)
        s_hc = 0;
    const unsigned long long cnt = min(*qin_count, J.qcap);
    for (unsigned long long b0 = (unsigned long long)blockIdx.x * kPairChunk;
         b0 < cnt; b0 += (unsigned long long)gridDim.x * kPairChunk) {
        uint32_t ch[kPairPer], cl[kPairPer], prt[kPairPer];
        bool live[kPairPer], pass[kPairPer];
#pragma unroll
        for (int u = 0; u < kPairPer; u++) {
            const unsigned long long k = b0 + (unsigned long long)u * kTPB + tid;
            live[u] = k < cnt;
            const uint2 v = live[u] ? qin[k] : make_uint2(0u, 0u);
            ch[u] = v.x;
            cl[u] = v.y;
            prt[u] = live[u] ? (uint32_t)qpin[k] : 1u;
            // string i is the candidate's partner, or was tested in the
            // filter stage (string 2 for candidates whose partner is s_2):
            // it passes without a test
            pass[u] = live[u] && ((int)prt[u] == i ||
                                  (prt[u] == 1u && i == 2));
            live[u] &= !pass[u];
        }
        scan_string(J, i, ch, cl, live, hc);
#pragma unroll
        for (int u = 0; u < kPairPer; u++)
            live[u] |= pass[u];
        emit(J, i >= J.n - 1, ch, cl, live, prt, qout, qpout, qout_count);
    }
    if (hc)
        atomicAdd(&s_hc, hc);
    __syncthreads();
    if (tid == 0 && s_hc)
        atomicAdd(J.tests, s_hc);
}

hipError_t launch_pair_queue(const PairJob &J, int i, const uint2 *qin,
                             const uint16_t *qpin,
                             const unsigned long long *qin_count, uint2 *qout,
                             uint16_t *qpout, unsigned long long *qout_count,
                             int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_pair_queue, dim3(grid), dim3(kTPB), 0, st, J, i, qin,
                       qpin, qin_count, qout, qpout, qout_count);
    return hipGetLastError();
}

__global__ __launch_bounds__(kTPB) void
k_pair_items(PairJob J, unsigned long long npairs, uint32_t *item_pair)
{
    for (unsigned long long p = (unsigned long long)blockIdx.x * kTPB +
                                threadIdx.x;
         p < npairs; p += (unsigned long long)gridDim.x * kTPB)
        for (uint64_t it = J.item_pos[p]; it < J.item_pos[p + 1]; it++)
            item_pair[it] = (uint32_t)p;
}

hipError_t launch_pair_items(const PairJob &J, unsigned long long npairs,
                             uint32_t *item_pair, hipStream_t st)
{
    const unsigned long long blocks = (npairs + kTPB - 1) / kTPB;
    hipLaunchKernelGGL(k_pair_items,
                       dim3((unsigned)std::min<unsigned long long>(blocks,
                                                                   65535)),
                       dim3(kTPB), 0, st, J, npairs, item_pair);
    return hipGetLastError();
}

hipError_t launch_pair_list(const PairJob &J, hipStream_t st)
{
    const uint64_t tot = (uint64_t)J.L * J.L;
    hipLaunchKernelGGL(k_pair_list, dim3((unsigned)((tot + kTPB - 1) / kTPB)),
                       dim3(kTPB), 0, st, J);
    return hipGetLastError();
}

hipError_t launch_pair_filter(const PairJob &J, unsigned long long it1,
                              unsigned long long npairs, int grid,
                              hipStream_t st)
{
    if (npairs == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pair_filter, dim3(grid), dim3(kTPB), 0, st, J, it1,
                       npairs);
    return hipGetLastError();
}

int pair_chunk() { return kPairChunk; }

int pair_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pair_filter, kTPB,
                                                     0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

}  // namespace pms
