// k_pair.hip -- pair-based candidates (Observation 3.3 with q = n).
//
// A motif M has an l-mer x in s_1 and an l-mer y in s_2 within distance d,
// so d_H(x,y) <= 2d and M is in B(x,d) ∩ B(y,d). The candidates of a pair are
// enumerated directly: on the D positions where x and y differ, M takes x's
// letter (a of them), y's letter (b) or one of the 2 other letters (c); on
// the l-D positions where they agree it changes e of them (3 letters each);
// M is in the intersection iff b+c+e <= d and a+c+e <= d. A flat index over
// the intersection is unranked on the device into such a tuple (a,b,c,e),
// the colouring of the differing positions, the other-letter bits, the set
// of changed agreeing positions and their letters. Each candidate already
// has d-neighbours in s_1 and s_2; it is tested against s_3..s_n in order
// with the XOR/popcount Hamming form of Sec. 3.3.1 and early exit. A motif
// reached from several pairs is reported once per pair; the caller sorts
// and drops repeats.
#include "pms_internal.h"

namespace pms {

constexpr int kPairPer = 4;                    // candidates per thread
constexpr int kPairChunk = kTPB * kPairPer;    // candidates per work item

__global__ __launch_bounds__(kTPB) void
k_pair_list(PairJob J)
{
    const uint64_t g = (uint64_t)blockIdx.x * kTPB + threadIdx.x;
    const uint64_t L = (uint64_t)J.L;
    if (g >= L * L)
        return;
    const uint32_t j = (uint32_t)(g / L), k = (uint32_t)(g % L);
    const uint2 x = J.planes[j], y = J.planes[L + k];      // s_1, s_2
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

__device__ __forceinline__ uint64_t multinom(const uint64_t *fact, int n,
                                             int a, int b, int c)
{
    return fact[n] / (fact[a] * fact[b] * fact[c]);
}

__device__ __forceinline__ void set_letter(uint32_t &hi, uint32_t &lo, int p,
                                           uint32_t v)
{
    hi = (hi & ~(1u << p)) | (((v >> 1) & 1u) << p);
    lo = (lo & ~(1u << p)) | ((v & 1u) << p);
}

__global__ __launch_bounds__(kTPB) void
k_pair_filter(PairJob J, unsigned long long nitems, unsigned long long npairs)
{
    __shared__ unsigned long long s_item, s_pair, s_hc;
    const int tid = threadIdx.x;
    const uint32_t lmask = (J.l >= 32) ? ~0u : ((1u << J.l) - 1u);
    unsigned long long hc = 0;
    if (tid == 0)
        s_hc = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const unsigned long long it = atomicAdd(J.next, 1ull);
            s_item = it;
            // the pair whose chunk range holds the item
            unsigned long long lo = 0, hi = npairs - 1;
            if (it < nitems) {
                while (lo < hi) {
                    const unsigned long long mid = (lo + hi + 1) / 2;
                    if (J.item_pos[mid] <= it)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
            }
            s_pair = lo;
        }
        __syncthreads();
        const unsigned long long it = s_item;
        if (it >= nitems)
            break;
        const unsigned long long pi = s_pair;
        const uint2 pr = J.pairs[pi];
        const uint2 x = J.planes[pr.x], y = J.planes[(uint64_t)J.L + pr.y];
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
                if (J.tup[mid].first <= r)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const PairTuple T = J.tup[lo];
            uint64_t q = r - T.first;
            const uint64_t n3 = J.pow3[T.e];
            const uint64_t ns = J.binom[(J.l - D) * (kMaxL + 1) + T.e];
            uint64_t agl = q % n3;
            q /= n3;
            uint64_t ags = q % ns;
            q /= ns;
            uint64_t oth = q & ((1ull << T.c) - 1ull);
            uint64_t col = q >> T.c;
            // colour the differing positions in increasing order
            int ra = T.a, rb = T.b, rc = T.c, rem = D;
            uint32_t m = dm;
            while (m) {
                const int p = __ffs(m) - 1;
                m &= m - 1;
                rem--;
                const uint64_t n0 = ra ? multinom(J.fact, rem, ra - 1, rb, rc)
                                       : 0;
                if (col < n0) {
                    ra--;                                 // x's letter
                    continue;
                }
                col -= n0;
                const uint64_t n1 = rb ? multinom(J.fact, rem, ra, rb - 1, rc)
                                       : 0;
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
                const uint32_t w = (oth & 1ull) ? (z == 3u ? 2u : 3u)
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
                const uint64_t skip = J.binom[after * (kMaxL + 1) + re];
                if (ags < skip)
                    continue;
                ags -= skip;
                re--;
                const uint32_t xv = (((x.x >> p) & 1u) << 1) | ((x.y >> p) & 1u);
                const uint32_t w = 1u + (uint32_t)(agl % 3ull);
                agl /= 3ull;
                set_letter(ch[u], cl[u], p, xv ^ w);
            }
        }
        // strings s_3..s_n in order, early exit per string and per wave
        for (int i = 2; i < J.n; i++) {
            bool any = false;
#pragma unroll
            for (int u = 0; u < kPairPer; u++)
                any |= live[u];
            if (__ballot(any) == 0)
                break;
            const c_u64 *row = (const c_u64 *)(const void *)(
                J.planes + (size_t)i * J.L);
            bool hit[kPairPer];
#pragma unroll
            for (int u = 0; u < kPairPer; u++) {
                hit[u] = !live[u];
                hc += live[u] ? (unsigned long long)J.L : 0ull;
            }
            for (int y0 = 0; y0 < J.L; y0 += 8) {
                const int y1 = min(y0 + 8, J.L);
                for (int yy = y0; yy < y1; yy++) {
                    const unsigned long long v = row[yy];
                    const uint32_t vh = (uint32_t)v, vl = (uint32_t)(v >> 32);
#pragma unroll
                    for (int u = 0; u < kPairPer; u++)
                        hit[u] |= __popc((ch[u] ^ vh) | (cl[u] ^ vl)) <= J.d;
                }
                bool done = true;
#pragma unroll
                for (int u = 0; u < kPairPer; u++)
                    done &= hit[u];
                if (__all(done))
                    break;
            }
#pragma unroll
            for (int u = 0; u < kPairPer; u++)
                live[u] &= hit[u];
        }
#pragma unroll
        for (int u = 0; u < kPairPer; u++) {
            if (!live[u])
                continue;
            uint64_t code = 0;
            for (int p = 0; p < J.l; p++)
                code = (code << 2) | (((ch[u] >> p) & 1u) << 1) |
                       ((cl[u] >> p) & 1u);
            const unsigned long long at = atomicAdd(J.heap_top, 1ull);
            if (at < J.heap_cap)
                J.heap[at] = code;
        }
    }
    if (hc)
        atomicAdd(&s_hc, hc);
    __syncthreads();
    if (tid == 0 && s_hc)
        atomicAdd(J.tests, s_hc);
}

hipError_t launch_pair_list(const PairJob &J, hipStream_t st)
{
    const uint64_t tot = (uint64_t)J.L * J.L;
    hipLaunchKernelGGL(k_pair_list, dim3((unsigned)((tot + kTPB - 1) / kTPB)),
                       dim3(kTPB), 0, st, J);
    return hipGetLastError();
}

hipError_t launch_pair_filter(const PairJob &J, unsigned long long nitems,
                              unsigned long long npairs, int grid,
                              hipStream_t st)
{
    if (nitems == 0 || npairs == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pair_filter, dim3(grid), dim3(kTPB), 0, st, J,
                       nitems, npairs);
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
