// k_filter.hip -- sample-driven path: d-neighbourhood candidates of the
// l-mers of s_1, filtered by XOR/popcount Hamming tests against s_2..s_n.
//
// Observation 3.1 with q = n: every motif lies in B(x, d) for some l-mer x
// of s_1, so the candidates are x XOR mu for every l-mer x of s_1 and every
// mu in Mask(l, d), the set of digit-wise XOR masks with at most d nonzero
// 2-bit digits (XOR of a base code with 1, 2 or 3 gives each of the three
// other bases, so x XOR Mask(l,d) is B(x,d), each element once; |Mask| =
// n_B(l,d) of Table 3.1).
//
// The filter is PMS8's "find motifs for some strings, then test them
// against the rest" (Sec. 3.2.4) with the Hamming test of Sec. 3.3.1 on bit
// planes: d_H = popcount((hi_a ^ hi_b) | (lo_a ^ lo_b)). A candidate is
// tested against s_2, s_3, ... in input order and dropped at the first
// string with no l-mer within distance d. Between strings the survivors of
// a workgroup are compacted so that every lane keeps testing live
// candidates.
//
// Each motif can be reached from several x. It is kept only from the first
// (lowest offset) l-mer x of s_1 within distance d of it, so the survivors
// are already free of repeats; they are sorted afterwards.
#include "pms_internal.h"

namespace pms {

constexpr int kFPer = 8;                    // candidates per thread
constexpr int kFBlock = kTPB * kFPer;       // candidates per block step
#ifndef PMS_FILTER_REFS
#define PMS_FILTER_REFS 8
#endif
constexpr int kFilterRefs = PMS_FILTER_REFS;  // references per block
constexpr int kFilterRefsMinMasks = 16 * (kFBlock / kFilterRefs);
static_assert(kFBlock % kFilterRefs == 0 && kFilterRefs <= kFBlock + 2,
              "filter block layout");

__device__ __forceinline__ uint64_t binom(int n, int k)
{
    if (k < 0 || k > n)
        return 0;
    uint64_t c = 1;
    for (int i = 0; i < k; i++)
        c = c * (uint64_t)(n - i) / (uint64_t)(i + 1);
    return c;
}

// Entry e of Mask(l, d) in bit-plane form. Entries are ordered by weight k,
// then by the rank of the position set (lexicographic), then by the base-3
// digits that pick the XOR value 1..3 at each chosen position.
__global__ void k_masks(int l, int d, uint2 *masks, uint64_t nb)
{
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb)
        return;
    uint64_t r = e;
    int k = 0;
    uint64_t p3 = 1;
    for (;;) {
        const uint64_t cnt = binom(l, k) * p3;
        if (r < cnt || k == d)
            break;
        r -= cnt;
        k++;
        p3 *= 3;
    }
    uint64_t comb = r / p3;
    uint64_t digs = r - comb * p3;
    uint32_t hi = 0, lo = 0;
    int left = k;
    for (int v = 0; v < l && left > 0; v++) {
        const uint64_t c = binom(l - 1 - v, left - 1);
        if (comb < c) {
            const uint32_t delta = 1u + (uint32_t)(digs % 3);
            digs /= 3;
            hi |= (delta >> 1) << v;
            lo |= (delta & 1u) << v;
            left--;
        } else {
            comb -= c;
        }
    }
    masks[e] = make_uint2(hi, lo);
}

hipError_t launch_masks(int l, int d, uint2 *masks, uint64_t nb,
                        hipStream_t st)
{
    const uint64_t blocks = (nb + 255) / 256;
    hipLaunchKernelGGL(k_masks, dim3((unsigned)blocks), dim3(256), 0, st, l,
                       d, masks, nb);
    return hipGetLastError();
}

struct FilterShared {
    uint2 cand[kFBlock];       // live candidates (bit planes)
    uint32_t ref[kFBlock];     // offset of the generating l-mer of s_1
    uint32_t hc[kFBlock + 2];  // canonical tests per reference in the block
    unsigned int red[kWaves];
    unsigned long long blk;
    unsigned long long off;
};

__device__ __forceinline__ unsigned int blk_exscan(unsigned int v,
                                                   unsigned int *red,
                                                   unsigned int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned int y = __shfl_up(x, o, 64);
        if (lane >= o)
            x += y;
    }
    __syncthreads();
    if (lane == 63)
        red[wid] = x;
    __syncthreads();
    unsigned int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
        if (w < wid)
            before += red[w];
        tot += red[w];
    }
    *total = uni(tot);
    return before + x - v;
}

// One string's l-mers read with wave-uniform addresses through the global
// address space (the loads broadcast one 16-byte row to the wave; on this
// loop they measured faster than scalar loads, which must all land before
// any use).
struct BRow {
    const __attribute__((address_space(1))) unsigned long long *p;
    __device__ __forceinline__ uint2 operator[](size_t i) const
    {
        const unsigned long long v = p[i];
        return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
    }
};

// Minimum distance from each of the thread's first K candidates to the
// l-mers of one string; the l-mer is the same for the whole wave. Returns
// the number of l-mers the wave tested (it stops once every live candidate
// has a hit).
template <int K>
__device__ __forceinline__ int scan_string(const BRow yp, int L,
                                            const uint2 *c, uint32_t *mind,
                                            int d, unsigned int live_mask)
{
    int j = 0;
    for (; j + 16 <= L; j += 16) {
#pragma unroll
        for (int u = 0; u < 16; u += 2) {
            const uint2 y0 = yp[j + u], y1 = yp[j + u + 1];
#pragma unroll
            for (int k = 0; k < K; k++) {
                const uint32_t h0 = __popc((c[k].x ^ y0.x) | (c[k].y ^ y0.y));
                const uint32_t h1 = __popc((c[k].x ^ y1.x) | (c[k].y ^ y1.y));
                mind[k] = min(mind[k], min(h0, h1));
            }
        }
        bool done = true;
#pragma unroll
        for (int k = 0; k < K; k++)
            done = done && (!((live_mask >> k) & 1u) || mind[k] <= (uint32_t)d);
        if (__all(done))
            return j + 16;
    }
    for (; j < L; j++) {
        const uint2 y = yp[j];
#pragma unroll
        for (int k = 0; k < K; k++)
            mind[k] = min(mind[k],
                          (uint32_t)__popc((c[k].x ^ y.x) | (c[k].y ^ y.y)));
    }
    return L;
}

// Candidate layout: with G = 1 a block takes kFBlock consecutive (x, e)
// in reference-major order (x = offset of the reference l-mer in s_1, e =
// index in Mask(l,d)); with G > 1 (large spheres) a block takes G
// consecutive references times kFBlock/G consecutive masks, so that each
// slice of the mask table is read once per G references instead of once
// per reference.
template <int G>
__global__ __launch_bounds__(kTPB) void
k_filter(const InstDev *inst, const uint2 *masks, uint64_t nb,
         unsigned long long *next_block, uint64_t *heap,
         unsigned long long *heap_top, unsigned long long heap_cap,
         unsigned long long *hc_per_ref, unsigned long long *hexec_out)
{
    __shared__ FilterShared sh;
    // tests executed by this thread: K candidate slots x l-mers scanned
    // (the same in every lane of a wave)
    unsigned long long hexec = 0;
    const InstDev I = *inst;
    const int tid = threadIdx.x;
    const int L = I.L, d = I.d, l = I.l;
    const PlaneRow x_planes = planes_row(I.planes, 0);   // row 0 = s_1
    const uint64_t total = (uint64_t)L * nb;
    // G > 1: blocks of G references x E masks, mask chunks inner
    constexpr uint32_t E = (uint32_t)(kFBlock / G);
    const uint64_t nec = (nb + E - 1) / E;
    const uint64_t nblocks =
        G == 1 ? (total + kFBlock - 1) / kFBlock
               : (uint64_t)((L + G - 1) / G) * nec;

    for (;;) {
        __syncthreads();
        if (tid == 0)
            sh.blk = atomicAdd(next_block, 1ull);
        __syncthreads();
        const uint64_t b = uni(sh.blk);
        if (b >= nblocks)
            break;
        const uint64_t f0 = b * kFBlock;
        const uint32_t x_first =
            G == 1 ? (uint32_t)(f0 / nb) : (uint32_t)(b / nec) * (uint32_t)G;
        const uint64_t e_first = G == 1 ? 0 : (b % nec) * E;
        for (int i = tid; i < kFBlock + 2; i += kTPB)
            sh.hc[i] = 0;

        // stage 0: build this thread's candidates
        uint2 c[kFPer];
        uint32_t ref[kFPer];
        unsigned int live = 0;
#pragma unroll
        for (int k = 0; k < kFPer; k++) {
            const uint32_t i = (uint32_t)(k * kTPB + tid);
            uint32_t x;
            uint64_t e;
            bool ok;
            if constexpr (G == 1) {
                const uint64_t f = f0 + i;
                ok = f < total;
                x = ok ? (uint32_t)(f / nb) : 0u;
                e = f - (uint64_t)x * nb;
            } else {
                x = x_first + i / E;
                e = e_first + i % E;
                ok = x < (uint32_t)L && e < nb;
            }
            c[k] = make_uint2(0, 0);
            ref[k] = 0;
            if (ok) {
                const uint2 xp = x_planes[x];
                const uint2 mu = masks[e];
                c[k] = make_uint2(xp.x ^ mu.x, xp.y ^ mu.y);
                ref[k] = x;
                live |= 1u << k;
            }
        }
        __syncthreads();   // hc cleared

        // an upper bound on the live slots (with G > 1 the empty ones of a
        // partial block are scattered; their live bits are clear)
        int nlive = G == 1 ? (int)min<uint64_t>((uint64_t)kFBlock, total - f0)
                           : kFBlock;
        for (int si = 1; si < I.n && nlive > 0; si++) {
            const BRow yp{(const __attribute__((address_space(1))) unsigned
                           long long *)(const void *)(I.planes +
                                                     (size_t)si * L)};
            uint32_t mind[kFPer];
#pragma unroll
            for (int k = 0; k < kFPer; k++) {
                mind[k] = 255;
                if ((live >> k) & 1u)
                    atomicAdd(&sh.hc[ref[k] - x_first], (uint32_t)L);
            }
            // after compaction the live candidates fill slots 0..kk-1: scan
            // only those (3 and 6 slots as well as powers of two: after the
            // first string about a third of a block is live, 3 of the 8
            // slots, which a 4-slot scan would pad by a third)
            const int kk = (nlive + kTPB - 1) / kTPB;
            if (__any(live != 0)) {
                if (kk <= 1)
                    hexec += (unsigned long long)scan_string<1>(
                        yp, L, c, mind, d, live);
                else if (kk <= 2)
                    hexec += 2ull * (unsigned long long)scan_string<2>(
                        yp, L, c, mind, d, live);
                else if (kk <= 3)
                    hexec += 3ull * (unsigned long long)scan_string<3>(
                        yp, L, c, mind, d, live);
                else if (kk <= 4)
                    hexec += 4ull * (unsigned long long)scan_string<4>(
                        yp, L, c, mind, d, live);
                else if (kk <= 6)
                    hexec += 6ull * (unsigned long long)scan_string<6>(
                        yp, L, c, mind, d, live);
                else
                    hexec += (unsigned long long)kFPer *
                             (unsigned long long)scan_string<kFPer>(
                                 yp, L, c, mind, d, live);
            }
            unsigned int keep = 0, nk = 0;
#pragma unroll
            for (int k = 0; k < kFPer; k++)
                if (((live >> k) & 1u) && mind[k] <= (uint32_t)d) {
                    keep |= 1u << k;
                    nk++;
                }
            // compact the survivors of the block and deal them out again
            unsigned int tot;
            const unsigned int pos = blk_exscan(nk, sh.red, &tot);
            unsigned int w = pos;
#pragma unroll
            for (int k = 0; k < kFPer; k++)
                if ((keep >> k) & 1u) {
                    sh.cand[w] = c[k];
                    sh.ref[w] = ref[k];
                    w++;
                }
            __syncthreads();
            nlive = (int)tot;
            live = 0;
#pragma unroll
            for (int k = 0; k < kFPer; k++) {
                const int i = k * kTPB + tid;
                if (i < nlive) {
                    c[k] = sh.cand[i];
                    ref[k] = sh.ref[i];
                    live |= 1u << k;
                }
            }
            __syncthreads();
        }

        // survivors of every string: keep each motif from its first x only
        unsigned int keep = 0, nk = 0;
#pragma unroll
        for (int k = 0; k < kFPer; k++) {
            if (!((live >> k) & 1u))
                continue;
            bool first = true;
            for (uint32_t xj = 0; xj < ref[k] && first; xj++) {
                const uint2 y = x_planes[xj];
                first = __popc((c[k].x ^ y.x) | (c[k].y ^ y.y)) > d;
            }
            if (first) {
                keep |= 1u << k;
                nk++;
            }
        }
        unsigned int tot;
        const unsigned int pos = blk_exscan(nk, sh.red, &tot);
        if (tid == 0 && tot)
            sh.off = atomicAdd(heap_top, (unsigned long long)tot);
        __syncthreads();
        if (tot) {
            const unsigned long long off = uni(sh.off);
            unsigned int w = pos;
#pragma unroll
            for (int k = 0; k < kFPer; k++)
                if ((keep >> k) & 1u) {
                    if (off + w < heap_cap) {
                        // planes -> code, first base in the top digit
                        uint64_t code = 0;
                        for (int p = 0; p < l; p++)
                            code = (code << 2) |
                                   ((((c[k].x >> p) & 1u) << 1) |
                                    ((c[k].y >> p) & 1u));
                        heap[off + w] = code;
                    }
                    w++;
                }
        }
        // flush the per-reference test counts of this block
        if (hc_per_ref) {
            const uint64_t f1 = min(f0 + kFBlock, total);
            const uint32_t x_last =
                G == 1 ? (uint32_t)((f1 - 1) / nb)
                       : min(x_first + (uint32_t)G, (uint32_t)L) - 1u;
            for (uint32_t x = x_first + tid; x <= x_last; x += kTPB)
                if (sh.hc[x - x_first])
                    atomicAdd(&hc_per_ref[x],
                              (unsigned long long)sh.hc[x - x_first]);
        }
    }
    if (hexec_out && (threadIdx.x & 63) == 0 && hexec)
        atomicAdd(hexec_out, 64ull * hexec);
}

hipError_t launch_filter(const InstDev *d_inst, const uint2 *masks,
                         uint64_t nb, unsigned long long *next_block,
                         uint64_t *heap, unsigned long long *heap_top,
                         unsigned long long heap_cap,
                         unsigned long long *hc_per_ref,
                         unsigned long long *hexec, int grid, hipStream_t st)
{
    // references per block: 8 where the sphere is large enough that the
    // blocks of 256 masks waste little at its end, else 1
    if (nb >= (uint64_t)kFilterRefsMinMasks)
        hipLaunchKernelGGL(k_filter<kFilterRefs>, dim3(grid), dim3(kTPB), 0,
                           st, d_inst, masks, nb, next_block, heap, heap_top,
                           heap_cap, hc_per_ref, hexec);
    else
        hipLaunchKernelGGL(k_filter<1>, dim3(grid), dim3(kTPB), 0, st, d_inst,
                           masks, nb, next_block, heap, heap_top, heap_cap,
                           hc_per_ref, hexec);
    return hipGetLastError();
}

// ---- quorum motifs (q < n) on the sample-driven path ---------------------
// Observation 3.1: the first string in which an (l,d,q)-motif has a
// d-neighbour is one of s_1..s_R, R = n-q+1, so the candidates are the
// spheres B(x,d) of the l-mers of those strings. Each candidate carries the
// number of strings in which it has no d-neighbour; the strings are tested
// in input order and a candidate is dropped
//   * at a hit in a string before its reference string (it is generated
//     again from that earlier string, which is where it is kept),
//   * once it has missed more than n-q strings;
// its own reference string passes untested. A survivor is kept only from
// the first offset of its reference string within distance d of it, so
// the output is free of repeats. The reference index and the miss count
// share one word: reference (R*L of them) in the low 27 bits, misses above.
constexpr uint32_t kQRefBits = 27;
constexpr uint32_t kQRefMask = (1u << kQRefBits) - 1u;

__global__ __launch_bounds__(kTPB) void
k_filter_quorum(const InstDev *inst, const uint2 *masks, uint64_t nb, int R,
                unsigned long long *next_block, uint64_t *heap,
                unsigned long long *heap_top, unsigned long long heap_cap)
{
    __shared__ FilterShared sh;
    const InstDev I = *inst;
    const int tid = threadIdx.x;
    const int L = I.L, d = I.d, l = I.l, n = I.n;
    const uint32_t T = (uint32_t)(I.n - I.q);    // misses a motif may have
    const PlaneRow all = planes_row(I.planes, 0);  // strings back to back
    const uint64_t total = (uint64_t)R * (uint64_t)L * nb;
    const uint64_t nblocks = (total + kFBlock - 1) / kFBlock;

    for (;;) {
        __syncthreads();
        if (tid == 0)
            sh.blk = atomicAdd(next_block, 1ull);
        __syncthreads();
        const uint64_t b = uni(sh.blk);
        if (b >= nblocks)
            break;
        const uint64_t f0 = b * kFBlock;
        uint2 c[kFPer];
        uint32_t ref[kFPer];
        unsigned int live = 0;
#pragma unroll
        for (int k = 0; k < kFPer; k++) {
            const uint64_t f = f0 + (uint64_t)k * kTPB + tid;
            c[k] = make_uint2(0, 0);
            ref[k] = 0;
            if (f < total) {
                const uint32_t x = (uint32_t)(f / nb);   // string*L + offset
                const uint64_t e = f - (uint64_t)x * nb;
                const uint2 xp = all[x];
                const uint2 mu = masks[e];
                c[k] = make_uint2(xp.x ^ mu.x, xp.y ^ mu.y);
                // misses start at the number of strings before x's string
                ref[k] = x | ((x / (uint32_t)L) << kQRefBits);
                live |= 1u << k;
            }
        }
        int nlive = (int)min<uint64_t>((uint64_t)kFBlock, total - f0);
        for (int si = 0; si < n && nlive > 0; si++) {
            const BRow yp{(const __attribute__((address_space(1))) unsigned
                           long long *)(const void *)(I.planes +
                                                     (size_t)si * L)};
            uint32_t mind[kFPer];
            unsigned int test = 0;
#pragma unroll
            for (int k = 0; k < kFPer; k++) {
                mind[k] = 255;
                const bool own = ((ref[k] & kQRefMask) / (uint32_t)L) ==
                                 (uint32_t)si;
                if (((live >> k) & 1u) && !own)
                    test |= 1u << k;
            }
            const int kk = (nlive + kTPB - 1) / kTPB;
            if (__any(test != 0)) {
                // slot counts as in k_filter
                if (kk <= 1)
                    scan_string<1>(yp, L, c, mind, d, test);
                else if (kk <= 2)
                    scan_string<2>(yp, L, c, mind, d, test);
                else if (kk <= 3)
                    scan_string<3>(yp, L, c, mind, d, test);
                else if (kk <= 4)
                    scan_string<4>(yp, L, c, mind, d, test);
                else if (kk <= 6)
                    scan_string<6>(yp, L, c, mind, d, test);
                else
                    scan_string<kFPer>(yp, L, c, mind, d, test);
            }
            unsigned int keep = 0, nk = 0;
#pragma unroll
            for (int k = 0; k < kFPer; k++) {
                if (!((live >> k) & 1u))
                    continue;
                bool stay = true;
                if ((test >> k) & 1u) {
                    const uint32_t rs = (ref[k] & kQRefMask) / (uint32_t)L;
                    const bool hit = mind[k] <= (uint32_t)d;
                    if ((uint32_t)si < rs) {
                        stay = !hit;   // counted among the misses already
                    } else if (!hit) {
                        const uint32_t ms = (ref[k] >> kQRefBits) + 1u;
                        ref[k] = (ref[k] & kQRefMask) | (ms << kQRefBits);
                        stay = ms <= T;
                    }
                }
                if (stay) {
                    keep |= 1u << k;
                    nk++;
                }
            }
            unsigned int tot;
            const unsigned int pos = blk_exscan(nk, sh.red, &tot);
            unsigned int w = pos;
#pragma unroll
            for (int k = 0; k < kFPer; k++)
                if ((keep >> k) & 1u) {
                    sh.cand[w] = c[k];
                    sh.ref[w] = ref[k];
                    w++;
                }
            __syncthreads();
            nlive = (int)tot;
            live = 0;
#pragma unroll
            for (int k = 0; k < kFPer; k++) {
                const int i = k * kTPB + tid;
                if (i < nlive) {
                    c[k] = sh.cand[i];
                    ref[k] = sh.ref[i];
                    live |= 1u << k;
                }
            }
            __syncthreads();
        }
        // keep each motif from the first offset of its reference string
        unsigned int keep = 0, nk = 0;
#pragma unroll
        for (int k = 0; k < kFPer; k++) {
            if (!((live >> k) & 1u))
                continue;
            const uint32_t x = ref[k] & kQRefMask;
            const uint32_t row0 = x - x % (uint32_t)L;
            bool first = true;
            for (uint32_t xj = row0; xj < x && first; xj++) {
                const uint2 y = all[xj];
                first = __popc((c[k].x ^ y.x) | (c[k].y ^ y.y)) > d;
            }
            if (first) {
                keep |= 1u << k;
                nk++;
            }
        }
        unsigned int tot;
        const unsigned int pos = blk_exscan(nk, sh.red, &tot);
        if (tid == 0 && tot)
            sh.off = atomicAdd(heap_top, (unsigned long long)tot);
        __syncthreads();
        if (tot) {
            const unsigned long long off = uni(sh.off);
            unsigned int w = pos;
#pragma unroll
            for (int k = 0; k < kFPer; k++)
                if ((keep >> k) & 1u) {
                    if (off + w < heap_cap) {
                        uint64_t code = 0;
                        for (int p = 0; p < l; p++)
                            code = (code << 2) |
                                   ((((c[k].x >> p) & 1u) << 1) |
                                    ((c[k].y >> p) & 1u));
                        heap[off + w] = code;
                    }
                    w++;
                }
        }
    }
}

hipError_t launch_filter_quorum(const InstDev *d_inst, const uint2 *masks,
                                uint64_t nb, int R,
                                unsigned long long *next_block, uint64_t *heap,
                                unsigned long long *heap_top,
                                unsigned long long heap_cap, int grid,
                                hipStream_t st)
{
    hipLaunchKernelGGL(k_filter_quorum, dim3(grid), dim3(kTPB), 0, st, d_inst,
                       masks, nb, R, next_block, heap, heap_top, heap_cap);
    return hipGetLastError();
}

uint32_t filter_quorum_max_refs() { return kQRefMask; }

int filter_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, k_filter<kFilterRefs>, kTPB, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

// ---- calibration: the Hamming-test instruction mix at full occupancy ----
// Each thread holds kCalCand candidates and kCalY l-mers in registers and
// takes the minimum distance of every candidate to every l-mer, `iters`
// times over (the l-mers made opaque per round so that no round can be
// folded away). A test is the filter's: v_xor, v_bitop3 (xor + or), v_bcnt
// and half a v_min3, i.e. 3.5 VALU ops; nothing else runs in the loop.
constexpr int kCalCand = 8, kCalY = 16;

__global__ __launch_bounds__(kTPB) void
k_test_rate(int iters, uint32_t seed, unsigned int *sink)
{
    uint32_t cx[kCalCand], cy[kCalCand], yx[kCalY], yy[kCalY];
    const uint32_t g = blockIdx.x * kTPB + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kCalCand; k++) {
        cx[k] = (g + (uint32_t)k) * 0x9E3779B9u ^ seed;
        cy[k] = (g ^ (uint32_t)k) * 0x85EBCA6Bu;
    }
#pragma unroll
    for (int j = 0; j < kCalY; j++) {
        yx[j] = (uint32_t)j * 0xC2B2AE35u ^ seed;
        yy[j] = (uint32_t)j * 0x27D4EB2Fu;
    }
    uint32_t mind[kCalCand];
#pragma unroll
    for (int k = 0; k < kCalCand; k++)
        mind[k] = 255;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int j = 0; j < kCalY; j++)
            asm volatile("" : "+v"(yx[j]), "+v"(yy[j]));
#pragma unroll
        for (int j = 0; j < kCalY; j += 2) {
#pragma unroll
            for (int k = 0; k < kCalCand; k++) {
                const uint32_t h0 = __popc((cx[k] ^ yx[j]) | (cy[k] ^ yy[j]));
                const uint32_t h1 =
                    __popc((cx[k] ^ yx[j + 1]) | (cy[k] ^ yy[j + 1]));
                mind[k] = min(mind[k], min(h0, h1));
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kCalCand; k++)
        acc += mind[k];
    if (acc == 0xFFFFFFFFu)   // never true; keeps the work observable
        atomicAdd(sink, acc);
}

hipError_t launch_test_rate(int grid, int iters, uint32_t seed,
                            unsigned int *sink, hipStream_t st)
{
    hipLaunchKernelGGL(k_test_rate, dim3(grid), dim3(kTPB), 0, st, iters,
                       seed, sink);
    return hipGetLastError();
}

int test_rate_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_test_rate, kTPB,
                                                     0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

uint64_t test_rate_tests_per_thread(int iters)
{
    return (uint64_t)iters * (uint64_t)(kCalCand * kCalY);
}

// LDS calibration: single-bit 32-bit atomic ORs, the tile kernels' mark, at
// their occupancy (512-thread workgroups, 32 KiB of LDS each, four per CU).
// Within each half wave the 32 lanes hit 32 different banks. Every index is
// masked into the array.
constexpr int kLdsCalWords = 8192;
constexpr int kLdsCalTPB = 512;
constexpr int kLdsCalUnroll = 16;

__global__ __launch_bounds__(kLdsCalTPB, kLdsCalTPB / 64) void
k_lds_rate(int iters, unsigned int *sink)
{
    __shared__ unsigned int buf[kLdsCalWords];
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < (uint32_t)kLdsCalWords; i += kLdsCalTPB)
        buf[i] = 0;
    __syncthreads();
    uint32_t off = ((tid >> 6) * 1024u + (tid & 63u)) & (kLdsCalWords - 1);
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int k = 0; k < kLdsCalUnroll; k++)
            atomicOr(&buf[(off + 64u * (uint32_t)k) & (kLdsCalWords - 1)],
                     1u << ((uint32_t)(it + k) & 31u));
        off = (off + 1024u) & (kLdsCalWords - 1);
    }
    __syncthreads();
    if (buf[tid] == 0x12345678u)   // never true; keeps the ORs observable
        atomicAdd(sink, 1u);
}

hipError_t launch_lds_rate(int grid, int iters, unsigned int *sink,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_lds_rate, dim3(grid), dim3(kLdsCalTPB), 0, st, iters,
                       sink);
    return hipGetLastError();
}

int lds_rate_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_lds_rate,
                                                     kLdsCalTPB, 0) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

uint64_t lds_rate_ors_per_block(int iters)
{
    return (uint64_t)iters * kLdsCalUnroll * kLdsCalTPB;
}

}  // namespace pms
