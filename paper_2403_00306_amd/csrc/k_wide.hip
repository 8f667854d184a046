// k_wide.hip -- long motifs, 1 <= l <= 64: the sample-driven path on 64-bit
// bit planes.
//
// Observation 3.1 with q = n: every motif lies in B(x, d) for some l-mer x
// of s_1. Each sphere is enumerated by unranking (weight k, then the set of
// k changed positions, then one of the 3 other bases at each), each
// candidate is tested against s_2, s_3, ... in input order with the
// bit-plane Hamming distance of Sec. 3.3.1, here on one 64-bit word per
// group, and dropped at the first string without an l-mer within d. A motif
// is kept only from the first l-mer of s_1 within distance d of it, so the
// survivors hold no repeats; they are sorted afterwards.
#include "pms_wide.h"

namespace pms {

constexpr int kWidePer = 4;                    // candidates per thread
constexpr int kWideChunk = kTPB * kWidePer;    // sphere indexes per item
constexpr int kWideGrab = 4;                   // items per counter update

__device__ __forceinline__ int wide_base(uint8_t ch)
{
    switch (ch) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
    }
}

// One thread per (string, offset). Every byte lies in some window (byte c in
// the one starting at min(c, L-1)), and a window reports its first bad byte,
// so the minimum over windows is the first bad byte of the input.
__global__ __launch_bounds__(kTPB) void
k_wide_index(const uint8_t *seqs, int n, int m, int l, ulonglong2 *planes,
             unsigned long long *bad)
{
    const int L = m - l + 1;
    const uint64_t idx = (uint64_t)blockIdx.x * kTPB + threadIdx.x;
    if (idx >= (uint64_t)n * (uint64_t)L)
        return;
    const int row = (int)(idx / (uint64_t)L);
    const int j = (int)(idx - (uint64_t)row * L);
    const uint8_t *s = seqs + (size_t)row * m + j;
    uint64_t hi = 0, lo = 0;
    int first_bad = -1;
    for (int p = 0; p < l; p++) {
        int b = wide_base(s[p]);
        if (b < 0) {
            if (first_bad < 0)
                first_bad = p;
            b = 0;
        }
        hi |= (uint64_t)(b >> 1) << p;
        lo |= (uint64_t)(b & 1) << p;
    }
    planes[idx] = make_ulonglong2(hi, lo);
    if (first_bad >= 0)
        atomicMin(bad, (unsigned long long)row * m + j + first_bad);
}

// d_H = popcount((hi_c ^ hi_y) | (lo_c ^ lo_y)) over the two 32-bit halves;
// v_bitop3 with truth table 0xF6 computes s0 | (s1 ^ s2) (table index
// s0*4 + s1*2 + s2), so a half costs an XOR, a v_bitop3 and a popcount.
__device__ __forceinline__ uint32_t dist64(ulonglong2 c, uint64_t yh,
                                           uint64_t yl)
{
    const uint32_t t0 = __builtin_amdgcn_bitop3_b32(
        (uint32_t)c.x ^ (uint32_t)yh, (uint32_t)c.y, (uint32_t)yl, 0xF6);
    const uint32_t t1 = __builtin_amdgcn_bitop3_b32(
        (uint32_t)(c.x >> 32) ^ (uint32_t)(yh >> 32), (uint32_t)(c.y >> 32),
        (uint32_t)(yl >> 32), 0xF6);
    return (uint32_t)__popc(t0) + (uint32_t)__popc(t1);
}

// The 32 bits of x to the even positions of a 64-bit word.
__device__ __forceinline__ uint64_t spread32(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// Planes (bit p = base p) to the code with base p in digit l-1-p.
__device__ __forceinline__ W128 wide_code(ulonglong2 c, int l)
{
    const uint64_t hr = __brevll(c.x) >> (64 - l);
    const uint64_t lr = __brevll(c.y) >> (64 - l);
    W128 w;
    w.lo = (spread32((uint32_t)hr) << 1) | spread32((uint32_t)lr);
    w.hi = (spread32((uint32_t)(hr >> 32)) << 1) |
           spread32((uint32_t)(lr >> 32));
    return w;
}

// Work items are (reference l-mer x of s_1, chunk of kWideChunk sphere
// indexes), taken kWideGrab at a time from a counter by persistent
// workgroups (every workgroup updates the same counter, so fewer updates
// keep it off the memory path).
__global__ __launch_bounds__(kTPB) void
k_wide_filter(WideJob J, unsigned long long *next, unsigned long long nitems)
{
    // the strings' l-mers are read with wave-uniform addresses: scalar loads
    typedef const __attribute__((address_space(4))) uint64_t c_u64;
    __shared__ unsigned long long s_item, s_hc;
    const int tid = threadIdx.x;
    if (tid == 0)
        s_hc = 0;
    unsigned long long hc = 0;
    const uint64_t per_ref = (J.nb + kWideChunk - 1) / kWideChunk;
    const uint32_t dd = (uint32_t)J.d;
    for (;;) {
        __syncthreads();
        if (tid == 0)
            s_item = atomicAdd(next, (unsigned long long)kWideGrab);
        __syncthreads();
        const unsigned long long it0 = s_item;
        if (it0 >= nitems)
            break;
        const unsigned long long it1 =
            min(it0 + (unsigned long long)kWideGrab, nitems);
        for (unsigned long long it = it0; it < it1; it++) {
            const int ref = (int)(it / per_ref);
            const uint64_t c0 = (it % per_ref) * kWideChunk;
            const ulonglong2 x = J.planes[ref];   // s_1 is row 0
            ulonglong2 cp[kWidePer];
            bool live[kWidePer];
#pragma unroll
            for (int u = 0; u < kWidePer; u++) {
                const uint64_t r = c0 + (uint64_t)u * kTPB + tid;
                live[u] = r < J.nb;
                cp[u] = x;
                if (!live[u])
                    continue;
                // unrank: weight k, position set, base-3 digits in
                // position order
                int k = 0;
                while (k < J.d && r >= J.cum[k + 1])
                    k++;
                const uint64_t rr = r - J.cum[k];
                const uint64_t pr = rr / J.pow3[k];
                uint64_t dig = rr - pr * J.pow3[k];
                uint64_t mask = J.posset[J.posoff[k] + pr];
                while (mask) {
                    const int p = __ffsll((unsigned long long)mask) - 1;
                    mask &= mask - 1;
                    const uint64_t delta = 1u + dig % 3u;
                    dig /= 3u;
                    cp[u].x ^= (delta >> 1) << p;
                    cp[u].y ^= (delta & 1u) << p;
                }
            }
            // strings s_2..s_n in order, early exit per string and per wave
            for (int i = 1; i < J.n; i++) {
                bool any = false;
#pragma unroll
                for (int u = 0; u < kWidePer; u++)
                    any |= live[u];
                if (__ballot(any) == 0)
                    break;
                const c_u64 *row = (const c_u64 *)(const void *)(
                    J.planes + (size_t)i * J.L);
                // running minimum distance per candidate; a dead candidate
                // starts at 0 so that it never holds the wave back
                uint32_t mind[kWidePer];
#pragma unroll
                for (int u = 0; u < kWidePer; u++) {
                    mind[u] = live[u] ? 255u : 0u;
                    hc += live[u] ? (unsigned long long)J.L : 0ull;
                }
                int y0 = 0;
                for (; y0 + 8 <= J.L; y0 += 8) {
#pragma unroll
                    for (int y = 0; y < 8; y += 2) {
                        const uint64_t ah = row[2 * (y0 + y)];
                        const uint64_t al = row[2 * (y0 + y) + 1];
                        const uint64_t bh = row[2 * (y0 + y) + 2];
                        const uint64_t bl = row[2 * (y0 + y) + 3];
#pragma unroll
                        for (int u = 0; u < kWidePer; u++)
                            mind[u] = min(mind[u], min(dist64(cp[u], ah, al),
                                                       dist64(cp[u], bh, bl)));
                    }
                    bool done = true;
#pragma unroll
                    for (int u = 0; u < kWidePer; u++)
                        done &= mind[u] <= dd;
                    if (__all(done))
                        break;
                }
                if (y0 + 8 > J.L) {
                    for (int y = y0; y < J.L; y++) {
                        const uint64_t ah = row[2 * y], al = row[2 * y + 1];
#pragma unroll
                        for (int u = 0; u < kWidePer; u++)
                            mind[u] = min(mind[u], dist64(cp[u], ah, al));
                    }
                }
#pragma unroll
                for (int u = 0; u < kWidePer; u++)
                    live[u] &= mind[u] <= dd;
            }
            // a motif is kept from the first l-mer of s_1 within d of it only
            const c_u64 *row0 = (const c_u64 *)(const void *)J.planes;
#pragma unroll
            for (int u = 0; u < kWidePer; u++) {
                if (!live[u])
                    continue;
                for (int j = 0; j < ref; j++)
                    if (dist64(cp[u], row0[2 * j], row0[2 * j + 1]) <= dd) {
                        live[u] = false;
                        break;
                    }
                if (!live[u])
                    continue;
                const unsigned long long at = atomicAdd(J.heap_top, 1ull);
                if (at < J.heap_cap)
                    J.heap[at] = wide_code(cp[u], J.l);
            }
        }
    }
    if (hc)
        atomicAdd(&s_hc, hc);
    __syncthreads();
    if (tid == 0 && s_hc)
        atomicAdd(J.hcanon, s_hc);
}

hipError_t launch_wide_index(const uint8_t *seqs, int n, int m, int l,
                             ulonglong2 *planes, unsigned long long *bad,
                             hipStream_t st)
{
    const uint64_t tot = (uint64_t)n * (uint64_t)(m - l + 1);
    hipLaunchKernelGGL(k_wide_index,
                       dim3((unsigned)((tot + kTPB - 1) / kTPB)), dim3(kTPB),
                       0, st, seqs, n, m, l, planes, bad);
    return hipGetLastError();
}

hipError_t launch_wide_filter(const WideJob &J, unsigned long long *next,
                              int grid, hipStream_t st)
{
    const uint64_t per_ref = (J.nb + kWideChunk - 1) / kWideChunk;
    const unsigned long long nitems = per_ref * (uint64_t)J.L;
    hipLaunchKernelGGL(k_wide_filter, dim3(grid), dim3(kTPB), 0, st, J, next,
                       nitems);
    return hipGetLastError();
}

int wide_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_wide_filter, kTPB,
                                                     0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

}  // namespace pms
