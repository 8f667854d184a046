// k_alpha.hip -- (l,d)-motifs over an arbitrary alphabet (2..32 letters).
//
// The problem is stated over any alphabet Sigma (Sec. 1.2.5); Table 3.1 gives
// the sphere size n_B(l,d) = sum_k C(l,k) (|Sigma|-1)^k. This is the
// sample-driven method (Observation 3.1 with q = n): every motif lies in the
// d-sphere of an l-mer x of s_1, so each candidate of each B(x,d) is tested
// against s_2..s_n in order and dropped at the first string without an
// l-mer within distance d. Letters are coded by their index in the
// alphabet; an l-mer is held as ceil(log2 |Sigma|) bit planes (plane b, bit
// p = bit b of letter p), the compression of Sec. 3.3.1 generalised, so that
// d_H = popcount(OR_b (a_b XOR c_b)).
//
// Candidates are not materialised: a flat index over the sphere is unranked
// into (k, position set, letter offsets) on the device; position p gets the
// letter (x[p] + offset) mod |Sigma|, offset in 1..|Sigma|-1. A motif reached
// from several x is reported once per x; the caller sorts and drops repeats.
#include "pms_internal.h"

namespace pms {

constexpr int kAlphaPlanes = 5;        // up to 32 letters
constexpr int kAlphaStride = 8;        // uint32 words per l-mer (aligned)
constexpr int kAlphaPer = 4;           // candidates per thread
constexpr int kAlphaChunk = kTPB * kAlphaPer;

// letters -> codes and bit planes. One thread per (string, offset): the
// l-mer starting there (if any), and the letter at that offset.
__global__ __launch_bounds__(kTPB) void
k_alpha_index(const uint8_t *seqs, const uint8_t *map, int n, int m, int l,
              int P, uint8_t *letters, uint32_t *planes,
              unsigned long long *bad)
{
    const uint64_t g = (uint64_t)blockIdx.x * kTPB + threadIdx.x;
    if (g >= (uint64_t)n * m)
        return;
    const int i = (int)(g / m), j = (int)(g % m);
    const uint8_t *s = seqs + (size_t)i * m;
    const uint8_t c = map[s[j]];
    letters[g] = c;
    if (c == 0xff)
        atomicMin(bad, (unsigned long long)g);
    const int L = m - l + 1;
    if (j >= L)
        return;
    uint32_t pl[kAlphaPlanes] = {0, 0, 0, 0, 0};
    for (int p = 0; p < l; p++) {
        const uint32_t v = map[s[j + p]];
#pragma unroll
        for (int b = 0; b < kAlphaPlanes; b++)
            pl[b] |= ((v >> b) & 1u) << p;
    }
    uint32_t *o = planes + ((size_t)i * L + j) * kAlphaStride;
#pragma unroll
    for (int b = 0; b < kAlphaPlanes; b++)
        o[b] = b < P ? pl[b] : 0u;
}

typedef __attribute__((address_space(4))) const uint32_t c_u32;

// Hamming distance between a candidate and an l-mer over 5 bit planes:
// popcount(OR_b (c_b XOR a_b)). v_bitop3 with truth table 0xF6 computes
// s0 | (s1 ^ s2) (table index s0*4 + s1*2 + s2), one instruction per plane
// after the first.
__device__ __forceinline__ uint32_t dist5(const uint32_t *c, uint32_t a0,
                                          uint32_t a1, uint32_t a2,
                                          uint32_t a3, uint32_t a4)
{
    uint32_t t = c[0] ^ a0;
    t = __builtin_amdgcn_bitop3_b32(t, c[1], a1, 0xF6);
    t = __builtin_amdgcn_bitop3_b32(t, c[2], a2, 0xF6);
    t = __builtin_amdgcn_bitop3_b32(t, c[3], a3, 0xF6);
    t = __builtin_amdgcn_bitop3_b32(t, c[4], a4, 0xF6);
    return (uint32_t)__popc(t);
}

__global__ __launch_bounds__(kTPB) void
k_alpha_filter(AlphaJob J, unsigned int *next, unsigned long long nitems)
{
    __shared__ uint8_t xl[kMaxL];
    __shared__ unsigned long long s_item;
    __shared__ unsigned long long s_hc;
    const int tid = threadIdx.x;
    unsigned long long hc = 0;   // this thread's canonical test count
    if (tid == 0)
        s_hc = 0;
    const uint64_t per_ref = (J.nb + kAlphaChunk - 1) / kAlphaChunk;
    for (;;) {
        __syncthreads();
        if (tid == 0)
            s_item = atomicAdd((unsigned long long *)next, 1ull);
        __syncthreads();
        const unsigned long long it = s_item;
        if (it >= nitems)
            break;
        const int ref = (int)(it / per_ref);
        const uint64_t c0 = (it % per_ref) * kAlphaChunk;
        if (tid < J.l)
            xl[tid] = J.letters[ref + tid];   // s_1 is row 0
        __syncthreads();
        const c_u32 *xp = (const c_u32 *)(const void *)(
            J.planes + (size_t)ref * kAlphaStride);
        uint32_t cp[kAlphaPer][kAlphaPlanes];
        bool live[kAlphaPer];
#pragma unroll
        for (int u = 0; u < kAlphaPer; u++) {
            const uint64_t r = c0 + (uint64_t)u * kTPB + tid;
            live[u] = r < J.nb;
#pragma unroll
            for (int b = 0; b < kAlphaPlanes; b++)
                cp[u][b] = xp[b];
            if (!live[u])
                continue;
            // unrank: weight k, position set, offsets in base sigma-1
            int k = 0;
            while (k < J.d && r >= J.cum[k + 1])
                k++;
            const uint64_t rr = r - J.cum[k];
            const uint64_t pr = rr / J.powr[k];
            uint64_t off = rr - pr * J.powr[k];
            uint32_t mask = J.posset[J.posoff[k] + pr];
            while (mask) {
                const int p = __ffs(mask) - 1;
                mask &= mask - 1;
                const uint32_t o = 1u + (uint32_t)(off % (uint64_t)(J.sigma - 1));
                off /= (uint64_t)(J.sigma - 1);
                uint32_t nl = xl[p] + o;
                nl = nl >= (uint32_t)J.sigma ? nl - J.sigma : nl;
#pragma unroll
                for (int b = 0; b < kAlphaPlanes; b++)
                    cp[u][b] = (cp[u][b] & ~(1u << p)) | (((nl >> b) & 1u) << p);
            }
        }
        // strings s_2..s_n in order, early exit per string and per wave
        for (int i = 1; i < J.n; i++) {
            bool any = false;
#pragma unroll
            for (int u = 0; u < kAlphaPer; u++)
                any |= live[u];
            if (__ballot(any) == 0)
                break;
            const c_u32 *row = (const c_u32 *)(const void *)(
                J.planes + (size_t)i * J.L * kAlphaStride);
            // running minimum distance per candidate; a dead candidate
            // starts at 0 so that it never holds the wave back
            uint32_t mind[kAlphaPer];
#pragma unroll
            for (int u = 0; u < kAlphaPer; u++) {
                mind[u] = live[u] ? 255u : 0u;
                hc += live[u] ? (unsigned long long)J.L : 0ull;
            }
            const uint32_t dd = (uint32_t)J.d;
            int y0 = 0;
            for (; y0 + 8 <= J.L; y0 += 8) {
#pragma unroll
                for (int y = 0; y < 8; y += 2) {
                    const c_u32 *yp = row + (size_t)(y0 + y) * kAlphaStride;
                    const c_u32 *zp = yp + kAlphaStride;
                    const uint32_t a0 = yp[0], a1 = yp[1], a2 = yp[2],
                                   a3 = yp[3], a4 = yp[4];
                    const uint32_t b0 = zp[0], b1 = zp[1], b2 = zp[2],
                                   b3 = zp[3], b4 = zp[4];
#pragma unroll
                    for (int u = 0; u < kAlphaPer; u++)
                        mind[u] = min(mind[u],
                                      min(dist5(cp[u], a0, a1, a2, a3, a4),
                                          dist5(cp[u], b0, b1, b2, b3, b4)));
                }
                bool done = true;
#pragma unroll
                for (int u = 0; u < kAlphaPer; u++)
                    done &= mind[u] <= dd;
                if (__all(done))
                    break;
            }
            if (y0 + 8 > J.L) {
                for (int y = y0; y < J.L; y++) {
                    const c_u32 *yp = row + (size_t)y * kAlphaStride;
                    const uint32_t a0 = yp[0], a1 = yp[1], a2 = yp[2],
                                   a3 = yp[3], a4 = yp[4];
#pragma unroll
                    for (int u = 0; u < kAlphaPer; u++)
                        mind[u] = min(mind[u],
                                      dist5(cp[u], a0, a1, a2, a3, a4));
                }
            }
#pragma unroll
            for (int u = 0; u < kAlphaPer; u++)
                live[u] &= mind[u] <= dd;
        }
        // survivors: base-sigma code, first letter in the top digit
#pragma unroll
        for (int u = 0; u < kAlphaPer; u++) {
            if (!live[u])
                continue;
            uint64_t code = 0;
            for (int p = 0; p < J.l; p++) {
                uint32_t v = 0;
#pragma unroll
                for (int b = 0; b < kAlphaPlanes; b++)
                    v |= ((cp[u][b] >> p) & 1u) << b;
                code = code * (uint64_t)J.sigma + v;
            }
            const unsigned long long at = atomicAdd(J.heap_top, 1ull);
            if (at < J.heap_cap)
                J.heap[at] = code;
        }
    }
    if (hc)
        atomicAdd(&s_hc, hc);
    __syncthreads();
    if (tid == 0 && s_hc)
        atomicAdd(J.hcanon, s_hc);
}

// 1 where a sorted array starts a new value.
__global__ __launch_bounds__(kTPB) void
k_unique_mark(const uint64_t *a, uint64_t n, uint32_t *flag)
{
    const uint64_t i = (uint64_t)blockIdx.x * kTPB + threadIdx.x;
    if (i < n)
        flag[i] = (i == 0 || a[i] != a[i - 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(kTPB) void
k_unique_scatter(const uint64_t *a, uint64_t n, const uint32_t *flag,
                 const uint64_t *pos, uint64_t *out)
{
    const uint64_t i = (uint64_t)blockIdx.x * kTPB + threadIdx.x;
    if (i < n && flag[i])
        out[pos[i]] = a[i];
}

hipError_t launch_alpha_index(const uint8_t *seqs, const uint8_t *map, int n,
                              int m, int l, int P, uint8_t *letters,
                              uint32_t *planes, unsigned long long *bad,
                              hipStream_t st)
{
    const uint64_t tot = (uint64_t)n * m;
    hipLaunchKernelGGL(k_alpha_index, dim3((unsigned)((tot + kTPB - 1) / kTPB)),
                       dim3(kTPB), 0, st, seqs, map, n, m, l, P, letters,
                       planes, bad);
    return hipGetLastError();
}

hipError_t launch_alpha_filter(const AlphaJob &J, unsigned int *next,
                               int grid, hipStream_t st)
{
    const uint64_t per_ref = (J.nb + kAlphaChunk - 1) / kAlphaChunk;
    const unsigned long long nitems = per_ref * (uint64_t)J.L;
    hipLaunchKernelGGL(k_alpha_filter, dim3(grid), dim3(kTPB), 0, st, J, next,
                       nitems);
    return hipGetLastError();
}

hipError_t launch_unique_count(const uint64_t *a, uint64_t n, uint32_t *flag,
                               uint64_t *pos, void *scan_scratch,
                               hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    const unsigned nb = (unsigned)((n + kTPB - 1) / kTPB);
    hipLaunchKernelGGL(k_unique_mark, dim3(nb), dim3(kTPB), 0, st, a, n, flag);
    return launch_scan_u32(flag, n, pos, scan_scratch, st);
}

hipError_t launch_unique_scatter(const uint64_t *a, uint64_t n,
                                 const uint32_t *flag, const uint64_t *pos,
                                 uint64_t *out, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    const unsigned nb = (unsigned)((n + kTPB - 1) / kTPB);
    hipLaunchKernelGGL(k_unique_scatter, dim3(nb), dim3(kTPB), 0, st, a, n,
                       flag, pos, out);
    return hipGetLastError();
}

int alpha_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_alpha_filter, kTPB,
                                                     0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

}  // namespace pms
