// k_scan.hip -- survivor compaction into the sorted motif set.
//
// The result is a set (Definition 5 asks for all motifs; duplicates carry
// no information), returned ascending. The tile kernels write each tile's
// survivors, already ascending, to a heap in whatever order tiles finish;
// an exclusive scan of the per-tile counts in tile order then gives every
// tile its final position, and an ordered gather moves the blocks there.
// The sample-driven filter path produces its survivors in no particular
// order, so it sorts them (LSD radix sort on device, 8 bits per pass).
#include "pms_wide.h"

#include <algorithm>

namespace pms {

constexpr int kScanPer = 16;
constexpr int kScanTile = kTPB * kScanPer;   // 4096 elements per block

__device__ __forceinline__ unsigned long long
wave_incl_scan64(unsigned long long x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long y = __shfl_up(x, o, 64);
        if (lane >= o)
            x += y;
    }
    return x;
}

// Exclusive prefix over the workgroup (thread order); *total = sum.
__device__ __forceinline__ unsigned long long
block_exscan64(unsigned long long v, unsigned long long *red,
               unsigned long long *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long x = wave_incl_scan64(v);
    __syncthreads();
    if (lane == 63)
        red[wid] = x;
    __syncthreads();
    unsigned long long before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
        if (w < wid)
            before += red[w];
        tot += red[w];
    }
    *total = tot;
    return before + x - v;
}

__global__ __launch_bounds__(kTPB) void k_scan_reduce(const uint32_t *in,
                                                      uint64_t n,
                                                      uint64_t *bsum)
{
    __shared__ unsigned long long red[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    unsigned long long s = 0;
    for (int k = 0; k < kScanPer; k++) {
        const uint64_t i = base + (uint64_t)k * kTPB + threadIdx.x;
        if (i < n)
            s += in[i];
    }
    unsigned long long tot;
    block_exscan64(s, red, &tot);
    if (threadIdx.x == 0)
        bsum[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of nb block sums in place; bsum[nb] = total.
__global__ __launch_bounds__(kTPB) void k_scan_top(uint64_t *bsum,
                                                   uint64_t nb)
{
    __shared__ unsigned long long red[kWaves];
    unsigned long long carry = 0;
    for (uint64_t c = 0; c < nb; c += kTPB) {
        const uint64_t i = c + threadIdx.x;
        const unsigned long long v = i < nb ? bsum[i] : 0;
        unsigned long long tot;
        const unsigned long long ex = block_exscan64(v, red, &tot);
        if (i < nb)
            bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0)
        bsum[nb] = carry;
}

// out[i] = sum of in[0..i); out[n] = total. Thread t of a block owns 16
// consecutive elements.
__global__ __launch_bounds__(kTPB) void k_scan_down(const uint32_t *in,
                                                    uint64_t n,
                                                    const uint64_t *bsum,
                                                    uint64_t *out)
{
    __shared__ unsigned long long red[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile +
                          (uint64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    unsigned long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; k++) {
        const uint64_t i = base + k;
        v[k] = i < n ? in[i] : 0u;
        s += v[k];
    }
    unsigned long long tot;
    unsigned long long run = bsum[blockIdx.x] + block_exscan64(s, red, &tot);
#pragma unroll
    for (int k = 0; k < kScanPer; k++) {
        const uint64_t i = base + k;
        if (i < n)
            out[i] = run;
        run += v[k];
        if (i + 1 == n)
            out[n] = run;
    }
}

size_t scan_scratch_bytes(uint64_t n)
{
    return sizeof(uint64_t) * ((n + kScanTile - 1) / kScanTile + 1);
}

hipError_t launch_scan_u32(const uint32_t *in, uint64_t n, uint64_t *out,
                           void *scratch, hipStream_t st)
{
    if (n == 0) {
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kTPB), 0, st, out,
                           (uint64_t)0);
        return hipGetLastError();
    }
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    uint64_t *bsum = (uint64_t *)scratch;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kTPB), 0, st,
                       in, n, bsum);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kTPB), 0, st, bsum, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kTPB), 0, st,
                       in, n, bsum, out);
    return hipGetLastError();
}

// Move every tile's block of codes from the heap to its final position.
// Small blocks are copied by one thread (in the groups with blockIdx.y 0);
// large ones by whole groups, each of the gridDim.y groups that share a
// blockIdx.x taking an interleaved slice.
__global__ __launch_bounds__(kTPB) void
k_gather(const uint32_t *tile_cnt, const uint64_t *heap_off,
         const uint64_t *tile_pos, const uint64_t *heap, uint64_t ntiles,
         uint64_t *out, unsigned long long cap, unsigned long long heap_cap)
{
    __shared__ uint64_t big[kTPB];
    __shared__ int nbig;
    for (uint64_t c0 = (uint64_t)blockIdx.x * kTPB; c0 < ntiles;
         c0 += (uint64_t)gridDim.x * kTPB) {
        if (threadIdx.x == 0)
            nbig = 0;
        __syncthreads();
        const uint64_t t = c0 + threadIdx.x;
        if (t < ntiles) {
            const uint32_t cnt = tile_cnt[t];
            if (cnt > 0) {
                const uint64_t pos = tile_pos[t];
                // a tile whose block did not fit in the heap wrote nothing;
                // the caller sees the overflow and runs again
                if (pos + cnt <= cap && heap_off[t] + cnt <= heap_cap) {
                    if (cnt <= 32) {
                        if (blockIdx.y == 0) {
                            const uint64_t src = heap_off[t];
                            for (uint32_t i = 0; i < cnt; i++)
                                out[pos + i] = heap[src + i];
                        }
                    } else {
                        big[atomicAdd(&nbig, 1)] = t;
                    }
                }
            }
        }
        __syncthreads();
        const int nb = nbig;
        for (int b = 0; b < nb; b++) {
            const uint64_t tt = big[b];
            const uint32_t cnt = tile_cnt[tt];
            const uint64_t src = heap_off[tt], dst = tile_pos[tt];
            // the blockIdx.y-th of gridDim.y interleaved slices
            for (uint32_t i = blockIdx.y * kTPB + threadIdx.x; i < cnt;
                 i += kTPB * gridDim.y)
                out[dst + i] = heap[src + i];
        }
        __syncthreads();
    }
}

hipError_t launch_gather(const uint32_t *tile_cnt, const uint64_t *heap_off,
                         const uint64_t *tile_pos, const uint64_t *heap,
                         uint64_t ntiles, uint64_t *out,
                         unsigned long long out_cap,
                         unsigned long long heap_cap, hipStream_t st)
{
    if (ntiles == 0)
        return hipSuccess;
    uint64_t blocks = (ntiles + kTPB - 1) / kTPB;
    if (blocks > 4096)
        blocks = 4096;
    // few tiles (possibly large ones): split each large tile's copy over
    // up to 64 blocks so that the grid still has ~4096 blocks
    const unsigned ys = (unsigned)std::max<uint64_t>(
        1, std::min<uint64_t>(64, 4096 / blocks));
    hipLaunchKernelGGL(k_gather, dim3((unsigned)blocks, ys), dim3(kTPB), 0, st,
                       tile_cnt, heap_off, tile_pos, heap, ntiles, out,
                       out_cap, heap_cap);
    return hipGetLastError();
}

// ranges[2i] = first output index of instance i, ranges[2i+1] = its count.
__global__ void k_ranges(const InstDev *insts, int ninst,
                         const uint64_t *tile_pos, uint64_t *ranges)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninst)
        return;
    const uint64_t b = insts[i].tile_base;
    const uint64_t e = b + insts[i].ntiles;
    ranges[2 * i] = tile_pos[b];
    ranges[2 * i + 1] = tile_pos[e] - tile_pos[b];
}

hipError_t launch_ranges(const InstDev *d_insts, int ninst,
                         const uint64_t *tile_pos, uint64_t *ranges,
                         hipStream_t st)
{
    if (ninst <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_ranges, dim3((ninst + 255) / 256), dim3(256), 0, st,
                       d_insts, ninst, tile_pos, ranges);
    return hipGetLastError();
}

// ---- sorting --------------------------------------------------------------
// Keys are 64-bit codes or, for long motifs, 128-bit codes (high word
// first); SortKey gives the digit, the order and the padding of each.

template <class K>
struct SortKey;

template <>
struct SortKey<uint64_t> {
    static constexpr int kSmall = 4096;   // one-workgroup sort up to this
    __device__ static uint32_t digit(uint64_t k, int shift)
    {
        return (uint32_t)(k >> shift) & 255u;
    }
    __device__ static bool less(uint64_t a, uint64_t b) { return a < b; }
    __device__ static uint64_t pad() { return ~0ull; }
};

template <>
struct SortKey<W128> {
    static constexpr int kSmall = 2048;   // 32 KiB of LDS
    __device__ static uint32_t digit(const W128 &k, int shift)
    {
        return (uint32_t)(shift < 64 ? k.lo >> shift : k.hi >> (shift - 64)) &
               255u;
    }
    __device__ static bool less(const W128 &a, const W128 &b)
    {
        return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
    }
    __device__ static W128 pad() { return W128{~0ull, ~0ull}; }
};

// Bitonic sort of n <= SortKey<K>::kSmall keys in one workgroup (padding
// sorts last).
template <class K>
__global__ __launch_bounds__(kTPB) void k_sort_small(K *keys, uint64_t n)
{
    typedef SortKey<K> S;
    __shared__ K a[S::kSmall];
    int N = 1;
    while ((uint64_t)N < n)
        N <<= 1;
    for (int i = threadIdx.x; i < N; i += kTPB)
        a[i] = (uint64_t)i < n ? keys[i] : S::pad();
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < N; i += kTPB) {
                const int p = i ^ j;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const K x = a[i], y = a[p];
                    if (S::less(y, x) == up) {
                        a[i] = y;
                        a[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; (uint64_t)i < n; i += kTPB)
        keys[i] = a[i];
}

// Per-block digit histograms, digit-major: hist[digit * nb + block].
template <class K>
__global__ __launch_bounds__(kTPB) void k_rs_hist(const K *keys, uint64_t n,
                                                  int shift, uint32_t *hist,
                                                  uint64_t nb)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    for (int k = 0; k < kScanPer; k++) {
        const uint64_t i = base + (uint64_t)k * kTPB + threadIdx.x;
        if (i < n)
            atomicAdd(&cnt[SortKey<K>::digit(keys[i], shift)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: keys of a block keep their relative order within each
// digit. Per round of 256 keys: peers with the same digit inside a wave are
// found with 8 ballots; waves are ordered through per-wave digit counts.
template <class K>
__global__ __launch_bounds__(kTPB) void
k_rs_scatter(const K *in, K *out, uint64_t n, int shift, const uint64_t *offs,
             uint64_t nb)
{
    __shared__ unsigned long long base[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int tid = threadIdx.x, wid = tid >> 6;
    base[tid] = offs[(uint64_t)tid * nb + blockIdx.x];
    for (int w = 0; w < kWaves; w++)
        wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanTile;
    for (int k = 0; k < kScanPer; k++) {
        const uint64_t i = b0 + (uint64_t)k * kTPB + tid;
        const bool valid = i < n;
        const K key = valid ? in[i] : K{};
        const uint32_t dig = SortKey<K>::digit(key, shift);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (dig >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
            (uint32_t)(peers >> 32),
            __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
        if (valid && rank == 0)
            wcnt[wid][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            unsigned long long pre = 0;
            for (int w = 0; w < wid; w++)
                pre += wcnt[w][dig];
            out[base[dig] + pre + rank] = key;
        }
        unsigned long long add = 0;
        for (int w = 0; w < kWaves; w++)
            add += wcnt[w][tid];
        __syncthreads();
        base[tid] += add;
        for (int w = 0; w < kWaves; w++)
            wcnt[w][tid] = 0;
        __syncthreads();
    }
}

// Scratch: temp keys (n), histogram (256*nb u32), offsets (256*nb+1 u64),
// scan scratch.
static size_t pad64(size_t b) { return (b + 63) / 64 * 64 + 64; }

template <class K>
static size_t sort_scratch(uint64_t n)
{
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    const uint64_t h = 256 * nb;
    return pad64(sizeof(K) * n) + pad64(sizeof(uint32_t) * h) +
           pad64(sizeof(uint64_t) * (h + 1)) + scan_scratch_bytes(h);
}

template <class K>
static hipError_t sort_keys(K *keys, uint64_t n, int key_bits, void *scratch,
                            hipStream_t st)
{
    if (n <= 1)
        return hipSuccess;
    if (n <= (uint64_t)SortKey<K>::kSmall) {
        hipLaunchKernelGGL(k_sort_small<K>, dim3(1), dim3(kTPB), 0, st, keys,
                           n);
        return hipGetLastError();
    }
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    const uint64_t h = 256 * nb;
    char *p = (char *)scratch;
    K *tmp = (K *)p;
    p += pad64(sizeof(K) * n);
    uint32_t *hist = (uint32_t *)p;
    p += pad64(sizeof(uint32_t) * h);
    uint64_t *offs = (uint64_t *)p;
    p += pad64(sizeof(uint64_t) * (h + 1));
    void *sscr = p;
    K *src = keys, *dst = tmp;
    const int passes = (key_bits + 7) / 8;
    for (int ps = 0; ps < passes; ps++) {
        const int shift = 8 * ps;
        hipLaunchKernelGGL(k_rs_hist<K>, dim3((unsigned)nb), dim3(kTPB), 0,
                           st, src, n, shift, hist, nb);
        hipError_t e = launch_scan_u32(hist, h, offs, sscr, st);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_rs_scatter<K>, dim3((unsigned)nb), dim3(kTPB), 0,
                           st, src, dst, n, shift, offs, nb);
        K *t = src;
        src = dst;
        dst = t;
    }
    if (src != keys)
        return hipMemcpyAsync(keys, src, sizeof(K) * n,
                              hipMemcpyDeviceToDevice, st);
    return hipGetLastError();
}

size_t sort_scratch_bytes(uint64_t n) { return sort_scratch<uint64_t>(n); }

hipError_t launch_sort_u64(uint64_t *keys, uint64_t n, int key_bits,
                           void *scratch, hipStream_t st)
{
    return sort_keys<uint64_t>(keys, n, key_bits, scratch, st);
}

size_t sort_scratch_bytes_w128(uint64_t n) { return sort_scratch<W128>(n); }

hipError_t launch_sort_w128(W128 *keys, uint64_t n, int key_bits,
                            void *scratch, hipStream_t st)
{
    return sort_keys<W128>(keys, n, key_bits, scratch, st);
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n,
                           unsigned long long v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned fill_blocks(uint64_t n)
{
    uint64_t b = (n + 255) / 256;
    if (b > 8192)
        b = 8192;
    return (unsigned)(b ? b : 1);
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, st, p,
                       n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, uint64_t n,
                           unsigned long long v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_blocks(n)), dim3(256), 0, st, p,
                       n, v);
    return hipGetLastError();
}

}  // namespace pms
