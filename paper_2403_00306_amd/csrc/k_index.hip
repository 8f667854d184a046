// k_index.hip -- 2-bit packing with validation, and the l-mer index.
//
// Packing follows the string compression of Sec. 3.3.1: each base becomes
// its 2-bit code (A=0, C=1, G=2, T=3) and the two code bits go to two bit
// planes ("groups"), so that the Hamming distance of two l-mers is the
// number of set bits of (hi_a ^ hi_b) | (lo_a ^ lo_b). The l-mer table of
// every string (the O(n(m-l+1)) compressed l-mers of PMS8, Sec. 3.2.4) holds
// both planes and the 2-bit code with the first base in the top digit.
#include "pms_internal.h"

namespace pms {

__device__ __forceinline__ int base_code(uint8_t ch)
{
    // A=65 C=67 G=71 T=84 -> 0,1,2,3; anything else -> -1
    switch (ch) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
    }
}

// One thread per (string, 32-base word). grid.y = instance.
__global__ __launch_bounds__(kTPB) void k_pack(const InstDev *insts)
{
    const InstDev I = insts[blockIdx.y];
    const int idx = blockIdx.x * kTPB + threadIdx.x;
    if (idx >= I.n * I.wpr)
        return;
    const int row = idx / I.wpr;
    const int w = idx - row * I.wpr;
    const int c0 = w * 32;
    const int c1 = min(c0 + 32, I.m);
    const uint8_t *src = I.seqs + (size_t)row * I.m;
    uint64_t packed = 0;
    uint32_t hi = 0, lo = 0;
    int bad = -1;
    for (int c = c0; c < c1; c++) {
        int b = base_code(src[c]);
        if (b < 0) {
            if (bad < 0)
                bad = c;
            b = 0;
        }
        const int k = c - c0;
        packed |= (uint64_t)b << (2 * k);
        hi |= (uint32_t)(b >> 1) << k;
        lo |= (uint32_t)(b & 1) << k;
    }
    I.packed[idx] = packed;
    I.phi[idx] = hi;
    I.plo[idx] = lo;
    if (bad >= 0)
        atomicMin(I.bad, (unsigned long long)row * I.m + bad);
}

// Spread the 32 bits of x to the even bit positions of a 64-bit word.
__device__ __forceinline__ uint64_t spread_even(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

__device__ __forceinline__ uint32_t window(const uint32_t *row, int wpr,
                                          int j, int l)
{
    const int w = j >> 5, o = j & 31;
    uint32_t v = row[w] >> o;
    if (o != 0 && o + l > 32 && w + 1 < wpr)
        v |= row[w + 1] << (32 - o);
    return l == 32 ? v : (v & ((1u << l) - 1u));
}

// One thread per (string, offset). grid.y = instance.
__global__ __launch_bounds__(kTPB) void k_lmers(const InstDev *insts)
{
    const InstDev I = insts[blockIdx.y];
    const int idx = blockIdx.x * kTPB + threadIdx.x;
    if (idx >= I.n * I.L)
        return;
    const int row = idx / I.L;
    const int j = idx - row * I.L;
    const uint32_t hi = window(I.phi + (size_t)row * I.wpr, I.wpr, j, I.l);
    const uint32_t lo = window(I.plo + (size_t)row * I.wpr, I.wpr, j, I.l);
    I.planes[idx] = make_uint2(hi, lo);
    // bit p of a plane is base p; the code wants base p in digit l-1-p
    const uint32_t rhi = __brev(hi) >> (32 - I.l);
    const uint32_t rlo = __brev(lo) >> (32 - I.l);
    I.codes[idx] = (spread_even(rhi) << 1) | spread_even(rlo);
}

hipError_t launch_index(const InstDev *d_insts, int ninst, int max_rows_words,
                        int max_lmers, hipStream_t st)
{
    if (ninst <= 0)
        return hipSuccess;
    dim3 g1((max_rows_words + kTPB - 1) / kTPB, ninst);
    hipLaunchKernelGGL(k_pack, g1, dim3(kTPB), 0, st, d_insts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    dim3 g2((max_lmers + kTPB - 1) / kTPB, ninst);
    hipLaunchKernelGGL(k_lmers, g2, dim3(kTPB), 0, st, d_insts);
    return hipGetLastError();
}

}  // namespace pms
