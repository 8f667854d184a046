// pms_internal.h -- structures shared by the host planner and the gfx950
// kernels of libpms. Not part of the public ABI (include/pms.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pms {

constexpr int kTPB = 256;          // threads per workgroup (4 wave64s)
constexpr int kWaves = kTPB / 64;
constexpr int kMaxL = 32;          // one uint32 per bit plane, one uint64 code
constexpr int kMinSuffix = 3;      // a tile word covers the last 3 bases
constexpr int kMaxSuffix = 9;      // 4^9 codes per tile = 4096 64-bit words
constexpr int kMaxWords = 1 << (2 * (kMaxSuffix - 3));
constexpr int kWordsPerThread = kMaxWords / kTPB;   // 16
constexpr int kYChunk = 640;       // l-mers staged per marking round
constexpr int kSurvMax = 256;      // survivor list of the filter stage
constexpr int kDefaultSurv = 64;   // default threshold to enter it
constexpr int kOrderMax = 64;      // per-tile string order for n up to this
#ifndef PMS_ORDER_REUSE
#define PMS_ORDER_REUSE 4
#endif
constexpr int kOrderReuse = PMS_ORDER_REUSE;   // tiles sharing one order
constexpr int kOrderReuseLog4 = kOrderReuse >= 16 ? 2 : kOrderReuse >= 4 ? 1 : 0;
constexpr int kQuorumMaxSuffix = 8;   // quorum tiles: 4^8 codes, so that
constexpr int kQuorumMaxMiss = 30;    //   5-bit miss counters of every code
                                      //   stay in registers (4 words/thread)
constexpr int kBallDigits = kMaxSuffix - 3;         // 6 word-index digits

// Read-only views of device arrays held in descriptors. The l-mer tables
// are written by the index kernels and only read afterwards, so kernels
// may read them through the constant address space: wave-uniform loads
// then become scalar loads and the rest global (not flat) loads. Bit-plane
// pairs are read as one 64-bit word (.x in the low half).
typedef __attribute__((address_space(4))) const unsigned long long g_u64;
struct PlaneRow {
    const g_u64 *p;
    __device__ __forceinline__ uint2 operator[](size_t i) const
    {
        const unsigned long long v = p[i];
        return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
    }
};
__device__ __forceinline__ PlaneRow planes_row(const uint2 *base, size_t off)
{
    return PlaneRow{(const g_u64 *)(const void *)(base + off)};
}
__device__ __forceinline__ const g_u64 *gptr(const uint64_t *p)
{
    return (const g_u64 *)(const void *)p;
}

// Values that are the same in every lane by construction (block-reduction
// results, counts read back from LDS after a barrier): tell the compiler,
// so that loops over them stay scalar.
__device__ __forceinline__ uint32_t uni(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ int uni(int v)
{
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ unsigned long long uni(unsigned long long v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// One instance as the kernels see it. All pointers are device memory.
struct InstDev {
    const uint8_t *seqs;     // n*m ASCII bytes, row-major
    uint64_t *packed;        // n*wpr words: base j of a row at bits 2(j%32)
    uint32_t *phi;           // n*wpr: bit j%32 = high code bit of base j
    uint32_t *plo;           // n*wpr: bit j%32 = low code bit of base j
    uint2 *planes;           // n*L l-mers: .x high plane, .y low plane,
                             //   bit p = base p of the l-mer
    uint64_t *codes;         // n*L l-mers, first base in the top digit
    const int *order;        // n: string order of the tile passes
    unsigned long long *bad; // first bad byte (row*m+col); ~0 if none
    // tile outputs (tiled path); tile indices are local to the instance
    uint32_t *tile_cnt;      // ntiles: motifs found in each tile
    uint64_t *tile_heap_off; // ntiles: where the tile's motifs sit in heap
    uint64_t *heap;          // unordered blocks of ascending codes
    unsigned long long *heap_top;
    unsigned long long heap_cap;
    uint64_t tile_base;      // first tile of this instance in a batch's
                             //   concatenated tile space
    uint64_t ntiles;         // 4^(l-s)
    int n, m, l, d, L, s, surv_t, wpr;
    int q;                   // quorum: a motif needs d-neighbours in at
                             //   least q strings (q = n: every string)
    int tile_order;          // tiled path: order the strings per tile
};

// The descriptor read by every thread of a workgroup is the same: make each
// of its words wave-uniform so that its fields live in scalar registers
// (loaded through a vector register they would hold a VGPR pair per
// pointer, which the 512-thread tile kernel spilled).
__device__ __forceinline__ InstDev uni_desc(const InstDev &x)
{
    static_assert(sizeof(InstDev) % 4 == 0, "descriptor words");
    constexpr int kW = (int)(sizeof(InstDev) / 4);
    uint32_t wd[kW];
    __builtin_memcpy(wd, &x, sizeof(InstDev));
#pragma unroll
    for (int i = 0; i < kW; i++)
        wd[i] = __builtin_amdgcn_readfirstlane(wd[i]);
    InstDev y;
    __builtin_memcpy(&y, wd, sizeof(InstDev));
    return y;
}

// A contiguous range of one instance's tiles.
struct WorkItem {
    int inst;
    int pad;
    uint64_t t0, t1;
};

// Device counters of the tiled and bitset kernels.
struct TileStats {
    unsigned long long passes;      // (tile, string) passes
    unsigned long long marks;       // 64-bit word ORs
    unsigned long long ftests;      // Hamming tests of the filter stage
    unsigned long long tiles;       // tiles finished
};

// LDS position of tile word w: the bank bits (low 5 bits of the word
// position) take the XOR of the word index's low 5 bits with its higher
// bit groups, so words that differ only in high digits still fall in
// different banks. A bijection on [0, 4^q) that keeps bits 5 and up. It is
// linear over GF(2) (shifts, masks and XORs of bits), so
// wpos(y ^ m) = wpos(y) ^ wpos(m).
__host__ __device__ __forceinline__ uint32_t wpos(uint32_t w)
{
    return w ^ ((w >> 5) & 31u) ^ ((w >> 10) & 31u);
}

// Group constants of the small-sphere marking: for a workgroup of TPB
// threads (256: set 0, 512: set 1) and a word-level sphere of bs entries,
// G = TPB / bs groups of bs lanes, and a multiplier mg with
// floor(v / bs) = (v * mg) >> 22 for every v < 1024.
constexpr int kGrpStride = 7 * 8 * 2;   // per set: (q*8 + rw) * 2 + {G, mg}
constexpr int kGrpShift = 22;

// Tables built once per context (device memory).
struct Tables {
    // Word-index ball table for q = s-3 digits: all 4^q XOR masks over q
    // 2-bit digits ordered by weight (number of nonzero digits); entry =
    // mask | weight << 12. ball_off[q*8 + w] = first entry of weight w
    // (ball_off[q*8 + q + 1] = 4^q).
    const uint16_t *ball;        // concatenated for q = 0..6
    const int *ball_base;        // start of table q in ball[]
    const int *ball_off;         // 7 x 8 offsets
    // The same entries in the form the marking loops use:
    // 8 * wpos(mask) | weight << 16 (the byte offset of the masked word's
    // part of an LDS address, and the weight).
    const uint32_t *ball32;
    const uint32_t *grp;         // 2 sets x kGrpStride group constants
    // Word masks: m3[b*4 + t] = bit z set iff the 3-base codes z and b
    // differ in at most t bases (t = 3: every z).
    const unsigned long long *m3;
};

// ---- kernel launchers (defined in the .hip files) -----------------------

// Pack + validate (a1) and l-mer index (a2) for ninst instances.
hipError_t launch_index(const InstDev *d_insts, int ninst, int max_rows_words,
                        int max_lmers, hipStream_t st);

// Tiled pattern-driven kernel over a work list (persistent workgroups).
// d_items == nullptr: instance 0's tiles in nitems chunks of `chunk`.
// wide: the 512-thread kernel (for tiles of 4^9 codes on the plain path)
hipError_t launch_tiled(const InstDev *d_insts, const WorkItem *d_items,
                        int nitems, uint64_t chunk, unsigned int *d_next,
                        Tables tb, TileStats *stats, int grid, hipStream_t st,
                        bool wide = false);
int tiled_blocks_per_cu(bool wide = false);
// Any-alphabet sample-driven filter (k_alpha.hip).
struct AlphaJob {
    const uint8_t *letters;      // n*m letter codes (index in the alphabet)
    const uint32_t *planes;      // n*L l-mers, 8 words each: bit planes 0..4
    const uint32_t *posset;      // position sets (bitmasks) by weight k,
    const uint64_t *posoff;      //   weight k starting at posoff[k]
    const uint64_t *cum;         // first flat sphere index of weight k
    const uint64_t *powr;        // (sigma-1)^k
    uint64_t nb;                 // sphere size n_B(l, d) over sigma letters
    uint64_t *heap;              // survivors (unordered, repeats possible)
    unsigned long long *heap_top;
    unsigned long long heap_cap;
    unsigned long long *hcanon;  // canonical Hamming tests (L per string
                                 //   examined, first failing one included)
    int n, m, l, d, L, sigma;
};
hipError_t launch_alpha_index(const uint8_t *seqs, const uint8_t *map, int n,
                              int m, int l, int P, uint8_t *letters,
                              uint32_t *planes, unsigned long long *bad,
                              hipStream_t st);
hipError_t launch_alpha_filter(const AlphaJob &J, unsigned int *next,
                               int grid, hipStream_t st);
// Sorted a[0..n): flag[i] = 1 where a value starts, pos = exclusive scan
// of flag (n+1 entries, pos[n] = number of distinct values); then the
// distinct values to out[0..pos[n]) (out must not overlap a).
hipError_t launch_unique_count(const uint64_t *a, uint64_t n, uint32_t *flag,
                               uint64_t *pos, void *scan_scratch,
                               hipStream_t st);
hipError_t launch_unique_scatter(const uint64_t *a, uint64_t n,
                                 const uint32_t *flag, const uint64_t *pos,
                                 uint64_t *out, hipStream_t st);
int alpha_blocks_per_cu();

// Pair-based candidates (k_pair.hip).
struct PairTuple {
    uint64_t first;              // first flat index of this tuple for its D
    uint8_t a, b, c, e;          // letters from x / from y / other on the
                                 //   differing positions; changed agreeing
    uint32_t n3;                 // 3^e
    uint32_t ns;                 // C(l-D, e)
    uint32_t pad;
};
constexpr int kPairMaxTuples = 1024;   // held in LDS by the filter
constexpr int kPairMaxD = 20;          // 2d <= 20: multinomials < 2^32
struct PairJob {
    const uint2 *planes;         // the instance's l-mer planes (row 0 = s_1)
    const uint64_t *nD;          // |B(x,d) ∩ B(y,d)| by D = d_H(x,y)
    const PairTuple *tup;        // tuples of every D, D's at tup_off[D]
    const int *tup_off;
    const uint64_t *binom;       // binom[n*(kMaxL+1)+k]
    const uint32_t *multi;       // multinomial (r; a, b, r-a-b) at
                                 //   [(r*(kPairMaxD+1)+a)*(kPairMaxD+1)+b]
    int ntup;
    uint2 *pairs;                // compatible pairs (index in s_1, in s_2)
    uint32_t *chunks;            // work items per pair
    unsigned long long *npairs, *ncand, *next, *tests;
    unsigned long long pairs_cap;
    const uint64_t *item_pos;    // exclusive scan of chunks (npairs+1)
    const uint32_t *item_pair;   // the pair of each work item
    uint64_t *heap;              // survivors (unordered, repeats possible)
    unsigned long long *heap_top;
    unsigned long long heap_cap;
    const uint32_t *partner;     // per l-mer x of s_1: the string its pairs
                                 //   take y from (1 = s_2 for every x)
    uint2 *q[2];                 // candidate queues between strings
    uint16_t *qp[2];             // partner string of each queued candidate
    unsigned long long *qcount;  // entries appended to q[0] by the filter
    unsigned long long qcap;
    unsigned int *overflow;      // set if a queue overflowed
    int n, L, l, d;
};
// partner[x] for every l-mer x of s_1: the string j >= 1 whose nearest
// l-mer is farthest from x (lowest j on ties).
hipError_t launch_pair_partner(const uint2 *planes, int n, int L,
                               uint32_t *partner, hipStream_t st);
hipError_t launch_pair_list(const PairJob &J, hipStream_t st);
// item_pair[it] = the pair whose work items hold it, for every item
hipError_t launch_pair_items(const PairJob &J, unsigned long long npairs,
                             uint32_t *item_pair, hipStream_t st);
// Candidates of the work items [*J.next, it1) against s_3, survivors to
// q[0] (count in *J.qcount); then each later string with launch_pair_queue.
hipError_t launch_pair_filter(const PairJob &J, unsigned long long it1,
                              unsigned long long npairs, int grid,
                              hipStream_t st);
hipError_t launch_pair_queue(const PairJob &J, int i, const uint2 *qin,
                             const uint16_t *qpin,
                             const unsigned long long *qin_count, uint2 *qout,
                             uint16_t *qpout, unsigned long long *qout_count,
                             int grid, hipStream_t st);
int pair_chunk();
int pair_blocks_per_cu();

// Quorum variant of launch_tiled (instances with q < n, tile suffix at
// most kQuorumMaxSuffix, n - q at most kQuorumMaxMiss).
hipError_t launch_tiled_quorum(const InstDev *d_insts, const WorkItem *d_items,
                               int nitems, uint64_t chunk,
                               unsigned int *d_next, Tables tb,
                               TileStats *stats, int grid, hipStream_t st);
int tiled_quorum_blocks_per_cu();

// Memory-heavy bitset path: one pass per string over the whole 4^l space.
// One string pass of the memory-heavy path; tiles are taken `chunk` at a
// time from *next (cleared by the caller before the launch).
// pass p of the bitset path: cnt holds 2n zeroed counters (chunk counter
// and output list length per pass); list0/list1 hold ntiles tile indices
// each (the live tiles, ping-pong); chunk0 = tiles per chunk in pass 0
hipError_t launch_bitset_pass(const InstDev *d_inst, int pass, Tables tb,
                              unsigned long long *A, uint8_t *alive,
                              const uint8_t *ord, unsigned int *cnt,
                              uint32_t *list0, uint32_t *list1, int chunk0,
                              TileStats *stats, int grid, hipStream_t st);
// per-tile string order of the bitset path: n bytes per tile in ord
// (n <= kOrderMax), through n 32-bit masses per tile in mass
hipError_t launch_bitset_order(const InstDev *d_inst, Tables tb,
                               uint32_t *mass, uint8_t *ord, uint64_t ntiles,
                               int n, hipStream_t st);
int bitset_blocks_per_cu();
hipError_t launch_bitset_count(const InstDev *d_inst,
                               const unsigned long long *A,
                               const uint8_t *alive, uint32_t *tile_cnt,
                               int grid, hipStream_t st);
hipError_t launch_bitset_emit(const InstDev *d_inst,
                              const unsigned long long *A,
                              const uint32_t *tile_cnt,
                              const uint64_t *tile_pos, uint64_t *out,
                              unsigned long long cap, int grid,
                              hipStream_t st);

// Sample-driven filter path.
hipError_t launch_masks(int l, int d, uint2 *masks, uint64_t nb,
                        hipStream_t st);
hipError_t launch_filter(const InstDev *d_inst, const uint2 *masks,
                         uint64_t nb, unsigned long long *next_block,
                         uint64_t *heap, unsigned long long *heap_top,
                         unsigned long long heap_cap,
                         unsigned long long *hc_per_ref,
                         unsigned long long *hexec, int grid, hipStream_t st);
int filter_blocks_per_cu();
// Quorum motifs (q = I.q < n) on the sample-driven path: candidates from the
// l-mers of the first R = n-q+1 strings, kept with at most n-q misses,
// free of repeats (each from its first reference); unsorted in heap.
hipError_t launch_filter_quorum(const InstDev *d_inst, const uint2 *masks,
                                uint64_t nb, int R,
                                unsigned long long *next_block, uint64_t *heap,
                                unsigned long long *heap_top,
                                unsigned long long heap_cap, int grid,
                                hipStream_t st);
uint32_t filter_quorum_max_refs();   // R*L must stay below this
// calibration kernel: the filter's Hamming-test mix from registers only
hipError_t launch_test_rate(int grid, int iters, uint32_t seed,
                            unsigned int *sink, hipStream_t st);
hipError_t launch_lds_rate(int grid, int iters, unsigned int *sink,
                           hipStream_t st);
int lds_rate_blocks_per_cu();
uint64_t lds_rate_ors_per_block(int iters);
int test_rate_blocks_per_cu();
uint64_t test_rate_tests_per_thread(int iters);

// Scans, ordered gathers and sorting (a6).
size_t scan_scratch_bytes(uint64_t n);
hipError_t launch_scan_u32(const uint32_t *in, uint64_t n, uint64_t *out,
                           void *scratch, hipStream_t st);
// Tiles whose block lies beyond heap_cap (heap overflow) are skipped.
hipError_t launch_gather(const uint32_t *tile_cnt, const uint64_t *heap_off,
                         const uint64_t *tile_pos, const uint64_t *heap,
                         uint64_t ntiles, uint64_t *out,
                         unsigned long long out_cap,
                         unsigned long long heap_cap, hipStream_t st);
hipError_t launch_ranges(const InstDev *d_insts, int ninst,
                         const uint64_t *tile_pos, uint64_t *ranges,
                         hipStream_t st);
size_t sort_scratch_bytes(uint64_t n);
hipError_t launch_sort_u64(uint64_t *keys, uint64_t n, int key_bits,
                           void *scratch, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v,
                           hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, uint64_t n,
                           unsigned long long v, hipStream_t st);

}  // namespace pms
