// k_tiles.hip -- pattern-driven kernels over the 4^l code space.
//
// The pattern-driven view (Sec. 1.3.1) asks, for every l-mer M, whether each
// string s_i has an l-mer y with d_H(M, y) <= d, i.e. whether M lies in
// U_i = union over y in s_i of the sphere B(y, d) (Table 3.1). The motif set
// is the intersection of U_1..U_n. These kernels hold U_i and the running
// intersection as bitsets over the code space, one bit per l-mer code
// (first base in the top digit, so bit order is code order).
//
// Tiling. A tile fixes the first l-s bases (the prefix P) and covers all
// 4^s suffixes: 4^(s-3) 64-bit words in LDS, word index = suffix bases
// 0..s-4, bit index = the last 3 bases. An l-mer y reaches the tile iff
// k = d_H(prefix(y), P) <= d, and then marks exactly the suffixes within
// distance r = d - k of suffix(y). Marking goes by words: for every XOR
// mask over the word-index digits with weight w <= r, the word
// (index(y) ^ mask) receives the precomputed mask of 3-base codes within
// distance min(r - w, 3) of y's last 3 bases.
//
// Tiled path (PMS_PATH_TILED): a workgroup keeps one tile's intersection in
// registers and ANDs the strings in one by one; the tile stops when it is
// empty, and when at most surv_t codes are left it tests those codes
// directly against the remaining strings (the XOR/popcount Hamming filter
// of Sec. 3.3.1 with early exit at the first string without a hit).
//
// Bitset path (PMS_PATH_BITSET, memory heavy): the whole 4^l-bit
// intersection lives in device memory and each string is one pass over
// every live tile: read 4^s bits, AND the string's union, write back.
#include "pms_internal.h"

#include <type_traits>

namespace pms {

// The tile code is written for a workgroup of TPB threads: kTPB (256, four
// waves) for every tiled kernel, and kTPBWide (512, eight waves at up to 64
// VGPRs) for a second plain-path kernel that keeps twice the waves per CU
// in flight; the planner takes it for tiles of 4^8 and 4^9 codes. Inside the
// templates kTPB, kWaves and kWordsPerThread are redeclared for TPB.
constexpr int kTPBWide = 512;
constexpr int kMaxTileWaves = kTPBWide / 64;
constexpr int kYPer = (kYChunk + kTPB - 1) / kTPB;    // l-mers per thread
constexpr int kYList = kYChunk + 4 * (kMaxL + 1);      // radius classes
                                                       // start 4-aligned
struct __align__(16) TileShared {
    unsigned long long U[kMaxWords];   // the string's union on this tile
    unsigned long long m3[256];        // word masks, copy of Tables::m3
    union {
        uint32_t ylist[kYList];        // suffix codes of reaching l-mers
        uint64_t surv[kSurvMax];       // filter stage: codes left
    };
    int rcnt[kMaxL + 1];               // reaching l-mers per radius r
    int roff[kMaxL + 2];
    int rpos[kMaxL + 1];
    unsigned long long red64[kMaxTileWaves];
    unsigned int red32[kMaxTileWaves];
    unsigned int redc[2][kMaxTileWaves];   // pass counts, by pass parity
    unsigned long long hitm[2][kSurvMax / 64];   // filter stage hits
    unsigned long long bcast;
    uint32_t mass[kOrderMax];          // per-tile string order: sphere mass
    int torder[kOrderMax];             //   of each string, strings by mass
    uint32_t cw[kMaxL + 1];            //   word entries of B at radius r
};

// the filter stage keeps two plane buffers, a code buffer and the hit
// flags in sh.U; each lane holds kFiltPer l-mers of a string at a time
constexpr int kFiltPer = 3;
constexpr int kFiltWords = 3 * kSurvMax + kSurvMax / 2;
static_assert(kFiltWords <= kMaxWords && kSurvMax <= kTPB,
              "filter scratch exceeds the tile");

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup; every thread gets the total.
template <int TPB>
__device__ __forceinline__ unsigned long long
block_sum64(unsigned long long v, unsigned long long *red)
{
    constexpr int kWaves = TPB / 64;
    v = wave_sum64(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++)
        t += red[w];
    return uni(t);
}

// Sum over the wave by DPP (no LDS): inclusive scans of the four rows of
// 16 lanes (row_shr 1, 2, 4, 8), then row 0's total into row 1 and row 2's
// into row 3 (row_bcast:15), then lane 31's into rows 2 and 3
// (row_bcast:31); lane 63 holds the sum. Lanes whose source is outside
// the row, or rows the mask leaves out, add the 0 passed as `old`.
__device__ __forceinline__ uint32_t wave_sum32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Sum over the workgroup with one barrier: the caller alternates between
// two `red` buffers on successive calls, and at least one other barrier
// separates a call from the next use of the same buffer, so no thread can
// overwrite a value another thread has yet to read.
template <int TPB>
__device__ __forceinline__ uint32_t block_sum32(uint32_t v, unsigned int *red)
{
    constexpr int kWaves = TPB / 64;
    v = wave_sum32(v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++)
        t += red[w];
    return uni(t);
}

// Exclusive prefix sum over the workgroup in thread order.
template <int TPB>
__device__ __forceinline__ unsigned int
block_exscan(unsigned int v, unsigned int *red, unsigned int *total)
{
    constexpr int kWaves = TPB / 64;
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

// Bit planes of a tile prefix (pl bases, first base in the top digit).
__device__ __forceinline__ void prefix_planes(uint64_t P, int pl,
                                              uint32_t &hi, uint32_t &lo)
{
    hi = 0;
    lo = 0;
    for (int p = 0; p < pl; p++) {
        const uint32_t dig = (uint32_t)(P >> (2 * (pl - 1 - p))) & 3u;
        hi |= (dig >> 1) << p;
        lo |= (dig & 1u) << p;
    }
}

// Tile words sit at LDS position wpos(w) (pms_internal.h). wpos is linear,
// so wpos(y ^ m) = wpos(y) ^ wpos(m): a lane keeps its XOR mask's part of
// the LDS address, and an l-mer's part is computed once when it is listed.
// A listed l-mer is a = (wpos(word index) << 6) | (last 3 bases); the byte
// offset of its word is ((a >> 3) & ~7), of the 32-bit half that holds its
// bit ((a >> 3) & ~3).
__device__ __forceinline__ uint32_t list_entry(uint32_t ysuf)
{
    return (wpos(ysuf >> 6) << 6) | (ysuf & 63u);
}

// OR a single bit with a 32-bit atomic on the half-word that holds it (one
// LDS bank per lane instead of two). off = byte offset in sh.U.
__device__ __forceinline__ void or32_at(TileShared &sh, uint32_t off,
                                        uint32_t v)
{
    atomicOr(reinterpret_cast<unsigned int *>(
                 reinterpret_cast<char *>(sh.U) + off), v);
}

__device__ __forceinline__ void or64_at(TileShared &sh, uint32_t off,
                                        unsigned long long v)
{
    atomicOr(reinterpret_cast<unsigned long long *>(
                 reinterpret_cast<char *>(sh.U) + off), v);
}

// OR into sh.U the union of the d-spheres of string `seq`'s l-mers,
// restricted to the tile with prefix planes (Phi, Plo). The ball table of
// q = s-3 must be in sh.ball. Ends with a barrier. Returns the number of
// word ORs done (same value in every thread).
//
// The reaching l-mers are grouped by radius r and every class is marked
// entry-parallel: each lane keeps one XOR mask of the class's word-level
// sphere in registers and walks the class's l-mers. When the sphere has
// more than kTPB/2 entries every wave walks the same l-mers (64 read at
// once, then broadcast into scalar registers by readlane); a smaller
// sphere is repeated in kTPB/bs lane groups that walk different l-mers.
// A caller-supplied hook(y0) runs in every listing round (y0 = the round's
// first l-mer), unconditionally, after the round's l-mer loads are issued
// and before their values are used: memory loads the hook issues then queue
// behind them, so the listing does not wait for the hook's loads (the memory
// counter is waited on in issue order; a branch around the hook would make
// the compiler wait for everything at the join).
struct NoHook {
    __device__ void operator()(int) const {}
};

template <int TPB, class Hook = NoHook>
__device__ __forceinline__ unsigned long long
mark_string(const InstDev &I, int seq, uint32_t Phi, uint32_t Plo,
            uint32_t premask, TileShared &sh, const Tables &tb,
            Hook &&hook = Hook())
{
    constexpr bool kHook = !std::is_same<typename std::decay<Hook>::type,
                                         NoHook>::value;
    constexpr int kTPB = TPB;
    constexpr int kYPer = (kYChunk + TPB - 1) / TPB;
    const int tid = threadIdx.x;
    const int d = I.d, s = I.s, q = s - 3;
    const PlaneRow yp = planes_row(I.planes, (size_t)seq * I.L);
    const uint32_t sufmask = (1u << (2 * s)) - 1u;
    // read-only tables through the constant address space: the uniform
    // reads (sphere sizes, group constants) become scalar loads
    typedef const __attribute__((address_space(4))) uint32_t c_u32;
    typedef const __attribute__((address_space(4))) int c_i32;
    // low words of the string's l-mer codes (the suffix fits in 18 bits)
    c_u32 *ycl = (c_u32 *)(const void *)(I.codes + (size_t)seq * I.L);
    c_i32 *boff = (c_i32 *)(const void *)(tb.ball_off + q * 8);
    c_u32 *grp = (c_u32 *)(const void *)(tb.grp + (TPB >= kTPBWide ? 1 : 0) *
                                                        kGrpStride +
                                         q * 16);
    // ball table q: each lane reads its entry once per class
    c_u32 *ball = (c_u32 *)(const void *)(
        tb.ball32 + ((c_i32 *)(const void *)tb.ball_base)[q]);
    unsigned long long marks = 0;
    for (int y0 = 0; y0 < I.L; y0 += kYChunk) {
        const int ny = min(kYChunk, I.L - y0);
        if (tid <= d)
            sh.rcnt[tid] = 0;
        __syncthreads();
        uint32_t ys[kYPer];
        int rr[kYPer];
        if constexpr (kHook) {
            // every load of the round first, then the hook, then the tests;
            // the code words through a plain global pointer, which the
            // compiler may not move past the hook (it would sink a
            // constant-space load into the branch that uses it)
            typedef const __attribute__((address_space(1))) uint32_t g_u32;
            g_u32 *ycg = (g_u32 *)(const void *)(I.codes + (size_t)seq * I.L);
            uint2 yv[kYPer];
            uint32_t ylv[kYPer];
#pragma unroll
            for (int u = 0; u < kYPer; u++) {
                const int j = min(tid + u * kTPB, ny - 1);
                yv[u] = yp[y0 + j];
                ylv[u] = ycg[2 * (y0 + j)];
            }
            // keep the scheduler from moving any of those loads past the
            // hook's
            asm volatile("" : : : "memory");
            hook(y0);
#pragma unroll
            for (int u = 0; u < kYPer; u++) {
                const int j = tid + u * kTPB;
                rr[u] = -1;
                const int k = __popc(((yv[u].x ^ Phi) | (yv[u].y ^ Plo)) &
                                     premask);
                if (j < ny && k <= d) {
                    rr[u] = d - k;
                    ys[u] = list_entry(ylv[u] & sufmask);
                    atomicAdd(&sh.rcnt[d - k], 1);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < kYPer; u++) {
                const int j = tid + u * kTPB;
                rr[u] = -1;
                if (j < ny) {
                    // both loads in flight together: one memory round trip
                    const uint2 y = yp[y0 + j];
                    const uint32_t yl = ycl[2 * (y0 + j)];
                    asm volatile("" : : "v"(yl));
                    const int k = __popc(((y.x ^ Phi) | (y.y ^ Plo)) &
                                         premask);
                    if (k <= d) {
                        rr[u] = d - k;
                        ys[u] = list_entry(yl & sufmask);
                        atomicAdd(&sh.rcnt[d - k], 1);
                    }
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int r = 0; r <= d; r++) {
                sh.roff[r] = acc;
                sh.rpos[r] = acc;
                acc += (sh.rcnt[r] + 3) & ~3;
            }
            sh.roff[d + 1] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kYPer; u++)
            if (rr[u] >= 0)
                sh.ylist[atomicAdd(&sh.rpos[rr[u]], 1)] = ys[u];
        __syncthreads();
        const uint32_t lane = (uint32_t)tid & 63u;
        // every class's count and list offset in one read per lane (d < 32),
        // then taken per class by readlane
        const int vcnt = (int)lane <= d ? sh.rcnt[lane] : 0;
        const int voff = (int)lane <= d ? sh.roff[lane] : 0;
        for (int r = 0; r <= d; r++) {
            const int c = __builtin_amdgcn_readlane(vcnt, r);
            if (c == 0)
                continue;
            const int rw = min(r, q);
            const uint32_t bs = (uint32_t)boff[rw + 1];
            const uint32_t *yl = sh.ylist + __builtin_amdgcn_readlane(voff, r);
            marks += (unsigned long long)c * bs;
            // rotate the lane assignment per class so that the lanes a
            // class leaves idle fall in a different wave each time
            const uint32_t rot = 64u * (uint32_t)r;
            if (bs > (uint32_t)kTPB / 2) {
                // These waves issue their ORs back to back, with no wait;
                // a raised issue priority keeps the LDS fed from them while
                // the CU's other waves sit in latency-bound phases (listing,
                // AND and count, survivor tests). Raised for the lane-group
                // classes too, it slowed the small tiles of (13,4).
                __builtin_amdgcn_s_setprio(1);
                // Entry-parallel: lane owns entries e, e+kTPB, ... of the
                // sphere and the wave walks the class's l-mers, 64 at a
                // time: one LDS read per lane, then broadcast by readlane.
                // Every lane of a working wave stays active (readlane needs
                // the source lane's value): a lane past the end of the
                // sphere repeats an entry that another wave, or itself in
                // the previous round, already ORs; ORs are idempotent.
                const uint32_t wfirst =
                    uni(((uint32_t)tid - lane + rot) & (uint32_t)(kTPB - 1));
                // a class of at most 64 l-mers (nearly all) is read once for
                // all its rounds: every LDS read waits for the wave's
                // earlier ORs to complete
                int v1 = 0;
                if (c <= 64 && wfirst < bs) {
                    const int vl = (int)yl[min((int)lane, c - 1)];
                    asm volatile("v_mov_b32 %0, %1" : "=v"(v1) : "v"(vl));
                }
                for (uint32_t eb = 0; eb < bs; eb += kTPB) {
                    const uint32_t e0 = wfirst + eb;
                    if (e0 >= bs)
                        continue;
                    uint32_t e = e0 + lane;
                    e = e < bs ? e : e - (eb ? (uint32_t)kTPB : bs);
                    const uint32_t ent = ball[e];
                    const uint32_t lc = ent & 0xffffu;
                    const int tt = min(r - (int)(ent >> 16), 3);
                    const unsigned long long *mt = sh.m3 + tt;
                    const bool single = __ballot(tt != 0) == 0;
                    for (int y0c = 0; y0c < c; y0c += 64) {
                        const int nc = min(64, c - y0c);
                        int v = v1;
                        if (c > 64) {
                            const int vl =
                                (int)yl[y0c + min((int)lane, nc - 1)];
                            // a VALU copy: the LDS read is waited for here,
                            // once, and not at every readlane below (where
                            // a wait would also drain this wave's pending
                            // ORs)
                            asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "v"(vl));
                        }
                        int j = 0;
                        if (single) {
                            // in-word radius 0 in the whole wave: the word
                            // mask is the single bit of the last 3 bases
                            for (; j + 4 <= nc; j += 4) {
                                const uint32_t a0 = __builtin_amdgcn_readlane(v, j);
                                const uint32_t a1 = __builtin_amdgcn_readlane(v, j + 1);
                                const uint32_t a2 = __builtin_amdgcn_readlane(v, j + 2);
                                const uint32_t a3 = __builtin_amdgcn_readlane(v, j + 3);
                                or32_at(sh, ((a0 >> 3) & ~3u) ^ lc, 1u << (a0 & 31u));
                                or32_at(sh, ((a1 >> 3) & ~3u) ^ lc, 1u << (a1 & 31u));
                                or32_at(sh, ((a2 >> 3) & ~3u) ^ lc, 1u << (a2 & 31u));
                                or32_at(sh, ((a3 >> 3) & ~3u) ^ lc, 1u << (a3 & 31u));
                            }
                            for (; j < nc; j++) {
                                const uint32_t a0 = __builtin_amdgcn_readlane(v, j);
                                or32_at(sh, ((a0 >> 3) & ~3u) ^ lc, 1u << (a0 & 31u));
                            }
                        } else {
                            for (; j + 4 <= nc; j += 4) {
                                const uint32_t a0 = __builtin_amdgcn_readlane(v, j);
                                const uint32_t a1 = __builtin_amdgcn_readlane(v, j + 1);
                                const uint32_t a2 = __builtin_amdgcn_readlane(v, j + 2);
                                const uint32_t a3 = __builtin_amdgcn_readlane(v, j + 3);
                                const unsigned long long m0 = mt[(a0 & 63u) * 4u];
                                const unsigned long long m1 = mt[(a1 & 63u) * 4u];
                                const unsigned long long m2 = mt[(a2 & 63u) * 4u];
                                const unsigned long long m3v = mt[(a3 & 63u) * 4u];
                                or64_at(sh, ((a0 >> 3) & ~7u) ^ lc, m0);
                                or64_at(sh, ((a1 >> 3) & ~7u) ^ lc, m1);
                                or64_at(sh, ((a2 >> 3) & ~7u) ^ lc, m2);
                                or64_at(sh, ((a3 >> 3) & ~7u) ^ lc, m3v);
                            }
                            for (; j < nc; j++) {
                                const uint32_t a0 = __builtin_amdgcn_readlane(v, j);
                                or64_at(sh, ((a0 >> 3) & ~7u) ^ lc,
                                        mt[(a0 & 63u) * 4u]);
                            }
                        }
                    }
                }
            } else {
                __builtin_amdgcn_s_setprio(0);
                // G = kTPB/bs groups of bs lanes: each lane owns one entry
                // and its group walks every G-th l-mer of the class (the
                // division by bs is a multiply by a host-made constant)
                const uint32_t vt = ((uint32_t)tid + rot) & (uint32_t)(kTPB - 1);
                const uint32_t G = grp[rw * 2];
                const uint32_t slot = (vt * grp[rw * 2 + 1]) >> kGrpShift;
                const uint32_t e = vt - slot * bs;
                if (slot < G) {
                    const uint32_t ent = ball[e];
                    const uint32_t lc = ent & 0xffffu;
                    const uint32_t tt = (uint32_t)min(r - (int)(ent >> 16), 3);
                    const unsigned long long *mt = sh.m3 + tt;
                    // the group's l-mers are a contiguous block, read four
                    // at a time (class lists start 4-aligned and are padded
                    // to a multiple of 4; entries past the block are not
                    // marked)
                    uint32_t blk = 4;
                    while (blk * G < (uint32_t)c)
                        blk += 4;
                    const uint32_t b0 = slot * blk;
                    const uint32_t b1 = min((uint32_t)c, b0 + blk);
                    const uint4 *yl4 = reinterpret_cast<const uint4 *>(yl);
                    if (__ballot(tt != 0) == 0) {
                        // in-word radius 0 in every active lane: single bit
                        for (uint32_t b = b0; b < b1; b += 4) {
                            const uint4 v4 = yl4[b >> 2];
                            const uint32_t av[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                            for (uint32_t k = 0; k < 4; k++)
                                if (b + k < b1)
                                    or32_at(sh, ((av[k] >> 3) & ~3u) ^ lc,
                                            1u << (av[k] & 31u));
                        }
                        continue;
                    }
                    for (uint32_t b = b0; b < b1; b += 4) {
                        const uint4 v4 = yl4[b >> 2];
                        const uint32_t av[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
                        for (uint32_t k = 0; k < 4; k++)
                            if (b + k < b1)
                                or64_at(sh, ((av[k] >> 3) & ~7u) ^ lc,
                                        mt[(av[k] & 63u) * 4u]);
                    }
                }
            }
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(0);
    }
    return marks;
}

// The codes of the set bits of words w0..w1 of sh.U, ascending, written
// to dst[pos..). Codes: (tile << 2s) | (word << 6) | bit.
__device__ __forceinline__ void emit_bits(const TileShared &sh, int w0,
                                          int w1, uint64_t tile, int s,
                                          uint64_t *dst, unsigned int pos)
{
    const uint64_t base = tile << (2 * s);
    for (int w = w0; w < w1; w++) {
        unsigned long long v = sh.U[w];
        while (v) {
            const int b = __ffsll(v) - 1;
            v &= v - 1;
            dst[pos++] = base | ((uint64_t)w << 6) | (uint64_t)b;
        }
    }
}

// Write the set bits of the tile (words 0..W-1 of sh.U) as ascending codes
// to dst[0..). Thread t owns a contiguous block of words so that thread
// order is code order.
template <int TPB>
__device__ void emit_words(const TileShared &sh, int W, uint64_t tile, int s,
                           uint64_t *dst, bool write, unsigned int *red)
{
    constexpr int kTPB = TPB;
    const int tid = threadIdx.x;
    const int per = (W + kTPB - 1) / kTPB;
    const int w0 = tid * per;
    const int w1 = min(w0 + per, W);
    unsigned int cnt = 0;
    for (int w = w0; w < w1; w++)
        cnt += __popcll(sh.U[w]);
    unsigned int tot;
    unsigned int pos = block_exscan<TPB>(cnt, red, &tot);
    if (!write)
        return;
    emit_bits(sh, w0, w1, tile, s, dst, pos);
}

// Emit tile g's codes (words 0..W-1 of sh.U) into the instance's heap: the
// count comes from the same scan that places the codes, so the space taken
// from heap_top always matches what is written. Records the tile's count
// and heap offset; writes nothing once the heap is full (heap_top then
// tells the host how much it needed). Returns the count.
template <int TPB>
__device__ unsigned int emit_tile(TileShared &sh, int W, uint64_t tile,
                                  uint64_t g, int s, const InstDev &I)
{
    constexpr int kTPB = TPB;
    const int tid = threadIdx.x;
    const int per = (W + kTPB - 1) / kTPB;
    const int w0 = tid * per;
    const int w1 = min(w0 + per, W);
    unsigned int cnt = 0;
    for (int w = w0; w < w1; w++)
        cnt += __popcll(sh.U[w]);
    unsigned int tot;
    const unsigned int pos = block_exscan<TPB>(cnt, sh.red32, &tot);
    if (tid == 0) {
        const unsigned long long off =
            tot ? atomicAdd(I.heap_top, (unsigned long long)tot) : 0ull;
        sh.bcast = off;
        I.tile_cnt[g] = tot;
        I.tile_heap_off[g] = off;
    }
    __syncthreads();
    const unsigned long long off = uni(sh.bcast);
    if (off + tot <= I.heap_cap)
        emit_bits(sh, w0, w1, tile, s, I.heap + off, pos);
    return tot;
}

// Convert a code (first base in the top digit) to bit planes.
__device__ __forceinline__ uint2 code_planes(uint64_t c, int l)
{
    uint32_t hi = 0, lo = 0;
    for (int p = 0; p < l; p++) {
        const uint32_t dig = (uint32_t)(c >> (2 * (l - 1 - p))) & 3u;
        hi |= (dig >> 1) << p;
        lo |= (dig & 1u) << p;
    }
    return make_uint2(hi, lo);
}

struct StatAcc {
    unsigned long long passes, marks, ftests, tiles;
};

// One tile of the tiled path.
// Strings in ascending order of the word marks their reaching l-mers would
// make on a tile (the sizes of their word-level spheres): small unions empty
// the intersection soonest and cost least, as PMS8's rows sorted by size do
// (Sec. 3.2.4). Any order gives the same set. With oe > 0 the masses are
// summed over the 4^oe sibling tiles that share the prefix without its last
// oe bases (an l-mer at distance k from that shorter prefix is at k + j from
// C(oe,j) 3^j of the siblings). Writes sh.torder[0..n); ends with a barrier.
// The caller's previous use of sh.U must be over by the first barrier here.
template <int TPB>
__device__ void order_strings(const InstDev &I, uint32_t Phi, uint32_t Plo,
                              uint32_t premask, int oe, TileShared &sh,
                              const Tables &tb)
{
    constexpr int kWaves = TPB / 64;
    const int tid = threadIdx.x;
    const int q = I.s - 3, pl = I.l - I.s;
    const uint32_t omask = premask & ~(((1u << oe) - 1u) << (pl - oe));
    if (tid <= I.d) {
        uint32_t v = 0, cf = 1;
        for (int j = 0; j <= oe && tid + j <= I.d; j++) {
            v += cf * (uint32_t)tb.ball_off[q * 8 + min(I.d - tid - j, q) + 1];
            cf = cf * 3u * (uint32_t)(oe - j) / (uint32_t)(j + 1);
        }
        sh.cw[tid] = v;   // indexed by k, not by the radius d - k
    }
    __syncthreads();
    // one wave per string; each lane loads kOrdPer l-mers at once so that a
    // string costs about one round trip to L2
    constexpr int kOrdPer = TPB >= kTPBWide ? 4 : 8;
    const int wid = tid >> 6, lane = tid & 63;
    for (int i = wid; i < I.n; i += kWaves) {
        const PlaneRow yp = planes_row(I.planes, (size_t)i * I.L);
        uint32_t mass = 0;
        for (int j0 = lane; j0 < I.L; j0 += 64 * kOrdPer) {
            uint2 y[kOrdPer];
#pragma unroll
            for (int u = 0; u < kOrdPer; u++)
                y[u] = yp[min(j0 + 64 * u, I.L - 1)];
#pragma unroll
            for (int u = 0; u < kOrdPer; u++) {
                const int k = __popc(((y[u].x ^ Phi) | (y[u].y ^ Plo)) &
                                     omask);
                if (j0 + 64 * u < I.L && k <= I.d)
                    mass += sh.cw[k];
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            mass += __shfl_xor(mass, o, 64);
        if (lane == 0)
            sh.mass[i] = mass;
    }
    __syncthreads();
    if (tid < I.n) {
        const uint32_t mi = sh.mass[tid];
        int rank = 0;
        for (int j = 0; j < I.n; j++) {
            const uint32_t mj = sh.mass[j];
            rank += (mj < mi) || (mj == mi && j < tid);
        }
        sh.torder[rank] = tid;
    }
    __syncthreads();
}

template <int TPB>
__device__ void run_tile(const InstDev &I, uint64_t t, TileShared &sh,
                         const Tables &tb, StatAcc &acc, int order_mode)
{
    constexpr int kTPB = TPB, kWaves = TPB / 64;
    constexpr int kWordsPerThread = kMaxWords / TPB;
    // l-mers per lane in the survivor stage (one round covers 768 or 1024)
    constexpr int kFiltPer = TPB >= kTPBWide ? 2 : 3;
    uint32_t *tile_cnt = I.tile_cnt;
    uint64_t *tile_heap_off = I.tile_heap_off;
    uint64_t *heap = I.heap;
    unsigned long long *heap_top = I.heap_top;
    const unsigned long long heap_cap = I.heap_cap;
    const int tid = threadIdx.x;
    const int s = I.s, q = s - 3, pl = I.l - s;
    const int W = 1 << (2 * q);
    const uint64_t g = t;
    uint32_t Phi, Plo;
    prefix_planes(t, pl, Phi, Plo);
    const uint32_t premask = (pl >= 32) ? ~0u : ((1u << pl) - 1u);
    // Strings in ascending order of their sphere mass on this tile (see
    // order_strings). The host turns it on where a pass's marks outweigh the
    // n*L prefix tests it costs. order_mode: 0 keeps the previous tile's
    // order, 1 orders for this tile alone, 2 for the kOrderReuse sibling
    // tiles that share the prefix without its last log4(kOrderReuse) bases.
    const bool tile_order = I.tile_order != 0 && I.n <= kOrderMax;
    const bool make_order = tile_order && order_mode != 0;
    const int oe = (order_mode == 2) ? min(kOrderReuseLog4, pl) : 0;
    if (make_order)
        order_strings<TPB>(I, Phi, Plo, premask, oe, sh, tb);
    else
        __syncthreads();   // the previous tile may still be reading sh.U

    // the running intersection; every code is in it before the first string
    unsigned long long A[kWordsPerThread];
#pragma unroll
    for (int k = 0; k < kWordsPerThread; k++)
        A[k] = ~0ull;
    uint32_t total = 0;
    int si = 0;
    bool to_filter = false;
    for (si = 0; si < I.n; si++) {
        const int seq = tile_order ? uni(sh.torder[si]) : uni(I.order[si]);
        // U is all zero here: cleared at kernel start, by the previous
        // pass's AND step, or after the previous tile's emission
        const unsigned long long mk = mark_string<TPB>(I, seq, Phi, Plo, premask,
                                                  sh, tb);
        uint32_t cnt = 0;
        // word tid + k*kTPB sits at wpos(tid) ^ wpos(k*kTPB) (wpos is
        // XOR-linear, the two parts share no bits); the base is made opaque
        // per pass so that the compiler does not hold one address per word
        // across the pass loop (at 64 VGPRs it spilled them to scratch)
        uint32_t tw = (uint32_t)tid;
        asm volatile("" : "+v"(tw));
        const uint32_t pbase = wpos(tw);
#pragma unroll
        for (int k = 0; k < kWordsPerThread; k++) {
            const int w = tid + k * kTPB;
            if (w < W) {
                const uint32_t pw = pbase ^ wpos((uint32_t)(k * kTPB));
                // read and clear in one LDS instruction
                const unsigned long long u = __hip_atomic_exchange(
                    &sh.U[pw], 0ull, __ATOMIC_RELAXED,
                    __HIP_MEMORY_SCOPE_WORKGROUP);
                A[k] &= u;
                cnt += (uint32_t)__popcll(A[k]);
            }
        }
        // at most 4^9 codes: the count fits in 32 bits
        total = block_sum32<TPB>(cnt, sh.redc[acc.passes & 1]);
        // work counters: every thread adds the same (uniform) amounts, so
        // they stay in scalar registers (thread 0 flushes them at the end)
        acc.passes++;
        acc.marks += mk;
        if (total == 0)
            break;
        if (total <= (uint32_t)I.surv_t && si + 1 < I.n) {
            to_filter = true;
            break;
        }
    }
    acc.tiles++;
    if (total == 0) {
        if (tid == 0) {
            tile_cnt[g] = 0;
            tile_heap_off[g] = 0;
        }
        return;
    }
    if (!to_filter) {
        // every string ANDed in: all remaining codes are motifs; the
        // intersection goes back to LDS, in word order, and out in code order
#pragma unroll
        for (int k = 0; k < kWordsPerThread; k++) {
            const int w = tid + k * kTPB;
            if (w < W)
                sh.U[w] = A[k];
        }
        __syncthreads();
        emit_tile<TPB>(sh, W, t, g, s, I);
        __syncthreads();
        for (int w = tid; w < W; w += kTPB)   // U is zero for the next tile
            sh.U[w] = 0;
        return;
    }

    // ---- filter stage: test the few codes left against the rest --------
    // The live codes (at most surv_t <= kSurvMax) are listed straight from
    // the registers with their bit planes, into LDS words that are all zero
    // at this point (U was cleared as it was read). Each lane holds up to
    // kFiltPer l-mers of the current string in registers, loaded one string
    // ahead, and every wave tests every live code (read from LDS with one
    // broadcast per wave) against its l-mers; a code with a hit in any wave
    // is flagged and the unflagged ones drop out before the next string.
    // The list is in thread order; the survivors are ranked by code when
    // they are written out.
    uint2 *const plb0 = reinterpret_cast<uint2 *>(sh.U);
    uint2 *const plb1 = plb0 + kSurvMax;
    uint64_t *const cdb1 = reinterpret_cast<uint64_t *>(sh.U) + 2 * kSurvMax;
    const int L = I.L;
    int N;
    {
        unsigned int c = 0;
#pragma unroll
        for (int k = 0; k < kWordsPerThread; k++)
            if (tid + k * kTPB < W)
                c += (unsigned int)__popcll(A[k]);
        unsigned int nt;
        unsigned int pos = block_exscan<TPB>(c, sh.red32, &nt);
        const uint64_t base = t << (2 * s);
#pragma unroll
        for (int k = 0; k < kWordsPerThread; k++) {
            const int w = tid + k * kTPB;
            unsigned long long v = (w < W) ? A[k] : 0ull;
            // (pos < kSurvMax always: the pass count that sent the tile
            // here is the same number; the bound only keeps the writes in
            // the buffer whatever happens)
            while (v && pos < (unsigned int)kSurvMax) {
                const int b = __ffsll(v) - 1;
                v &= v - 1;
                const uint64_t code = base | ((uint64_t)w << 6) | (uint64_t)b;
                sh.surv[pos] = code;
                plb0[pos] = code_planes(code, I.l);
                pos++;
            }
        }
        N = (int)min(nt, (unsigned int)kSurvMax);
    }
    auto seq_at = [&](int j) {
        return tile_order ? uni(sh.torder[j]) : uni(I.order[j]);
    };
    // l-mers of a round: lane t holds l-mers r0 + kFiltPer*t + u, so that
    // they fill the first ceil(L/kFiltPer) lanes and the waves past them
    // skip the round; past the end, the last l-mer again (a repeat leaves
    // every minimum unchanged)
    auto load_ys = [&](int sq, int r0, uint2 (&y)[kFiltPer]) {
        const uint2 *row = I.planes + (size_t)sq * (size_t)L;
#pragma unroll
        for (int u = 0; u < kFiltPer; u++)
            y[u] = row[min(r0 + kFiltPer * tid + u, L - 1)];
    };
    constexpr int kRound = kFiltPer * kTPB;
    constexpr int kMaskWords = kSurvMax / 64;
    const int rounds = (L + kRound - 1) / kRound;
    const int lane = tid & 63;
    const int wid = uni(tid >> 6);
    uint2 y[kFiltPer];
    if (si + 1 < I.n)
        load_ys(seq_at(si + 1), 0, y);
    if (tid < 2 * kMaskWords)
        (&sh.hitm[0][0])[tid] = 0ull;
    __syncthreads();   // the list is complete, the hit masks are clear
    int cur = 0;
    for (int sj = si + 1; sj < I.n && N > 0; sj++) {
        acc.ftests += (unsigned long long)N * (unsigned long long)L;
        const uint2 *plc = cur ? plb1 : plb0;
        const uint64_t *cdc = cur ? cdb1 : sh.surv;
        const int par = (sj - si - 1) & 1;
        for (int r = 0; r < rounds; r++) {
            // the next load: this string's next round, else the next
            // string's first
            uint2 yn[kFiltPer];
            if (r + 1 < rounds)
                load_ys(seq_at(sj), (r + 1) * kRound, yn);
            else if (sj + 1 < I.n)
                load_ys(seq_at(sj + 1), 0, yn);
            // a wave whose lanes hold no l-mer of this round has nothing
            // to test
            if (r * kRound + kFiltPer * 64 * wid < L) {
                // the codes in blocks of 64: bit v of hm = some lane of the
                // wave has an l-mer within d of code kb*64 + v
                for (int kb = 0; kb * 64 < N; kb++) {
                    unsigned long long hm = 0;
                    const int cend = min(N, kb * 64 + 64);
                    for (int c0 = kb * 64; c0 < cend; c0 += 4) {
                        uint2 cp[4];
#pragma unroll
                        for (int v = 0; v < 4; v++)
                            cp[v] = plc[min(c0 + v, N - 1)];
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            uint32_t h = 255;
#pragma unroll
                            for (int u = 0; u < kFiltPer; u++)
                                h = min(h, (uint32_t)__popc((cp[v].x ^ y[u].x) |
                                                            (cp[v].y ^ y[u].y)));
                            if (__ballot(h <= (uint32_t)I.d) != 0)
                                hm |= 1ull << (c0 + v - kb * 64);
                        }
                    }
                    // codes past the end repeated code N-1: drop their bits
                    const int nv = cend - kb * 64;
                    if (nv < 64)
                        hm &= (1ull << nv) - 1ull;
                    if (lane == 0 && hm != 0)
                        atomicOr(&sh.hitm[par][kb], hm);
                }
            }
#pragma unroll
            for (int u = 0; u < kFiltPer; u++)
                y[u] = yn[u];
        }
        __syncthreads();   // every wave's hits are in
        // the codes with a hit stay, in their order: a code's new index is
        // the number of kept codes before it
        unsigned long long mk[kMaskWords];
        int nkeep = 0;
#pragma unroll
        for (int k = 0; k < kMaskWords; k++) {
            mk[k] = uni(sh.hitm[par][k]);
            nkeep += __popcll(mk[k]);
        }
        if (tid < N) {
            const int kw = tid >> 6;
            const unsigned long long below = (1ull << (tid & 63)) - 1ull;
            int pos = 0;
            bool keep = false;
#pragma unroll
            for (int k = 0; k < kMaskWords; k++) {
                if (k < kw)
                    pos += __popcll(mk[k]);
                if (k == kw) {
                    pos += __popcll(mk[k] & below);
                    keep = (mk[k] >> (tid & 63)) & 1ull;
                }
            }
            if (keep) {
                (cur ? plb0 : plb1)[pos] = plc[tid];
                (cur ? sh.surv : cdb1)[pos] = cdc[tid];
            }
        }
        // the other string parity's masks were last read before this
        // string started: clear them for the next string
        if (tid < kMaskWords)
            sh.hitm[par ^ 1][tid] = 0ull;
        __syncthreads();
        cur ^= 1;
        N = nkeep;
    }
    // the survivors into the heap, each at its rank among them by code
    const uint64_t *cdc = cur ? cdb1 : sh.surv;
    if (tid == 0) {
        unsigned long long off = 0;
        if (N)
            off = atomicAdd(heap_top, (unsigned long long)N);
        sh.bcast = off;
        tile_cnt[g] = (uint32_t)N;
        tile_heap_off[g] = off;
    }
    __syncthreads();
    const unsigned long long off = sh.bcast;
    if (tid < N && off + (unsigned long long)N <= heap_cap) {
        const uint64_t me = cdc[tid];
        int rank = 0;
        for (int j = 0; j < N; j++)
            rank += cdc[j] < me ? 1 : 0;
        heap[off + rank] = me;
    }
    __syncthreads();
    // clear the scratch words for the next tile
    for (int w = tid; w < kFiltWords; w += kTPB)
        sh.U[w] = 0;
}

// One tile of the quorum path (q < n, Definition 5): every code of the tile
// keeps a count of the strings so far without a d-neighbour of it, bit-sliced
// (plane p holds bit p of the counts of 64 codes) in registers. A code stays
// live while its count is at most n - q; a string ORs its sphere union into
// U as on the plain path and every live code outside U counts one more miss.
// The tile stops when no code is live; after the last string the live codes
// are exactly the (l,d,q)-motifs of the tile.
constexpr int kQTileWords = 1 << (2 * (kQuorumMaxSuffix - 3));
constexpr int kQPlanes = 5;   // counts 0..kQuorumMaxMiss + 1
static_assert(kQTileWords >= kTPBWide && (kQuorumMaxMiss + 1) < (1 << kQPlanes),
              "quorum counters");

template <int TPB>
__device__ void run_tile_quorum(const InstDev &I, uint64_t t, TileShared &sh,
                                const Tables &tb, StatAcc &acc)
{
    constexpr int kTPB = TPB;
    constexpr int kQWords = kQTileWords / TPB;   // words per thread
    const int tid = threadIdx.x;
    const int s = I.s, q = s - 3, pl = I.l - s;
    const int W = 1 << (2 * q);
    const int T = I.n - I.q;                  // misses a motif may have
    uint32_t Phi, Plo;
    prefix_planes(t, pl, Phi, Plo);
    const uint32_t premask = (pl >= 32) ? ~0u : ((1u << pl) - 1u);
    __syncthreads();   // the previous tile may still be reading sh.U

    // Every counter starts at 2^kQPlanes - 1 - T: a code is still live
    // after T misses and its (T+1)-th miss carries out of the top plane,
    // which is the test itself (no compare with T per pass).
    unsigned long long C[kQPlanes][kQWords];
    unsigned long long live[kQWords];
    const uint32_t c0 = (uint32_t)((1 << kQPlanes) - 1 - T);
#pragma unroll
    for (int k = 0; k < kQWords; k++) {
        live[k] = (tid + k * kTPB < W) ? ~0ull : 0ull;
#pragma unroll
        for (int p = 0; p < kQPlanes; p++)
            C[p][k] = ((c0 >> p) & 1u) ? ~0ull : 0ull;
    }
    bool any = true;
    for (int si = 0; si < I.n; si++) {
        const int seq = uni(I.order[si]);
        const unsigned long long mk = mark_string<TPB>(I, seq, Phi, Plo, premask,
                                                  sh, tb);
        int nz = 0;
        // per-pass word addresses from an opaque tid (see run_tile)
        uint32_t tw = (uint32_t)tid;
        asm volatile("" : "+v"(tw));
        const uint32_t pbase = wpos(tw);
#pragma unroll
        for (int k = 0; k < kQWords; k++) {
            const int w = tid + k * kTPB;
            if (w < W) {
                const uint32_t pw = pbase ^ wpos((uint32_t)(k * kTPB));
                const unsigned long long u = sh.U[pw];
                sh.U[pw] = 0;
                // add 1 to the count of every live code outside U
                unsigned long long carry = live[k] & ~u;
#pragma unroll
                for (int p = 0; p < kQPlanes; p++) {
                    const unsigned long long c2 = C[p][k] & carry;
                    C[p][k] ^= carry;
                    carry = c2;
                }
                // a carry out of the top plane is the (T+1)-th miss
                live[k] &= ~carry;
                nz |= live[k] != 0;
            }
        }
        // work counters: every thread adds the same (uniform) amounts, so
        // they stay in scalar registers (thread 0 flushes them at the end)
        acc.passes++;
        acc.marks += mk;
        if (!__syncthreads_or(nz)) {
            any = false;
            break;
        }
    }
    acc.tiles++;
    if (!any) {
        if (tid == 0) {
            I.tile_cnt[t] = 0;
            I.tile_heap_off[t] = 0;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < kQWords; k++) {
        const int w = tid + k * kTPB;
        if (w < W)
            sh.U[w] = live[k];
    }
    __syncthreads();
    emit_tile<TPB>(sh, W, t, t, s, I);
    __syncthreads();
    for (int w = tid; w < W; w += kTPB)   // U is zero for the next tile
        sh.U[w] = 0;
}

// Persistent loop shared by the tiled kernels: workgroups take work items
// (tile ranges) from a counter until none is left.
template <int TPB, bool Quorum>
__device__ __forceinline__ void drain_items(const InstDev *insts,
                                            const WorkItem *items, int nitems,
                                            uint64_t chunk, unsigned int *next,
                                            const Tables &tb, TileStats *stats)
{
    constexpr int kTPB = TPB;
    __shared__ TileShared sh;
    __shared__ int s_item;
    for (int i = threadIdx.x; i < 256; i += kTPB)
        sh.m3[i] = tb.m3[i];
    for (int i = threadIdx.x; i < kMaxWords; i += kTPB)
        sh.U[i] = 0;
    StatAcc acc = {0, 0, 0, 0};
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_item = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int it = uni(s_item);
        if (it >= nitems)
            break;
        WorkItem w;
        if (items) {
            w = items[it];
        } else {
            // implicit list: instance 0 split into chunks of `chunk` tiles
            w.inst = 0;
            w.t0 = (uint64_t)it * chunk;
            w.t1 = min(w.t0 + chunk, insts[0].ntiles);
        }
        w.inst = uni(w.inst);
        w.t0 = uni((unsigned long long)w.t0);
        w.t1 = uni((unsigned long long)w.t1);
        // the descriptor in scalar registers: it removed the VGPR spills of
        // the 512-thread and quorum kernels; the plain 256-thread kernel
        // has none and only gained SGPR spills from it
        const InstDev I = (TPB >= kTPBWide || Quorum)
                              ? uni_desc(insts[w.inst])
                              : insts[w.inst];
        for (uint64_t t = w.t0; t < w.t1; t++) {
            if (Quorum)
                run_tile_quorum<TPB>(I, t, sh, tb, acc);
            else
                run_tile<TPB>(I, t, sh, tb, acc,
                         (t != w.t0 && (t & (uint64_t)(kOrderReuse - 1)) != 0)
                             ? 0
                             : (w.t1 - w.t0 >= 2 ? 2 : 1));
        }
    }
    if (threadIdx.x == 0 && stats) {
        atomicAdd(&stats->passes, acc.passes);
        atomicAdd(&stats->marks, acc.marks);
        atomicAdd(&stats->ftests, acc.ftests);
        atomicAdd(&stats->tiles, acc.tiles);
    }
}

// (launch bounds: four workgroups per CU, i.e. TPB/64 waves per SIMD)
__global__ __launch_bounds__(kTPB, kTPB / 64) void
k_tiled(const InstDev *insts, const WorkItem *items, int nitems,
        uint64_t chunk, unsigned int *next, Tables tb, TileStats *stats)
{
    drain_items<kTPB, false>(insts, items, nitems, chunk, next, tb, stats);
}

__global__ __launch_bounds__(kTPBWide, kTPBWide / 64) void
k_tiled_512(const InstDev *insts, const WorkItem *items, int nitems,
            uint64_t chunk, unsigned int *next, Tables tb, TileStats *stats)
{
    drain_items<kTPBWide, false>(insts, items, nitems, chunk, next, tb,
                                 stats);
}

// 256 threads: at 512 the bit-sliced counters spill at 64 VGPRs; with the
// preloaded counters that costs about what the extra waves gain
constexpr int kQuorumTPB = kTPB;

__global__ __launch_bounds__(kQuorumTPB, kQuorumTPB / 64) void
k_tiled_quorum(const InstDev *insts, const WorkItem *items, int nitems,
               uint64_t chunk, unsigned int *next, Tables tb,
               TileStats *stats)
{
    drain_items<kQuorumTPB, true>(insts, items, nitems, chunk, next, tb,
                                  stats);
}

hipError_t launch_tiled(const InstDev *d_insts, const WorkItem *d_items,
                        int nitems, uint64_t chunk, unsigned int *d_next,
                        Tables tb, TileStats *stats, int grid, hipStream_t st,
                        bool wide)
{
    if (nitems <= 0)
        return hipSuccess;
    if (wide)
        hipLaunchKernelGGL(k_tiled_512, dim3(grid), dim3(kTPBWide), 0, st,
                           d_insts, d_items, nitems, chunk, d_next, tb, stats);
    else
        hipLaunchKernelGGL(k_tiled, dim3(grid), dim3(kTPB), 0, st, d_insts,
                           d_items, nitems, chunk, d_next, tb, stats);
    return hipGetLastError();
}

hipError_t launch_tiled_quorum(const InstDev *d_insts, const WorkItem *d_items,
                               int nitems, uint64_t chunk,
                               unsigned int *d_next, Tables tb,
                               TileStats *stats, int grid, hipStream_t st)
{
    if (nitems <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_tiled_quorum, dim3(grid), dim3(kQuorumTPB), 0, st,
                       d_insts, d_items, nitems, chunk, d_next, tb, stats);
    return hipGetLastError();
}

int tiled_quorum_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiled_quorum,
                                                     kQuorumTPB, 0) != hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

int tiled_blocks_per_cu(bool wide)
{
    int nb = 0;
    const hipError_t e =
        wide ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiled_512,
                                                            kTPBWide, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tiled,
                                                            kTPB, 0);
    if (e != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

// ---- memory-heavy bitset path ---------------------------------------------

// raw buffer access (CDNA): the descriptor's last word for untyped 32-bit
// data, and the cache-policy operand that marks an access non-temporal
constexpr int kBufDword3 = 0x00020000;
constexpr int kBufNonTemporal = 2;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Byte p[i] (i uniform) through a scalar load of its aligned 32-bit word:
// scalar loads are waited on by their own counter, so this read does not
// wait for the vector stores still in flight (the previous tile's A). The
// buffer behind p must extend to the end of that word, and no launch that
// reads it may write it (the scalar cache is not kept coherent with vector
// stores): here, the per-tile string order.
__device__ __forceinline__ uint32_t uniform_byte(const uint8_t *p, uint64_t i)
{
    typedef const __attribute__((address_space(4))) uint32_t c_u32;
    const uintptr_t a = (uintptr_t)(p + i);
    const uint32_t w = *(c_u32 *)(const void *)(a & ~(uintptr_t)3);
    return (w >> (8u * (uint32_t)(a & 3u))) & 0xffu;
}

// One string pass of the memory-heavy path over every live tile. A tile's
// words of the resident intersection A are loaded into registers while its
// string's l-mers are listed and its sphere union marked in LDS; then
// A &= U is written back (U read and cleared in one LDS instruction) and
// the tile's liveness recorded. Pass 0 runs over every tile; each pass
// appends its live tiles to a list that the next pass runs over, so no pass
// scans dead tiles and the work shares stay even when the live tiles are
// clustered. Items are taken in chunks from a counter, sized from the
// list's length so that every workgroup gets several. 256 threads: the 16
// words of A per thread stay in registers without spills. With ord (n
// bytes per tile, from k_bitset_mass and k_bitset_rank) pass p ANDs each
// tile's p-th string in its own order, else string I.order[p] on every
// tile.
//
// cnt[2p] is pass p's chunk counter, cnt[2p+1] the length of the list pass
// p writes (lists[(p+1)&1]); all start at zero. kLoad is false for pass 0
// only, where A is all ones, nothing is read and the items are the tiles.
template <int TPB, bool kLoad>
__device__ void bitset_pass(const InstDev *inst, int pass, const Tables &tb,
                            unsigned long long *A, uint8_t *alive,
                            const uint8_t *ord, unsigned int *cnt,
                            uint32_t *const *lists, int chunk0,
                            TileStats *stats, TileShared &sh,
                            unsigned int &s_chunk)
{
    constexpr int kTPB = TPB;
    constexpr int kPer = kMaxWords / TPB;   // words of A per thread
    typedef const __attribute__((address_space(4))) uint32_t c_u32;
    __shared__ uint32_t s_keep[8];          // live tiles of a chunk (<= 8)
    const InstDev I = uni_desc(*inst);
    const int tid = threadIdx.x;
    const int s = I.s, q = s - 3, pl = I.l - s;
    const int W = 1 << (2 * q);
    const uint32_t premask = (pl >= 32) ? ~0u : ((1u << pl) - 1u);
    const int gseq = uni(I.order[pass]);
    const uint32_t *list_in = lists[pass & 1];
    uint32_t *list_out = lists[(pass + 1) & 1];
    // items: the tiles (pass 0) or the previous pass's live tiles
    uint64_t nitems = I.ntiles;
    uint64_t chunk = (uint64_t)chunk0;
    if (kLoad) {
        nitems = ((c_u32 *)(const void *)cnt)[2 * pass - 1];
        chunk = min<uint64_t>(8, max<uint64_t>(1, nitems /
                                                      (8ull * gridDim.x)));
    }
    for (int i = tid; i < 256; i += kTPB)
        sh.m3[i] = tb.m3[i];
    for (int i = tid; i < kMaxWords; i += kTPB)
        sh.U[i] = 0;
    unsigned long long marks = 0, passes = 0;
    const uint64_t nchunks = (nitems + chunk - 1) / chunk;
    for (;;) {
        __syncthreads();
        if (tid == 0)
            s_chunk = atomicAdd(&cnt[2 * pass], 1u);
        __syncthreads();
        const uint64_t ch = uni(s_chunk);
        if (ch >= nchunks)
            break;
        const uint64_t i1 = min((ch + 1) * chunk, nitems);
        unsigned int nkeep = 0;   // thread 0: the chunk's live tiles so far
        for (uint64_t it = ch * chunk; it < i1; it++) {
            // the list entry through a scalar load: it does not wait for
            // the previous tile's stores
            const uint64_t t =
                kLoad ? (uint64_t)((c_u32 *)(const void *)list_in)[it] : it;
            const int seq =
                ord ? (int)uniform_byte(ord, t * (uint64_t)I.n + pass) : gseq;
            unsigned long long *Ag = A + t * (uint64_t)W;
            unsigned long long a[kPer];
            uint32_t Phi, Plo;
            prefix_planes(t, pl, Phi, Plo);
            if constexpr (kLoad) {
                // A's words are loaded while the string's l-mers are listed
                // and its union marked, issued after the listing's own loads
                // so that the listing waits for its own loads only. Through a
                // buffer resource over the tile's W words: one address
                // register per load, and an access out of its range reads 0
                // without touching memory. That covers words past W (never
                // stored) and the later listing rounds of a long string,
                // whose resource has no range at all.
#pragma unroll
                for (int k = 0; k < kPer; k++)
                    a[k] = 0;
                marks += mark_string<kTPB>(
                    I, seq, Phi, Plo, premask, sh, tb, [&](int y0) {
                        const __amdgpu_buffer_rsrc_t rA =
                            __builtin_amdgcn_make_buffer_rsrc(
                                Ag, 0, y0 == 0 ? W * 8 : 0, kBufDword3);
#pragma unroll
                        for (int k = 0; k < kPer; k++) {
                            // streamed once per pass: non-temporal access
                            const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(
                                rA, (uint32_t)(tid + k * kTPB) * 8u, 0,
                                kBufNonTemporal);
                            a[k] |= ((unsigned long long)v.y << 32) | v.x;
                        }
                    });
            } else {
#pragma unroll
                for (int k = 0; k < kPer; k++)
                    a[k] = ~0ull;
                marks += mark_string<kTPB>(I, seq, Phi, Plo, premask, sh, tb);
            }
            passes++;
            // A's words are needed now: one wait for all of them here, so
            // that the stores below are not each followed by a wait for
            // every outstanding memory operation
#pragma unroll
            for (int k = 0; k < kPer; k++)
                asm volatile("" : "+v"(a[k]));
            int nz = 0;
            uint32_t tw = (uint32_t)tid;
            asm volatile("" : "+v"(tw));
            const uint32_t pbase = wpos(tw);
            // a tile of at least kTPB words (s >= 7) takes whole rows of
            // kTPB words, a uniform test; a smaller one its first W lanes
            const bool rows = W >= kTPB;
#pragma unroll
            for (int k = 0; k < kPer; k++) {
                const int w = tid + k * kTPB;
                if (rows ? (k * kTPB < W) : (k == 0 && tid < W)) {
                    const unsigned long long u = __hip_atomic_exchange(
                        &sh.U[pbase ^ wpos((uint32_t)(k * kTPB))], 0ull,
                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    const unsigned long long v = a[k] & u;
                    __builtin_nontemporal_store(v, &Ag[w]);
                    nz |= (v != 0);
                }
            }
            const int any = __syncthreads_or(nz);
            if (tid == 0) {
                alive[t] = (uint8_t)(any != 0);
                if (any)
                    s_keep[nkeep++] = (uint32_t)t;
            }
        }
        // the chunk's live tiles to the next pass's list with one atomic
        // (every workgroup appends to the same counter)
        if (tid == 0 && nkeep) {
            const unsigned int at = atomicAdd(&cnt[2 * pass + 1], nkeep);
            for (unsigned int k = 0; k < nkeep; k++)
                list_out[at + k] = s_keep[k];
        }
    }
    if (tid == 0 && stats) {
        atomicAdd(&stats->passes, passes);
        atomicAdd(&stats->marks, marks);
    }
}

#ifndef PMS_BITSET_TPB
#define PMS_BITSET_TPB 256
#endif
constexpr int kBitsetTPB = PMS_BITSET_TPB;

__global__ __launch_bounds__(kBitsetTPB, kBitsetTPB / 64) void
k_bitset_pass(const InstDev *inst, int pass, Tables tb,
              unsigned long long *A, uint8_t *alive, const uint8_t *ord,
              unsigned int *cnt, uint32_t *list0, uint32_t *list1, int chunk0,
              TileStats *stats)
{
    __shared__ TileShared sh;
    __shared__ unsigned int s_chunk;
    uint32_t *const lists[2] = {list0, list1};
    if (pass == 0)
        bitset_pass<kBitsetTPB, false>(inst, pass, tb, A, alive, ord, cnt,
                                       lists, chunk0, stats, sh, s_chunk);
    else
        bitset_pass<kBitsetTPB, true>(inst, pass, tb, A, alive, ord, cnt,
                                      lists, chunk0, stats, sh, s_chunk);
}

hipError_t launch_bitset_pass(const InstDev *d_inst, int pass, Tables tb,
                              unsigned long long *A, uint8_t *alive,
                              const uint8_t *ord, unsigned int *cnt,
                              uint32_t *list0, uint32_t *list1, int chunk0,
                              TileStats *stats, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_bitset_pass, dim3(grid), dim3(kBitsetTPB), 0, st,
                       d_inst, pass, tb, A, alive, ord, cnt, list0, list1,
                       chunk0, stats);
    return hipGetLastError();
}

// The bitset path's string order, per tile: ord[t*n + p] is the string that
// pass p ANDs into tile t, the strings in ascending order of their sphere
// mass on the tile (the masses order_strings computes for a tile alone;
// ties by string index). First k_bitset_mass, one thread per (tile,
// string): the string's l-mers are staged in LDS and every lane tests each
// of them (a broadcast read) against its own tile's prefix. Then
// k_bitset_rank, one thread per tile. The caller guarantees n <= kOrderMax.
constexpr int kOrderTPB = 128;
constexpr int kOrderChunk = 1024;   // l-mers staged at a time

__global__ __launch_bounds__(kOrderTPB) void
k_bitset_mass(const InstDev *inst, Tables tb, uint32_t *mass)
{
    __shared__ unsigned long long yrow[kOrderChunk];
    __shared__ uint32_t cw[kMaxL + 1];
    const InstDev I = uni_desc(*inst);
    const int tid = threadIdx.x, i = blockIdx.y;
    const int q = I.s - 3, pl = I.l - I.s, d = I.d, n = I.n, L = I.L;
    const uint32_t premask = (pl >= 32) ? ~0u : ((1u << pl) - 1u);
    // word marks of one reaching l-mer at prefix distance k (0 past d; the
    // distance is at most pl <= kMaxL)
    for (int k = tid; k <= kMaxL; k += kOrderTPB)
        cw[k] = k <= d ? (uint32_t)tb.ball_off[q * 8 + min(d - k, q) + 1] : 0u;
    const unsigned long long *row =
        (const unsigned long long *)(const void *)I.planes + (size_t)i * L;
    for (uint64_t t0 = (uint64_t)blockIdx.x * kOrderTPB; t0 < I.ntiles;
         t0 += (uint64_t)gridDim.x * kOrderTPB) {
        const uint64_t t = t0 + tid;
        uint32_t Phi, Plo;
        prefix_planes(t < I.ntiles ? t : 0, pl, Phi, Plo);
        uint32_t m = 0;
        for (int j0 = 0; j0 < L; j0 += kOrderChunk) {
            const int cnt = min(kOrderChunk, L - j0);
            __syncthreads();   // cw is set; the previous chunk has been read
            for (int j = tid; j < cnt; j += kOrderTPB)
                yrow[j] = row[j0 + j];
            __syncthreads();
#pragma unroll 8
            for (int j = 0; j < cnt; j++) {
                const unsigned long long y = yrow[j];
                const int k = __popc((((uint32_t)y ^ Phi) |
                                      ((uint32_t)(y >> 32) ^ Plo)) &
                                     premask);
                m += cw[k];
            }
        }
        if (t < I.ntiles)
            mass[t * (uint64_t)n + i] = m;
    }
}

__global__ __launch_bounds__(kTPB) void
k_bitset_rank(const InstDev *inst, const uint32_t *mass, uint8_t *ord)
{
    const InstDev I = uni_desc(*inst);
    const int n = I.n;
    for (uint64_t t = (uint64_t)blockIdx.x * kTPB + threadIdx.x; t < I.ntiles;
         t += (uint64_t)gridDim.x * kTPB) {
        const uint32_t *mt = mass + t * (uint64_t)n;
        for (int i = 0; i < n; i++) {
            const uint32_t mi = mt[i];
            int rank = 0;
            for (int j = 0; j < n; j++) {
                const uint32_t mj = mt[j];
                rank += (mj < mi) || (mj == mi && j < i);
            }
            ord[t * (uint64_t)n + rank] = (uint8_t)i;
        }
    }
}

hipError_t launch_bitset_order(const InstDev *d_inst, Tables tb,
                               uint32_t *mass, uint8_t *ord, uint64_t ntiles,
                               int n, hipStream_t st)
{
    const uint64_t mblocks = (ntiles + kOrderTPB - 1) / kOrderTPB;
    hipLaunchKernelGGL(k_bitset_mass,
                       dim3((unsigned)std::min<uint64_t>(mblocks, 65535),
                            (unsigned)n),
                       dim3(kOrderTPB), 0, st, d_inst, tb, mass);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const uint64_t rblocks = (ntiles + kTPB - 1) / kTPB;
    hipLaunchKernelGGL(k_bitset_rank,
                       dim3((unsigned)std::min<uint64_t>(rblocks, 65535)),
                       dim3(kTPB), 0, st, d_inst, mass, ord);
    return hipGetLastError();
}

int bitset_blocks_per_cu()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bitset_pass,
                                                     kBitsetTPB, 0) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

__global__ __launch_bounds__(kTPB) void
k_bitset_count(const InstDev *inst, const unsigned long long *A,
               const uint8_t *alive, uint32_t *tile_cnt)
{
    __shared__ unsigned long long red[kWaves];
    const InstDev I = *inst;
    const int W = 1 << (2 * (I.s - 3));
    for (uint64_t t = blockIdx.x; t < I.ntiles; t += gridDim.x) {
        unsigned long long c = 0;
        if (alive[t]) {
            const unsigned long long *Ag = A + t * (uint64_t)W;
            for (int w = threadIdx.x; w < W; w += kTPB)
                c += __popcll(Ag[w]);
        }
        c = block_sum64<kTPB>(c, red);
        if (threadIdx.x == 0)
            tile_cnt[t] = (uint32_t)c;
    }
}

hipError_t launch_bitset_count(const InstDev *d_inst,
                               const unsigned long long *A,
                               const uint8_t *alive, uint32_t *tile_cnt,
                               int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_bitset_count, dim3(grid), dim3(kTPB), 0, st, d_inst,
                       A, alive, tile_cnt);
    return hipGetLastError();
}

__global__ __launch_bounds__(kTPB) void
k_bitset_emit(const InstDev *inst, const unsigned long long *A,
              const uint32_t *tile_cnt, const uint64_t *tile_pos,
              uint64_t *out, unsigned long long cap)
{
    __shared__ TileShared sh;
    const InstDev I = *inst;
    const int W = 1 << (2 * (I.s - 3));
    for (uint64_t t = blockIdx.x; t < I.ntiles; t += gridDim.x) {
        if (tile_cnt[t] == 0)
            continue;
        const unsigned long long *Ag = A + t * (uint64_t)W;
        for (int w = threadIdx.x; w < W; w += kTPB)
            sh.U[w] = Ag[w];
        __syncthreads();
        const uint64_t pos = tile_pos[t];
        const bool fits = pos + tile_cnt[t] <= cap;
        emit_words<kTPB>(sh, W, t, I.s, out + (fits ? pos : 0), fits, sh.red32);
        __syncthreads();
    }
}

hipError_t launch_bitset_emit(const InstDev *d_inst,
                              const unsigned long long *A,
                              const uint32_t *tile_cnt,
                              const uint64_t *tile_pos, uint64_t *out,
                              unsigned long long cap, int grid,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_bitset_emit, dim3(grid), dim3(kTPB), 0, st, d_inst,
                       A, tile_cnt, tile_pos, out, cap);
    return hipGetLastError();
}

}  // namespace pms
