// pms_wide.h -- long motifs (l up to 64): the device job, the launchers and
// the 128-bit code type shared by the long-motif kernels and the sort.
//
// Sec. 3.3.1 keeps an l-mer in ceil(l/32) words per group when one word is
// too short; here each group (bit plane) of an l-mer is one 64-bit word, and
// a motif code (first base in the top digit) takes 128 bits.
#pragma once

#include "pms_internal.h"

namespace pms {

constexpr int kWideMaxL = 64;

// A motif code of up to 128 bits, high word first (the output layout:
// motif i is words 2i and 2i+1).
struct W128 {
    uint64_t hi, lo;
};

struct WideJob {
    const ulonglong2 *planes;    // n*L l-mers: .x high plane, .y low plane,
                                 //   bit p = base p of the l-mer
    const uint64_t *posset;      // position sets (bit masks over the l
                                 //   positions) of every weight k <= d
    const uint64_t *posoff;      // weight k starts at posset[posoff[k]]
    const uint64_t *cum;         // first sphere index of weight k
    const uint64_t *pow3;        // 3^k
    uint64_t nb;                 // sphere size n_B(l, d)
    W128 *heap;                  // survivors, unordered, no repeats
    unsigned long long *heap_top;
    unsigned long long heap_cap;
    unsigned long long *hcanon;  // canonical Hamming tests (L per string
                                 //   examined, first failing one included)
    int n, m, l, d, L;
};

// Validates the bytes (first bad one: atomicMin of row*m+col into *bad) and
// writes the two 64-bit planes of every l-mer.
hipError_t launch_wide_index(const uint8_t *seqs, int n, int m, int l,
                             ulonglong2 *planes, unsigned long long *bad,
                             hipStream_t st);
// The sample-driven filter over the spheres of the l-mers of s_1; *next is
// the work-item counter (zero before the launch).
hipError_t launch_wide_filter(const WideJob &J, unsigned long long *next,
                              int grid, hipStream_t st);
int wide_blocks_per_cu();

// Ascending sort of 128-bit codes (key_bits: the low bits that may be set).
size_t sort_scratch_bytes_w128(uint64_t n);
hipError_t launch_sort_w128(W128 *keys, uint64_t n, int key_bits,
                            void *scratch, hipStream_t st);

}  // namespace pms
