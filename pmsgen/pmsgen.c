/*
 * pmsgen.c -- seeded synthetic planted-motif instances (FM model).
 *
 * This module only draws random inputs. It contains none of the motif-search
 * arithmetic (no Hamming distance, no neighbourhoods, no filtering), so both
 * the CPU oracle and the GPU library can consume its bytes without sharing
 * any code with each other.
 *
 * Generator: xoshiro256** 1.0 (Blackman and Vigna, "Scrambled linear
 * pseudorandom number generators", 2018), state filled from the seed by
 * SplitMix64 (Steele, Lea and Flood, 2014), as recommended by its authors.
 * Bounded integers use Lemire's multiply-and-reject method (2019), which is
 * exactly uniform.
 *
 * Planting rule (the FM model of Pevzner and Sze that the thesis's datasets
 * follow, with the details fixed here):
 *   1. background: n*m bases row-major, each uniform over {A,C,G,T}; one
 *      64-bit draw yields 32 bases, base k taken from bits 2k..2k+1;
 *   2. motif: l bases, one bounded draw in [0,4) each;
 *   3. for each sequence in order: its start position uniform in [0,m-l];
 *      its d mutated positions by a partial Fisher-Yates shuffle of [0,l);
 *      each mutated base b replaced by (b + 1 + U{0,1,2}) mod 4, i.e. one of
 *      the three other bases uniformly; the occurrence overwrites the
 *      background.
 * Bases are emitted as ASCII with A=0, C=1, G=2, T=3.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t s[4];
} pmsgen_rng;

static uint64_t splitmix64_next(uint64_t *x)
{
    uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t rotl64(uint64_t x, int k)
{
    return (x << k) | (x >> (64 - k));
}

uint64_t pmsgen_splitmix64(uint64_t *state)
{
    return splitmix64_next(state);
}

void pmsgen_seed(pmsgen_rng *r, uint64_t seed)
{
    uint64_t x = seed;
    for (int i = 0; i < 4; i++)
        r->s[i] = splitmix64_next(&x);
}

uint64_t pmsgen_next(pmsgen_rng *r)
{
    uint64_t *s = r->s;
    const uint64_t result = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return result;
}

/* Uniform integer in [0, range), range >= 1 (Lemire 2019). */
uint64_t pmsgen_bounded(pmsgen_rng *r, uint64_t range)
{
    uint64_t x = pmsgen_next(r);
    __uint128_t m = (__uint128_t)x * range;
    uint64_t lo = (uint64_t)m;
    if (lo < range) {
        uint64_t t = (0 - range) % range;
        while (lo < t) {
            x = pmsgen_next(r);
            m = (__uint128_t)x * range;
            lo = (uint64_t)m;
        }
    }
    return (uint64_t)(m >> 64);
}

/* Uniform double in [0,1) from the top 53 bits of one draw. */
double pmsgen_uniform01(pmsgen_rng *r)
{
    return (double)(pmsgen_next(r) >> 11) * (1.0 / 9007199254740992.0);
}

static const char kBase[4] = {'A', 'C', 'G', 'T'};

/*
 * Fill seqs (n*m bytes, row-major ASCII), motif (l bytes ASCII), pos (n
 * start positions) and mut (n*d mutated offsets within the occurrence, in
 * draw order). motif, pos and mut may be NULL. Returns 0, or -1 on bad sizes.
 */
int pmsgen_planted(uint64_t seed, int n, int m, int l, int d, char *seqs,
                   char *motif, int32_t *pos, int32_t *mut)
{
    if (n < 1 || m < 1 || l < 1 || l > m || d < 0 || d > l || !seqs)
        return -1;
    pmsgen_rng r;
    pmsgen_seed(&r, seed);
    size_t total = (size_t)n * (size_t)m;
    uint64_t word = 0;
    for (size_t k = 0; k < total; k++) {
        if ((k & 31) == 0)
            word = pmsgen_next(&r);
        seqs[k] = kBase[(word >> (2 * (k & 31))) & 3];
    }
    unsigned char mot[64];
    unsigned char *mb = (l <= 64) ? mot : (unsigned char *)malloc((size_t)l);
    int *idx = (int *)malloc(sizeof(int) * (size_t)l);
    if (!mb || !idx) {
        if (mb != mot)
            free(mb);
        free(idx);
        return -1;
    }
    for (int j = 0; j < l; j++)
        mb[j] = (unsigned char)pmsgen_bounded(&r, 4);
    if (motif)
        for (int j = 0; j < l; j++)
            motif[j] = kBase[mb[j]];
    for (int i = 0; i < n; i++) {
        int p = (int)pmsgen_bounded(&r, (uint64_t)(m - l + 1));
        char *occ = seqs + (size_t)i * m + p;
        for (int j = 0; j < l; j++) {
            idx[j] = j;
            occ[j] = kBase[mb[j]];
        }
        for (int t = 0; t < d; t++) {
            int q = t + (int)pmsgen_bounded(&r, (uint64_t)(l - t));
            int tmp = idx[t];
            idx[t] = idx[q];
            idx[q] = tmp;
            int b = mb[idx[t]];
            int nb = (b + 1 + (int)pmsgen_bounded(&r, 3)) & 3;
            occ[idx[t]] = kBase[nb];
            if (mut)
                mut[(size_t)i * d + t] = idx[t];
        }
        if (pos)
            pos[i] = p;
    }
    if (mb != mot)
        free(mb);
    free(idx);
    return 0;
}

/* Opaque-handle helpers for ctypes callers. */
pmsgen_rng *pmsgen_rng_new(uint64_t seed)
{
    pmsgen_rng *r = (pmsgen_rng *)malloc(sizeof(pmsgen_rng));
    if (r)
        pmsgen_seed(r, seed);
    return r;
}

/* The same FM-model planting over an alphabet of sigma letters (the bytes
 * alpha[0..sigma-1], 2 <= sigma <= 32): background letters row-major, one
 * bounded draw each; the motif (l draws); then per string a start position,
 * d distinct positions (partial Fisher-Yates) and for each a letter among
 * the sigma-1 others, (b + 1 + U{0..sigma-2}) mod sigma. */
int pmsgen_planted_alpha(uint64_t seed, int n, int m, int l, int d,
                         const char *alpha, int sigma, char *seqs,
                         char *motif)
{
    if (n < 1 || m < 1 || l < 1 || l > m || d < 0 || d > l || !seqs ||
        !alpha || sigma < 2 || sigma > 32)
        return -1;
    pmsgen_rng r;
    pmsgen_seed(&r, seed);
    size_t total = (size_t)n * (size_t)m;
    for (size_t k = 0; k < total; k++)
        seqs[k] = alpha[pmsgen_bounded(&r, (uint64_t)sigma)];
    int *mb = (int *)malloc(sizeof(int) * (size_t)l);
    int *idx = (int *)malloc(sizeof(int) * (size_t)l);
    if (!mb || !idx) {
        free(mb);
        free(idx);
        return -1;
    }
    for (int j = 0; j < l; j++)
        mb[j] = (int)pmsgen_bounded(&r, (uint64_t)sigma);
    if (motif)
        for (int j = 0; j < l; j++)
            motif[j] = alpha[mb[j]];
    for (int i = 0; i < n; i++) {
        int p = (int)pmsgen_bounded(&r, (uint64_t)(m - l + 1));
        char *occ = seqs + (size_t)i * m + p;
        for (int j = 0; j < l; j++) {
            idx[j] = j;
            occ[j] = alpha[mb[j]];
        }
        for (int t = 0; t < d; t++) {
            int q = t + (int)pmsgen_bounded(&r, (uint64_t)(l - t));
            int tmp = idx[t];
            idx[t] = idx[q];
            idx[q] = tmp;
            int b = mb[idx[t]];
            int nb = (b + 1 + (int)pmsgen_bounded(&r, (uint64_t)(sigma - 1))) %
                     sigma;
            occ[idx[t]] = alpha[nb];
        }
    }
    free(mb);
    free(idx);
    return 0;
}

void pmsgen_rng_free(pmsgen_rng *r)
{
    free(r);
}
