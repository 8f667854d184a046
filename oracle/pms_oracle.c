/*
 * pms_oracle.c -- plain, slow CPU oracle for exact planted (l,d)-motif search.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it. It shares no code with the GPU library.
 *
 * What it computes (Sec. 1.2.5, Definitions 1-5 and the qPMS definition
 * with q = n, which is plain PMS):
 *
 *   R(s_1..s_n, l, d) = all l-mers M over {A,C,G,T} such that every input
 *   string s_i has an l-mer y (one of its m-l+1 substrings of length l)
 *   with Hamming distance d_H(M, y) <= d.
 *
 * Readings taken where the text is silent or garbled:
 *   - an l-mer of s starts at any of the m-l+1 offsets, the last one
 *     included (Definition 2 is garbled; this is its evident meaning);
 *   - "no more than d" means <= d (Definition 5);
 *   - bases are coded A=0, C=1, G=2, T=3, as in the compression example of
 *     Sec. 3.3.1 (AGGCTA -> 022130); any other byte is an input error;
 *   - a motif is reported as the integer sum_j code(M[j]) * 4^(l-1-j): first
 *     base in the highest digit, so numeric order is lexicographic order;
 *   - one strand only (reverse complements are never mentioned).
 *
 * Two independent ways to get R:
 *   O1 (sample-driven, Sec. 1.3.1 and Observation 3.1 with q = n): every
 *      motif lies in the d-sphere B(x,d) of some l-mer x of the first string,
 *      so enumerate each B(x,d) (the tree T_d(x) of Sec. 3.2.1, every node
 *      once) and keep the candidates that have a d-neighbour in every other
 *      string, testing the strings in input order and stopping at the first
 *      one with none. The candidate test uses a packed XOR/popcount Hamming
 *      distance written here (Sec. 3.3.1 describes the bitwise form).
 *   O0 (pattern-driven, Sec. 1.3.1): try every one of the 4^l l-mers and
 *      compare it character by character with every l-mer of every string.
 *
 * Quorum (the qPMS definition with q <= n, Definition 5): M is an
 * (l,d,q)-motif when at least q of the n strings have an l-mer within
 * distance d of it. Two more independent ways to get that set:
 *   Q1 (Observation 3.1): the first string in which a motif has a
 *      d-neighbour is one of s_1..s_{n-q+1}, so every motif lies in B(x,d)
 *      for some l-mer x of one of those strings; enumerate those spheres and
 *      keep the candidates with a d-neighbour in at least q strings.
 *   Q0 (pattern-driven): every one of the 4^l l-mers, compared character by
 *      character with every l-mer of every string, kept when at least q
 *      strings have a d-neighbour.
 *
 * Pair-based candidates (Observation 3.3 with q = n): a motif M has an
 * l-mer x in s_1 and an l-mer y in s_2 within distance d of it, so
 * d_H(x,y) <= 2d and M lies in B(x,d) ∩ B(y,d). P1 takes every such pair,
 * walks T_d(x), keeps the candidates within d of y (the intersection) and
 * tests them against s_3..s_n; repeats (one motif, several pairs) dropped.
 *
 * Other alphabets (Sec. 1.2.5 defines the problem over any alphabet Sigma;
 * Table 3.1 gives n_B for any |Sigma|): S1 and S0 are O1 and O0 over an
 * alphabet of sigma letters given by the caller (letter code = its index
 * in the alphabet string), with codes in base sigma, first letter in the
 * top digit, and character-by-character distances.
 *
 * Long motifs (Sec. 3.3.1 stores an l-mer in ceil(l/32) words per group
 * when it does not fit one): W1 is O1 for 1 <= l <= 64, with 128-bit codes
 * (the same first-base-in-the-top-digit order) returned as a high and a low
 * 64-bit word per motif.
 *
 * O1 also counts the canonical number of Hamming tests, H_canon: for each
 * enumerated candidate (with multiplicity over references x), (m-l+1) times
 * the number of strings s_2..s_n examined, up to and including the first one
 * that has no d-neighbour.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

enum { OR_OK = 0, OR_EINVAL = -1, OR_EBASE = -2, OR_ENOMEM = -3 };

/* ---- encoding (Sec. 3.3.1 example: A=0, C=1, G=2, T=3) ---------------- */

static int base_code(unsigned char ch)
{
    switch (ch) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
    }
}

/* ASCII rows -> base codes. Returns the index of the first bad byte, or -1. */
static long long decode(const char *seqs, size_t total, unsigned char *out)
{
    for (size_t k = 0; k < total; k++) {
        int b = base_code((unsigned char)seqs[k]);
        if (b < 0)
            return (long long)k;
        out[k] = (unsigned char)b;
    }
    return -1;
}

int oracle_encode(const char *seqs, long long total, unsigned char *out,
                  long long *bad)
{
    long long k = decode(seqs, (size_t)total, out);
    if (bad)
        *bad = k;
    return k < 0 ? OR_OK : OR_EBASE;
}

/* l-mer starting at b[0..l-1] -> code with the first base in the top digit. */
static uint64_t lmer_code(const unsigned char *b, int l)
{
    uint64_t c = 0;
    for (int j = 0; j < l; j++)
        c = (c << 2) | b[j];
    return c;
}

uint64_t oracle_lmer_code(const char *lmer, int l)
{
    uint64_t c = 0;
    for (int j = 0; j < l; j++)
        c = (c << 2) | (uint64_t)base_code((unsigned char)lmer[j]);
    return c;
}

/* ---- distances ------------------------------------------------------- */

/* Definition 3: number of positions where the two l-mers differ. */
static int hamming_naive(const unsigned char *a, const unsigned char *b, int l)
{
    int h = 0;
    for (int j = 0; j < l; j++)
        h += (a[j] != b[j]);
    return h;
}

/* Same count on two packed codes: a digit differs iff either of its two
 * bits differs. */
static inline int hamming_packed(uint64_t a, uint64_t b)
{
    uint64_t v = a ^ b;
    return __builtin_popcountll((v | (v >> 1)) & 0x5555555555555555ULL);
}

/* Sec. 3.3.1: an l-mer becomes ceil(log2 |Sigma|) = 2 groups (bit planes);
 * group k holds bit k of each base code, bit j of the group for base j.
 * The distance is the number of set bits of the OR of the per-group XORs.
 * Restricted to l <= 32 (one 32-bit word per group). */
int oracle_groups(const char *lmer, int l, uint32_t *g1, uint32_t *g0)
{
    if (l < 1 || l > 32)
        return OR_EINVAL;
    uint32_t hi = 0, lo = 0;
    for (int j = 0; j < l; j++) {
        int b = base_code((unsigned char)lmer[j]);
        if (b < 0)
            return OR_EBASE;
        hi |= (uint32_t)((b >> 1) & 1) << j;
        lo |= (uint32_t)(b & 1) << j;
    }
    *g1 = hi;
    *g0 = lo;
    return OR_OK;
}

int oracle_hamming_groups(uint32_t a1, uint32_t a0, uint32_t b1, uint32_t b0)
{
    return __builtin_popcount((a1 ^ b1) | (a0 ^ b0));
}

int oracle_hamming_naive(const char *a, const char *b, int l)
{
    int h = 0;
    for (int j = 0; j < l; j++)
        h += (a[j] != b[j]);
    return h;
}

/* ---- size of the sphere B(a, R) (Table 3.1) ---------------------------- */

/* n_B(l, d) = sum_{k=0..d} C(l, k) (|Sigma| - 1)^k: choose k positions and
 * one of the |Sigma|-1 other letters at each. */
uint64_t oracle_nb(int l, int d, int sigma)
{
    uint64_t total = 0;
    for (int k = 0; k <= d && k <= l; k++) {
        uint64_t c = 1;
        for (int i = 0; i < k; i++)
            c = c * (uint64_t)(l - i) / (uint64_t)(i + 1);
        uint64_t p = 1;
        for (int i = 0; i < k; i++)
            p *= (uint64_t)(sigma - 1);
        total += c * p;
    }
    return total;
}

/* ---- growable output vector ------------------------------------------ */

typedef struct {
    uint64_t *v;
    size_t n, cap;
    int oom;
} vec64;

static void vpush(vec64 *a, uint64_t x)
{
    if (a->oom)
        return;
    if (a->n == a->cap) {
        size_t nc = a->cap ? 2 * a->cap : 1024;
        uint64_t *nv = (uint64_t *)realloc(a->v, nc * sizeof(uint64_t));
        if (!nv) {
            a->oom = 1;
            return;
        }
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Sort ascending and drop repeats: the result is a set (one correct byte
 * representation). */
static size_t sort_unique(uint64_t *v, size_t n)
{
    if (n == 0)
        return 0;
    qsort(v, n, sizeof(uint64_t), cmp_u64);
    size_t w = 1;
    for (size_t i = 1; i < n; i++)
        if (v[i] != v[w - 1])
            v[w++] = v[i];
    return w;
}

static int pick_threads(int want)
{
    if (want > 0)
        return want;
    long p = sysconf(_SC_NPROCESSORS_ONLN);
    return p > 0 ? (int)p : 1;
}

/* ---- O1: sample-driven ----------------------------------------------- */

typedef struct {
    /* shared, read-only */
    const uint64_t *codes; /* n rows of L packed l-mer codes */
    const unsigned char *bases; /* row 0 base codes (the references) */
    int n, L, l, d;
    int ref_begin, ref_end, nthreads, tid;
    uint64_t *per_ref; /* optional: H_canon per reference */
    /* per thread */
    vec64 out;
    uint64_t hcanon;
} o1_job;

/* Candidate test: strings s_2..s_n in input order, stop at the first one
 * without an l-mer within distance d. Returns 1 if the candidate is a motif;
 * *examined receives the number of strings looked at. */
static int o1_test(const o1_job *J, uint64_t cand, int *examined)
{
    int e = 0;
    for (int i = 1; i < J->n; i++) {
        const uint64_t *row = J->codes + (size_t)i * J->L;
        int hit = 0;
        e++;
        for (int j = 0; j < J->L; j++) {
            if (hamming_packed(cand, row[j]) <= J->d) {
                hit = 1;
                break;
            }
        }
        if (!hit) {
            *examined = e;
            return 0;
        }
    }
    *examined = e;
    return 1;
}

/* Walk T_d(x): the root is x; a node that last changed position p has
 * children that change one position p' > p to one of the 3 other letters,
 * so every string within distance d of x is visited exactly once. */
static void o1_ball(o1_job *J, const unsigned char *x, uint64_t cand,
                    int from, int budget, uint64_t *h)
{
    int examined;
    if (o1_test(J, cand, &examined))
        vpush(&J->out, cand);
    *h += (uint64_t)examined * (uint64_t)J->L;
    if (budget == 0)
        return;
    for (int p = from; p < J->l; p++) {
        int shift = 2 * (J->l - 1 - p);
        for (int b = 0; b < 4; b++) {
            if (b == x[p])
                continue;
            uint64_t c2 = cand ^ ((uint64_t)(x[p] ^ b) << shift);
            o1_ball(J, x, c2, p + 1, budget - 1, h);
        }
    }
}

static void *o1_worker(void *arg)
{
    o1_job *J = (o1_job *)arg;
    int span = J->ref_end - J->ref_begin;
    int lo = J->ref_begin + (int)((long long)span * J->tid / J->nthreads);
    int hi = J->ref_begin + (int)((long long)span * (J->tid + 1) / J->nthreads);
    for (int j = lo; j < hi; j++) {
        const unsigned char *x = J->bases + j;
        uint64_t h = 0;
        o1_ball(J, x, lmer_code(x, J->l), 0, J->d, &h);
        J->hcanon += h;
        if (J->per_ref)
            J->per_ref[j - J->ref_begin] = h;
    }
    return NULL;
}

static int check_args(int n, int m, int l, int d)
{
    if (n < 1 || l < 1 || l > 32 || m < l || d < 0 || d >= l)
        return OR_EINVAL;
    return OR_OK;
}

/*
 * O1 over the references x = s_1[j..j+l-1] for j in [ref_begin, ref_end)
 * (ref_end < 0 means all m-l+1 of them). With the full range the output is R;
 * a partial range gives the motifs found from those references only.
 * *out is malloc'ed (free with oracle_free); *hcanon gets H_canon of the
 * range; per_ref (may be NULL) gets H_canon per reference.
 */
int oracle_o1(const char *seqs, int n, int m, int l, int d, int ref_begin,
              int ref_end, int nthreads, uint64_t **out, size_t *count,
              uint64_t *hcanon, uint64_t *per_ref)
{
    int rc = check_args(n, m, l, d);
    if (rc)
        return rc;
    int L = m - l + 1;
    if (ref_end < 0 || ref_end > L)
        ref_end = L;
    if (ref_begin < 0 || ref_begin > ref_end)
        return OR_EINVAL;
    size_t total = (size_t)n * (size_t)m;
    unsigned char *bases = (unsigned char *)malloc(total);
    uint64_t *codes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n * L);
    if (!bases || !codes) {
        free(bases);
        free(codes);
        return OR_ENOMEM;
    }
    if (decode(seqs, total, bases) >= 0) {
        free(bases);
        free(codes);
        return OR_EBASE;
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < L; j++)
            codes[(size_t)i * L + j] = lmer_code(bases + (size_t)i * m + j, l);

    int T = pick_threads(nthreads);
    if (T > ref_end - ref_begin)
        T = ref_end - ref_begin > 0 ? ref_end - ref_begin : 1;
    o1_job *jobs = (o1_job *)calloc((size_t)T, sizeof(o1_job));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    if (!jobs || !th) {
        free(bases);
        free(codes);
        free(jobs);
        free(th);
        return OR_ENOMEM;
    }
    for (int t = 0; t < T; t++) {
        o1_job *J = &jobs[t];
        J->codes = codes;
        J->bases = bases;
        J->n = n;
        J->L = L;
        J->l = l;
        J->d = d;
        J->ref_begin = ref_begin;
        J->ref_end = ref_end;
        J->nthreads = T;
        J->tid = t;
        J->per_ref = per_ref;
    }
    for (int t = 1; t < T; t++)
        pthread_create(&th[t], NULL, o1_worker, &jobs[t]);
    o1_worker(&jobs[0]);
    for (int t = 1; t < T; t++)
        pthread_join(th[t], NULL);

    size_t tot = 0;
    int oom = 0;
    uint64_t h = 0;
    for (int t = 0; t < T; t++) {
        tot += jobs[t].out.n;
        oom |= jobs[t].out.oom;
        h += jobs[t].hcanon;
    }
    uint64_t *res = (uint64_t *)malloc(sizeof(uint64_t) * (tot ? tot : 1));
    if (!res || oom) {
        free(res);
        res = NULL;
        rc = OR_ENOMEM;
    } else {
        size_t w = 0;
        for (int t = 0; t < T; t++) {
            if (jobs[t].out.n)
                memcpy(res + w, jobs[t].out.v, jobs[t].out.n * sizeof(uint64_t));
            w += jobs[t].out.n;
        }
        *count = sort_unique(res, tot);
        *out = res;
        if (hcanon)
            *hcanon = h;
    }
    for (int t = 0; t < T; t++)
        free(jobs[t].out.v);
    free(jobs);
    free(th);
    free(bases);
    free(codes);
    return rc;
}

/* ---- O0: pattern-driven brute force ---------------------------------- */

typedef struct {
    const unsigned char *bases;
    int n, m, l, d, nthreads, tid;
    vec64 out;
} o0_job;

/* Definition 4 and 5 written out: M qualifies iff every string has an
 * l-mer within distance d, compared character by character. */
static int o0_is_motif(const unsigned char *bases, int n, int m, int l, int d,
                       const unsigned char *M)
{
    for (int i = 0; i < n; i++) {
        const unsigned char *s = bases + (size_t)i * m;
        int ok = 0;
        for (int j = 0; j + l <= m && !ok; j++)
            ok = hamming_naive(M, s + j, l) <= d;
        if (!ok)
            return 0;
    }
    return 1;
}

static void *o0_worker(void *arg)
{
    o0_job *J = (o0_job *)arg;
    uint64_t space = 1ULL << (2 * J->l);
    uint64_t lo = (uint64_t)((__uint128_t)space * J->tid / J->nthreads);
    uint64_t hi = (uint64_t)((__uint128_t)space * (J->tid + 1) / J->nthreads);
    unsigned char M[32];
    for (uint64_t c = lo; c < hi; c++) {
        for (int j = 0; j < J->l; j++)
            M[j] = (unsigned char)((c >> (2 * (J->l - 1 - j))) & 3);
        if (o0_is_motif(J->bases, J->n, J->m, J->l, J->d, M))
            vpush(&J->out, c);
    }
    return NULL;
}

int oracle_o0(const char *seqs, int n, int m, int l, int d, int nthreads,
              uint64_t **out, size_t *count)
{
    int rc = check_args(n, m, l, d);
    if (rc)
        return rc;
    if (l > 16)
        return OR_EINVAL; /* 4^l candidates: only for small l */
    size_t total = (size_t)n * (size_t)m;
    unsigned char *bases = (unsigned char *)malloc(total);
    if (!bases)
        return OR_ENOMEM;
    if (decode(seqs, total, bases) >= 0) {
        free(bases);
        return OR_EBASE;
    }
    int T = pick_threads(nthreads);
    o0_job *jobs = (o0_job *)calloc((size_t)T, sizeof(o0_job));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    if (!jobs || !th) {
        free(bases);
        free(jobs);
        free(th);
        return OR_ENOMEM;
    }
    for (int t = 0; t < T; t++) {
        jobs[t].bases = bases;
        jobs[t].n = n;
        jobs[t].m = m;
        jobs[t].l = l;
        jobs[t].d = d;
        jobs[t].nthreads = T;
        jobs[t].tid = t;
    }
    for (int t = 1; t < T; t++)
        pthread_create(&th[t], NULL, o0_worker, &jobs[t]);
    o0_worker(&jobs[0]);
    for (int t = 1; t < T; t++)
        pthread_join(th[t], NULL);
    /* each thread covers an ascending code range, so the concatenation in
     * thread order is already sorted and free of repeats */
    size_t tot = 0;
    int oom = 0;
    for (int t = 0; t < T; t++) {
        tot += jobs[t].out.n;
        oom |= jobs[t].out.oom;
    }
    uint64_t *res = (uint64_t *)malloc(sizeof(uint64_t) * (tot ? tot : 1));
    if (!res || oom) {
        free(res);
        rc = OR_ENOMEM;
    } else {
        size_t w = 0;
        for (int t = 0; t < T; t++) {
            if (jobs[t].out.n)
                memcpy(res + w, jobs[t].out.v, jobs[t].out.n * sizeof(uint64_t));
            w += jobs[t].out.n;
        }
        *out = res;
        *count = tot;
    }
    for (int t = 0; t < T; t++)
        free(jobs[t].out.v);
    free(jobs);
    free(th);
    free(bases);
    return rc;
}

/* Direct check of one code against every string (Definitions 4-5), for
 * spot checks of outputs too large to recompute whole. 1 = motif, 0 = not,
 * negative = error. */
int oracle_is_motif(const char *seqs, int n, int m, int l, int d,
                    uint64_t code)
{
    int rc = check_args(n, m, l, d);
    if (rc)
        return rc;
    if (l < 32 && (code >> (2 * l)) != 0)
        return OR_EINVAL;
    unsigned char M[32];
    for (int j = 0; j < l; j++)
        M[j] = (unsigned char)((code >> (2 * (l - 1 - j))) & 3);
    for (int i = 0; i < n; i++) {
        const char *s = seqs + (size_t)i * m;
        int ok = 0;
        for (int j = 0; j + l <= m && !ok; j++) {
            int h = 0;
            for (int k = 0; k < l; k++) {
                int b = base_code((unsigned char)s[j + k]);
                if (b < 0)
                    return OR_EBASE;
                h += (b != M[k]);
            }
            ok = h <= d;
        }
        if (!ok)
            return 0;
    }
    return 1;
}

/* ---- quorum: (l,d,q)-motifs ------------------------------------------- */

static int check_q(int n, int m, int l, int d, int q)
{
    int rc = check_args(n, m, l, d);
    if (rc)
        return rc;
    return (q < 1 || q > n) ? OR_EINVAL : OR_OK;
}

/* Number of strings with an l-mer within distance d of the packed code,
 * counted until the answer is settled: returns q as soon as q strings have
 * one, and stops early when too few strings are left to reach q. */
static int q_hits(const uint64_t *codes, int n, int L, int d, int q,
                  uint64_t cand)
{
    int hits = 0;
    for (int i = 0; i < n; i++) {
        if (hits + (n - i) < q)
            break;
        const uint64_t *row = codes + (size_t)i * L;
        for (int j = 0; j < L; j++)
            if (hamming_packed(cand, row[j]) <= d) {
                hits++;
                break;
            }
        if (hits >= q)
            break;
    }
    return hits;
}

typedef struct {
    const uint64_t *codes;
    const unsigned char *bases;
    int n, m, L, l, d, q, nthreads, tid;
    vec64 out;
} q1_job;

/* T_d(x) as in O1: every element of B(x,d) once. */
static void q1_ball(q1_job *J, const unsigned char *x, uint64_t cand,
                    int from, int budget)
{
    if (q_hits(J->codes, J->n, J->L, J->d, J->q, cand) >= J->q)
        vpush(&J->out, cand);
    if (budget == 0)
        return;
    for (int p = from; p < J->l; p++) {
        int shift = 2 * (J->l - 1 - p);
        for (int b = 0; b < 4; b++) {
            if (b == x[p])
                continue;
            q1_ball(J, x, cand ^ ((uint64_t)(x[p] ^ b) << shift), p + 1,
                    budget - 1);
        }
    }
}

static void *q1_worker(void *arg)
{
    q1_job *J = (q1_job *)arg;
    /* references: every l-mer of s_1..s_{n-q+1}, split evenly */
    long long nref = (long long)(J->n - J->q + 1) * J->L;
    long long lo = nref * J->tid / J->nthreads;
    long long hi = nref * (J->tid + 1) / J->nthreads;
    for (long long r = lo; r < hi; r++) {
        int i = (int)(r / J->L), j = (int)(r % J->L);
        const unsigned char *x = J->bases + (size_t)i * J->m + j;
        q1_ball(J, x, lmer_code(x, J->l), 0, J->d);
    }
    return NULL;
}

/* Concatenate the per-thread vectors; sort and drop repeats if asked. */
static int gather_out(vec64 *v, int T, int dedup, uint64_t **out,
                      size_t *count)
{
    size_t tot = 0;
    int oom = 0;
    for (int t = 0; t < T; t++) {
        tot += v[t].n;
        oom |= v[t].oom;
    }
    uint64_t *res = (uint64_t *)malloc(sizeof(uint64_t) * (tot ? tot : 1));
    if (!res || oom) {
        free(res);
        return OR_ENOMEM;
    }
    size_t w = 0;
    for (int t = 0; t < T; t++) {
        if (v[t].n)
            memcpy(res + w, v[t].v, v[t].n * sizeof(uint64_t));
        w += v[t].n;
    }
    *count = dedup ? sort_unique(res, tot) : tot;
    *out = res;
    return OR_OK;
}

/* Q1: the (l,d,q)-motifs by Observation 3.1 (see the file header). */
int oracle_q1(const char *seqs, int n, int m, int l, int d, int q,
              int nthreads, uint64_t **out, size_t *count)
{
    int rc = check_q(n, m, l, d, q);
    if (rc)
        return rc;
    int L = m - l + 1;
    size_t total = (size_t)n * (size_t)m;
    unsigned char *bases = (unsigned char *)malloc(total);
    uint64_t *codes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n * L);
    int T = pick_threads(nthreads);
    q1_job *jobs = (q1_job *)calloc((size_t)T, sizeof(q1_job));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    vec64 *vs = (vec64 *)calloc((size_t)T, sizeof(vec64));
    if (!bases || !codes || !jobs || !th || !vs) {
        rc = OR_ENOMEM;
        goto done;
    }
    if (decode(seqs, total, bases) >= 0) {
        rc = OR_EBASE;
        goto done;
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < L; j++)
            codes[(size_t)i * L + j] = lmer_code(bases + (size_t)i * m + j, l);
    for (int t = 0; t < T; t++) {
        q1_job *J = &jobs[t];
        J->codes = codes;
        J->bases = bases;
        J->n = n;
        J->m = m;
        J->L = L;
        J->l = l;
        J->d = d;
        J->q = q;
        J->nthreads = T;
        J->tid = t;
    }
    for (int t = 1; t < T; t++)
        pthread_create(&th[t], NULL, q1_worker, &jobs[t]);
    q1_worker(&jobs[0]);
    for (int t = 1; t < T; t++)
        pthread_join(th[t], NULL);
    for (int t = 0; t < T; t++)
        vs[t] = jobs[t].out;
    rc = gather_out(vs, T, 1, out, count);
done:
    if (jobs)
        for (int t = 0; t < T; t++)
            free(jobs[t].out.v);
    free(vs);
    free(jobs);
    free(th);
    free(bases);
    free(codes);
    return rc;
}

typedef struct {
    const unsigned char *bases;
    int n, m, l, d, q, nthreads, tid;
    vec64 out;
} q0_job;

static void *q0_worker(void *arg)
{
    q0_job *J = (q0_job *)arg;
    uint64_t space = 1ULL << (2 * J->l);
    uint64_t lo = (uint64_t)((__uint128_t)space * J->tid / J->nthreads);
    uint64_t hi = (uint64_t)((__uint128_t)space * (J->tid + 1) / J->nthreads);
    unsigned char M[32];
    for (uint64_t c = lo; c < hi; c++) {
        for (int j = 0; j < J->l; j++)
            M[j] = (unsigned char)((c >> (2 * (J->l - 1 - j))) & 3);
        /* Definitions 4 and 5: count the strings with an l-mer within d */
        int hits = 0;
        for (int i = 0; i < J->n; i++) {
            const unsigned char *s = J->bases + (size_t)i * J->m;
            int ok = 0;
            for (int j = 0; j + J->l <= J->m && !ok; j++)
                ok = hamming_naive(M, s + j, J->l) <= J->d;
            hits += ok;
        }
        if (hits >= J->q)
            vpush(&J->out, c);
    }
    return NULL;
}

/* Q0: brute force over all 4^l codes (small l only). */
int oracle_q0(const char *seqs, int n, int m, int l, int d, int q,
              int nthreads, uint64_t **out, size_t *count)
{
    int rc = check_q(n, m, l, d, q);
    if (rc)
        return rc;
    if (l > 16)
        return OR_EINVAL;
    size_t total = (size_t)n * (size_t)m;
    unsigned char *bases = (unsigned char *)malloc(total);
    int T = pick_threads(nthreads);
    q0_job *jobs = (q0_job *)calloc((size_t)T, sizeof(q0_job));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    vec64 *vs = (vec64 *)calloc((size_t)T, sizeof(vec64));
    if (!bases || !jobs || !th || !vs) {
        rc = OR_ENOMEM;
        goto done;
    }
    if (decode(seqs, total, bases) >= 0) {
        rc = OR_EBASE;
        goto done;
    }
    for (int t = 0; t < T; t++) {
        jobs[t].bases = bases;
        jobs[t].n = n;
        jobs[t].m = m;
        jobs[t].l = l;
        jobs[t].d = d;
        jobs[t].q = q;
        jobs[t].nthreads = T;
        jobs[t].tid = t;
    }
    for (int t = 1; t < T; t++)
        pthread_create(&th[t], NULL, q0_worker, &jobs[t]);
    q0_worker(&jobs[0]);
    for (int t = 1; t < T; t++)
        pthread_join(th[t], NULL);
    for (int t = 0; t < T; t++)
        vs[t] = jobs[t].out;
    /* ascending code ranges per thread: already sorted, no repeats */
    rc = gather_out(vs, T, 0, out, count);
done:
    if (jobs)
        for (int t = 0; t < T; t++)
            free(jobs[t].out.v);
    free(vs);
    free(jobs);
    free(th);
    free(bases);
    return rc;
}

/* Number of strings that have an l-mer within distance d of the code
 * (Definitions 4-5, character by character): spot checks of quorum
 * outputs too large to recompute whole. Negative = error. */
int oracle_hit_count(const char *seqs, int n, int m, int l, int d,
                     uint64_t code)
{
    int rc = check_args(n, m, l, d);
    if (rc)
        return rc;
    if (l < 32 && (code >> (2 * l)) != 0)
        return OR_EINVAL;
    unsigned char M[32];
    for (int j = 0; j < l; j++)
        M[j] = (unsigned char)((code >> (2 * (l - 1 - j))) & 3);
    int hits = 0;
    for (int i = 0; i < n; i++) {
        const char *s = seqs + (size_t)i * m;
        int ok = 0;
        for (int j = 0; j + l <= m && !ok; j++) {
            int h = 0;
            for (int k = 0; k < l; k++) {
                int b = base_code((unsigned char)s[j + k]);
                if (b < 0)
                    return OR_EBASE;
                h += (b != M[k]);
            }
            ok = h <= d;
        }
        hits += ok;
    }
    return hits;
}

/* ---- P1: pair-based candidates (Observation 3.3) ---------------------- */

typedef struct {
    const uint64_t *codes;   /* n rows of L packed codes */
    const unsigned char *bases;
    int n, L, l, d, nthreads, tid;
    vec64 out;
    uint64_t ncand;          /* candidates: sum of |B(x,d) ∩ B(y,d)| */
} p1_job;

/* strings s_3..s_n in order, stop at the first without a d-neighbour */
static int p1_test(const p1_job *J, uint64_t cand)
{
    for (int i = 2; i < J->n; i++) {
        const uint64_t *row = J->codes + (size_t)i * J->L;
        int hit = 0;
        for (int j = 0; j < J->L && !hit; j++)
            hit = hamming_packed(cand, row[j]) <= J->d;
        if (!hit)
            return 0;
    }
    return 1;
}

/* T_d(x), keeping the nodes within distance d of y */
static void p1_ball(p1_job *J, const unsigned char *x, uint64_t y,
                    uint64_t cand, int from, int budget)
{
    if (hamming_packed(cand, y) <= J->d) {
        J->ncand++;
        if (p1_test(J, cand))
            vpush(&J->out, cand);
    }
    if (budget == 0)
        return;
    for (int p = from; p < J->l; p++) {
        int shift = 2 * (J->l - 1 - p);
        for (int b = 0; b < 4; b++) {
            if (b == x[p])
                continue;
            p1_ball(J, x, y, cand ^ ((uint64_t)(x[p] ^ b) << shift), p + 1,
                    budget - 1);
        }
    }
}

static void *p1_worker(void *arg)
{
    p1_job *J = (p1_job *)arg;
    int lo = (int)((long long)J->L * J->tid / J->nthreads);
    int hi = (int)((long long)J->L * (J->tid + 1) / J->nthreads);
    const uint64_t *row2 = J->codes + J->L;   /* s_2 */
    for (int j = lo; j < hi; j++) {
        const unsigned char *x = J->bases + j;
        const uint64_t xc = J->codes[j];
        for (int k = 0; k < J->L; k++)
            if (hamming_packed(xc, row2[k]) <= 2 * J->d)
                p1_ball(J, x, row2[k], xc, 0, J->d);
    }
    return NULL;
}

/* P1: the (l,d)-motifs from pair intersections (needs n >= 2). *ncand gets
 * the number of candidates, sum over pairs of |B(x,d) ∩ B(y,d)|. */
int oracle_p1(const char *seqs, int n, int m, int l, int d, int nthreads,
              uint64_t **out, size_t *count, uint64_t *ncand)
{
    int rc = check_args(n, m, l, d);
    if (rc)
        return rc;
    if (n < 2)
        return OR_EINVAL;
    int L = m - l + 1;
    size_t total = (size_t)n * (size_t)m;
    unsigned char *bases = (unsigned char *)malloc(total);
    uint64_t *codes = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n * L);
    int T = pick_threads(nthreads);
    if (T > L)
        T = L;
    p1_job *jobs = (p1_job *)calloc((size_t)T, sizeof(p1_job));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    vec64 *vs = (vec64 *)calloc((size_t)T, sizeof(vec64));
    if (!bases || !codes || !jobs || !th || !vs) {
        rc = OR_ENOMEM;
        goto done;
    }
    if (decode(seqs, total, bases) >= 0) {
        rc = OR_EBASE;
        goto done;
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < L; j++)
            codes[(size_t)i * L + j] = lmer_code(bases + (size_t)i * m + j, l);
    for (int t = 0; t < T; t++) {
        p1_job *J = &jobs[t];
        J->codes = codes;
        J->bases = bases;
        J->n = n;
        J->L = L;
        J->l = l;
        J->d = d;
        J->nthreads = T;
        J->tid = t;
    }
    for (int t = 1; t < T; t++)
        pthread_create(&th[t], NULL, p1_worker, &jobs[t]);
    p1_worker(&jobs[0]);
    for (int t = 1; t < T; t++)
        pthread_join(th[t], NULL);
    uint64_t nc = 0;
    for (int t = 0; t < T; t++) {
        vs[t] = jobs[t].out;
        nc += jobs[t].ncand;
    }
    rc = gather_out(vs, T, 1, out, count);
    if (!rc && ncand)
        *ncand = nc;
done:
    if (jobs)
        for (int t = 0; t < T; t++)
            free(jobs[t].out.v);
    free(vs);
    free(jobs);
    free(th);
    free(bases);
    free(codes);
    return rc;
}

/* ---- any alphabet: S1 (sample-driven) and S0 (brute force) ------------- */

typedef struct {
    signed char map[256];   /* byte -> letter code, -1 if not in alphabet */
    int sigma;
} alpha_t;

static int alpha_setup(alpha_t *A, const char *alphabet, int sigma)
{
    if (!alphabet || sigma < 2 || sigma > 32)
        return OR_EINVAL;
    memset(A->map, -1, sizeof(A->map));
    for (int i = 0; i < sigma; i++) {
        unsigned char ch = (unsigned char)alphabet[i];
        if (A->map[ch] >= 0)
            return OR_EINVAL; /* repeated letter */
        A->map[ch] = (signed char)i;
    }
    A->sigma = sigma;
    return OR_OK;
}

/* sigma^l must fit in 64 bits: codes are base-sigma integers */
static int alpha_space(int sigma, int l, uint64_t *space)
{
    __uint128_t v = 1;
    for (int j = 0; j < l; j++) {
        v *= (unsigned)sigma;
        if (v > ((__uint128_t)1 << 64))
            return OR_EINVAL;
    }
    *space = (v == ((__uint128_t)1 << 64)) ? 0 : (uint64_t)v;
    return OR_OK;
}

/* Definition 3 with an early stop: 1 if the two l-mers differ in at most
 * d positions. */
static int within_d(const unsigned char *a, const unsigned char *b, int l,
                    int d)
{
    int h = 0;
    for (int k = 0; k < l; k++)
        if (a[k] != b[k] && ++h > d)
            return 0;
    return 1;
}

typedef struct {
    const unsigned char *letters; /* n*m letter codes */
    int n, m, l, d, sigma, nthreads, tid;
    vec64 out;
} s1_job;

static uint64_t code_sigma(const unsigned char *M, int l, int sigma)
{
    uint64_t c = 0;
    for (int j = 0; j < l; j++)
        c = c * (uint64_t)sigma + M[j];
    return c;
}

/* A candidate is kept when every string s_2..s_n has an l-mer within d. */
static int s1_test(const s1_job *J, const unsigned char *M)
{
    for (int i = 1; i < J->n; i++) {
        const unsigned char *s = J->letters + (size_t)i * J->m;
        int hit = 0;
        for (int j = 0; j + J->l <= J->m && !hit; j++)
            hit = within_d(M, s + j, J->l, J->d);
        if (!hit)
            return 0;
    }
    return 1;
}

/* T_d(x) over sigma letters: a node that last changed position p has
 * children changing one position p' > p to one of the sigma-1 others. */
static void s1_ball(s1_job *J, unsigned char *M, const unsigned char *x,
                    int from, int budget)
{
    if (s1_test(J, M))
        vpush(&J->out, code_sigma(M, J->l, J->sigma));
    if (budget == 0)
        return;
    for (int p = from; p < J->l; p++) {
        for (int b = 0; b < J->sigma; b++) {
            if (b == x[p])
                continue;
            M[p] = (unsigned char)b;
            s1_ball(J, M, x, p + 1, budget - 1);
        }
        M[p] = x[p];
    }
}

static void *s1_worker(void *arg)
{
    s1_job *J = (s1_job *)arg;
    int L = J->m - J->l + 1;
    int lo = (int)((long long)L * J->tid / J->nthreads);
    int hi = (int)((long long)L * (J->tid + 1) / J->nthreads);
    unsigned char M[32];
    for (int j = lo; j < hi; j++) {
        const unsigned char *x = J->letters + j;
        memcpy(M, x, (size_t)J->l);
        s1_ball(J, M, x, 0, J->d);
    }
    return NULL;
}

static int alpha_decode(const alpha_t *A, const char *seqs, size_t total,
                        unsigned char *out)
{
    for (size_t k = 0; k < total; k++) {
        int c = A->map[(unsigned char)seqs[k]];
        if (c < 0)
            return OR_EBASE;
        out[k] = (unsigned char)c;
    }
    return OR_OK;
}

/* S1: the (l,d)-motifs over the given alphabet, sample-driven (every motif
 * lies in B(x,d) for an l-mer x of s_1). */
int oracle_s1(const char *seqs, const char *alphabet, int sigma, int n,
              int m, int l, int d, int nthreads, uint64_t **out,
              size_t *count)
{
    alpha_t A;
    uint64_t space;
    int rc = check_args(n, m, l, d);
    if (!rc)
        rc = alpha_setup(&A, alphabet, sigma);
    if (!rc)
        rc = alpha_space(sigma, l, &space);
    if (rc)
        return rc;
    size_t total = (size_t)n * (size_t)m;
    unsigned char *letters = (unsigned char *)malloc(total);
    int T = pick_threads(nthreads);
    int L = m - l + 1;
    if (T > L)
        T = L;
    s1_job *jobs = (s1_job *)calloc((size_t)T, sizeof(s1_job));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    vec64 *vs = (vec64 *)calloc((size_t)T, sizeof(vec64));
    if (!letters || !jobs || !th || !vs) {
        rc = OR_ENOMEM;
        goto done;
    }
    if ((rc = alpha_decode(&A, seqs, total, letters)))
        goto done;
    for (int t = 0; t < T; t++) {
        s1_job *J = &jobs[t];
        J->letters = letters;
        J->n = n;
        J->m = m;
        J->l = l;
        J->d = d;
        J->sigma = sigma;
        J->nthreads = T;
        J->tid = t;
    }
    for (int t = 1; t < T; t++)
        pthread_create(&th[t], NULL, s1_worker, &jobs[t]);
    s1_worker(&jobs[0]);
    for (int t = 1; t < T; t++)
        pthread_join(th[t], NULL);
    for (int t = 0; t < T; t++)
        vs[t] = jobs[t].out;
    rc = gather_out(vs, T, 1, out, count);
done:
    if (jobs)
        for (int t = 0; t < T; t++)
            free(jobs[t].out.v);
    free(vs);
    free(jobs);
    free(th);
    free(letters);
    return rc;
}

/* S0: every code of the sigma^l space (small spaces only), kept when every
 * string has an l-mer within distance d. */
int oracle_s0(const char *seqs, const char *alphabet, int sigma, int n,
              int m, int l, int d, uint64_t **out, size_t *count)
{
    alpha_t A;
    uint64_t space;
    int rc = check_args(n, m, l, d);
    if (!rc)
        rc = alpha_setup(&A, alphabet, sigma);
    if (!rc)
        rc = alpha_space(sigma, l, &space);
    if (rc)
        return rc;
    if (space == 0 || space > (1ULL << 26))
        return OR_EINVAL;
    size_t total = (size_t)n * (size_t)m;
    unsigned char *letters = (unsigned char *)malloc(total);
    vec64 v = {0};
    if (!letters)
        return OR_ENOMEM;
    if ((rc = alpha_decode(&A, seqs, total, letters))) {
        free(letters);
        return rc;
    }
    unsigned char M[32];
    for (uint64_t c = 0; c < space; c++) {
        uint64_t r = c;
        for (int j = l - 1; j >= 0; j--) {
            M[j] = (unsigned char)(r % (uint64_t)sigma);
            r /= (uint64_t)sigma;
        }
        int ok = 1;
        for (int i = 0; i < n && ok; i++) {
            const unsigned char *s = letters + (size_t)i * m;
            int hit = 0;
            for (int j = 0; j + l <= m && !hit; j++)
                hit = within_d(M, s + j, l, d);
            ok = hit;
        }
        if (ok)
            vpush(&v, c);
    }
    free(letters);
    rc = gather_out(&v, 1, 0, out, count);
    free(v.v);
    return rc;
}

/* ---- W1: sample-driven over 128-bit codes (1 <= l <= 64) -------------- */

typedef unsigned __int128 u128;

/* A growable vector of 128-bit codes. */
typedef struct {
    u128 *v;
    size_t n, cap;
    int oom;
} vec128;

static void wpush(vec128 *a, u128 x)
{
    if (a->oom)
        return;
    if (a->n == a->cap) {
        size_t nc = a->cap ? 2 * a->cap : 256;
        u128 *nv = (u128 *)realloc(a->v, nc * sizeof(u128));
        if (!nv) {
            a->oom = 1;
            return;
        }
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
}

static int cmp_u128(const void *a, const void *b)
{
    u128 x = *(const u128 *)a, y = *(const u128 *)b;
    return (x > y) - (x < y);
}

/* l-mer b[0..l-1] -> 128-bit code, first base in the top digit. */
static u128 lmer_code128(const unsigned char *b, int l)
{
    u128 c = 0;
    for (int j = 0; j < l; j++)
        c = (c << 2) | b[j];
    return c;
}

/* Digits that differ between two packed codes, counted on both halves. */
static inline int hamming_packed128(u128 a, u128 b)
{
    const uint64_t m = 0x5555555555555555ULL;
    u128 v = a ^ b;
    v = v | (v >> 1);
    return __builtin_popcountll((uint64_t)v & m) +
           __builtin_popcountll((uint64_t)(v >> 64) & m);
}

typedef struct {
    const u128 *codes;          /* n rows of L codes */
    const unsigned char *bases; /* row 0 base codes */
    int n, L, l, d, nthreads, tid;
    vec128 out;
    uint64_t hcanon;
} w1_job;

/* As o1_test: s_2..s_n in input order, stop at the first string with no
 * l-mer within distance d. */
static int w1_test(const w1_job *J, u128 cand, int *examined)
{
    int e = 0;
    for (int i = 1; i < J->n; i++) {
        const u128 *row = J->codes + (size_t)i * J->L;
        int hit = 0;
        e++;
        for (int j = 0; j < J->L && !hit; j++)
            hit = hamming_packed128(cand, row[j]) <= J->d;
        if (!hit) {
            *examined = e;
            return 0;
        }
    }
    *examined = e;
    return 1;
}

/* T_d(x) as in o1_ball, on 128-bit codes. */
static void w1_ball(w1_job *J, const unsigned char *x, u128 cand, int from,
                    int budget, uint64_t *h)
{
    int examined;
    if (w1_test(J, cand, &examined))
        wpush(&J->out, cand);
    *h += (uint64_t)examined * (uint64_t)J->L;
    if (budget == 0)
        return;
    for (int p = from; p < J->l; p++) {
        int shift = 2 * (J->l - 1 - p);
        for (int b = 0; b < 4; b++) {
            if (b == x[p])
                continue;
            w1_ball(J, x, cand ^ ((u128)(x[p] ^ b) << shift), p + 1,
                    budget - 1, h);
        }
    }
}

static void *w1_worker(void *arg)
{
    w1_job *J = (w1_job *)arg;
    int lo = (int)((long long)J->L * J->tid / J->nthreads);
    int hi = (int)((long long)J->L * (J->tid + 1) / J->nthreads);
    for (int j = lo; j < hi; j++) {
        const unsigned char *x = J->bases + j;
        uint64_t h = 0;
        w1_ball(J, x, lmer_code128(x, J->l), 0, J->d, &h);
        J->hcanon += h;
    }
    return NULL;
}

static int check_args_wide(int n, int m, int l, int d)
{
    if (n < 1 || l < 1 || l > 64 || m < l || d < 0 || d >= l)
        return OR_EINVAL;
    return OR_OK;
}

/*
 * W1: R for 1 <= l <= 64. *out (free with oracle_free) receives 2*count
 * words, motif i as out[2i] = bits 127..64 and out[2i+1] = bits 63..0 of its
 * code, ascending, no repeats; *hcanon gets H_canon.
 */
int oracle_o1_wide(const char *seqs, int n, int m, int l, int d, int nthreads,
                   uint64_t **out, size_t *count, uint64_t *hcanon)
{
    int rc = check_args_wide(n, m, l, d);
    if (rc)
        return rc;
    int L = m - l + 1;
    size_t total = (size_t)n * (size_t)m;
    unsigned char *bases = (unsigned char *)malloc(total);
    u128 *codes = (u128 *)malloc(sizeof(u128) * (size_t)n * L);
    if (!bases || !codes) {
        free(bases);
        free(codes);
        return OR_ENOMEM;
    }
    if (decode(seqs, total, bases) >= 0) {
        free(bases);
        free(codes);
        return OR_EBASE;
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < L; j++)
            codes[(size_t)i * L + j] =
                lmer_code128(bases + (size_t)i * m + j, l);
    int T = pick_threads(nthreads);
    if (T > L)
        T = L;
    w1_job *jobs = (w1_job *)calloc((size_t)T, sizeof(w1_job));
    pthread_t *th = (pthread_t *)calloc((size_t)T, sizeof(pthread_t));
    if (!jobs || !th) {
        free(bases);
        free(codes);
        free(jobs);
        free(th);
        return OR_ENOMEM;
    }
    for (int t = 0; t < T; t++) {
        w1_job *J = &jobs[t];
        J->codes = codes;
        J->bases = bases;
        J->n = n;
        J->L = L;
        J->l = l;
        J->d = d;
        J->nthreads = T;
        J->tid = t;
    }
    for (int t = 1; t < T; t++)
        pthread_create(&th[t], NULL, w1_worker, &jobs[t]);
    w1_worker(&jobs[0]);
    for (int t = 1; t < T; t++)
        pthread_join(th[t], NULL);
    size_t tot = 0;
    int oom = 0;
    uint64_t h = 0;
    for (int t = 0; t < T; t++) {
        tot += jobs[t].out.n;
        oom |= jobs[t].out.oom;
        h += jobs[t].hcanon;
    }
    u128 *all = (u128 *)malloc(sizeof(u128) * (tot ? tot : 1));
    uint64_t *res = (uint64_t *)malloc(2 * sizeof(uint64_t) * (tot ? tot : 1));
    if (!all || !res || oom) {
        free(res);
        rc = OR_ENOMEM;
    } else {
        size_t w = 0;
        for (int t = 0; t < T; t++) {
            if (jobs[t].out.n)
                memcpy(all + w, jobs[t].out.v, jobs[t].out.n * sizeof(u128));
            w += jobs[t].out.n;
        }
        /* a set: ascending, repeats dropped */
        if (tot)
            qsort(all, tot, sizeof(u128), cmp_u128);
        size_t u = 0;
        for (size_t i = 0; i < tot; i++)
            if (u == 0 || all[i] != all[u - 1])
                all[u++] = all[i];
        for (size_t i = 0; i < u; i++) {
            res[2 * i] = (uint64_t)(all[i] >> 64);
            res[2 * i + 1] = (uint64_t)all[i];
        }
        *out = res;
        *count = u;
        if (hcanon)
            *hcanon = h;
    }
    free(all);
    for (int t = 0; t < T; t++)
        free(jobs[t].out.v);
    free(jobs);
    free(th);
    free(bases);
    free(codes);
    return rc;
}

/* Definitions 4-5 for one 128-bit code (hi: bits 127..64, lo: bits 63..0),
 * compared character by character: 1 = motif, 0 = not, negative = error. */
int oracle_is_motif_wide(const char *seqs, int n, int m, int l, int d,
                         uint64_t hi, uint64_t lo)
{
    int rc = check_args_wide(n, m, l, d);
    if (rc)
        return rc;
    u128 code = ((u128)hi << 64) | lo;
    if (l < 64 && (code >> (2 * l)) != 0)
        return OR_EINVAL;
    unsigned char M[64];
    for (int j = 0; j < l; j++)
        M[j] = (unsigned char)((code >> (2 * (l - 1 - j))) & 3);
    for (int i = 0; i < n; i++) {
        const char *s = seqs + (size_t)i * m;
        int ok = 0;
        for (int j = 0; j + l <= m && !ok; j++) {
            int h = 0;
            for (int k = 0; k < l; k++) {
                int b = base_code((unsigned char)s[j + k]);
                if (b < 0)
                    return OR_EBASE;
                h += (b != M[k]);
            }
            ok = h <= d;
        }
        if (!ok)
            return 0;
    }
    return 1;
}

void oracle_free(void *p)
{
    free(p);
}
