/*
 * pms.h -- C ABI of libpms: exact planted (l,d)-motif search on one MI355X.
 *
 * The operation (Definitions 1-5 of Sec. 1.2.5 and the qPMS definition with
 * q = n, i.e. plain PMS): given n strings s_1..s_n of length m over
 * {A,C,G,T}, return every l-mer M such that each s_i contains an l-mer y
 * (any of its m-l+1 substrings of length l) with Hamming distance
 * d_H(M, y) <= d (Definition 3: the number of mismatching positions).
 *
 * Result encoding. A motif M[0..l-1] is returned as the uint64
 *     code(M) = sum_j b(M[j]) * 4^(l-1-j),  b(A)=0, b(C)=1, b(G)=2, b(T)=3
 * (the base coding of the compression example in Sec. 3.3.1; first base in
 * the most significant digit, so numeric order is lexicographic order).
 * Results are ascending and free of repeats: the result is a set.
 *
 * Domain. 1 <= n; 1 <= l <= 32; l <= m; 0 <= d < l. Input bytes must be
 * uppercase 'A','C','G','T'; anything else is PMS_EBASE, and
 * pms_last_error() names the string and offset of the first bad byte.
 *
 * Variants. pms_solve_quorum returns the (l,d,q)-motifs for any quorum
 * 1 <= q <= n (Definition 5); pms_solve_alphabet solves the same problem
 * over another alphabet of 2..32 letters (codes in base sigma, see there);
 * PMS_PATH_PAIR (an option of the context) computes the plain set from
 * pairs of l-mers of s_1 and s_2 (Observation 3.3); pms_solve_wide takes
 * motifs up to l = 64 (128-bit codes, see there).
 *
 * Ownership. Inputs are copied before a call returns (pms_submit included),
 * so the caller may free them at once. Result arrays belong to the context
 * and stay valid until the next call on that context that returns results
 * (pms_solve*, pms_solve_batch) or until pms_release / pms_destroy.
 *
 * Threads. A context is not thread-safe: use one per host thread. The
 * serving entry points (pms_submit / pms_poll / pms_release) may be called
 * while the context's own engine thread runs requests on the device.
 *
 * Errors. Every int-returning call returns PMS_OK (0), PMS_PENDING (1,
 * pms_poll only) or a negative PMS_E* status; pms_last_error() gives a
 * human-readable detail of the last failure on that context.
 */
#ifndef PMS_H
#define PMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PMS_OK = 0,
    PMS_PENDING = 1,      /* pms_poll: request admitted or queued, not done */
    PMS_EINVAL = -1,      /* bad sizes, parameters, ticket or NULL pointer */
    PMS_EBASE = -2,       /* an input byte is not one of A, C, G, T */
    PMS_ENOMEM = -3,      /* device memory budget or capacity too small */
    PMS_EDEVICE = -4,     /* HIP runtime error */
    PMS_EBUSY = -5        /* serving queue full */
};

/* Which device algorithm computes the set. All give identical results. */
enum {
    PMS_PATH_AUTO = 0,    /* cost model picks the cheapest of 1 and 3 */
    PMS_PATH_FILTER = 1,  /* sample-driven: d-neighbourhoods of the l-mers of
                             s_1 (Observation 3.1 with q = n) filtered by
                             XOR/popcount Hamming tests against s_2..s_n */
    PMS_PATH_BITSET = 2,  /* pattern-driven, memory-heavy: one bit per l-mer
                             of the 4^l space resident in device memory,
                             one pass per string ANDs in the union of the
                             d-spheres of its l-mers, each 4^9-code tile
                             taking the strings in its own order (needs
                             4^l/8 bytes, plus about 9 + 5n bytes per
                             tile for its order and liveness) */
    PMS_PATH_TILED = 3,   /* pattern-driven, tiled: the 4^l space split into
                             tiles held on chip; each tile ANDs the strings'
                             sphere unions until few codes are left, then
                             filters those by Hamming tests */
    PMS_PATH_PAIR = 4     /* sample-driven from pairs (Observation 3.3):
                             candidates from B(x,d) ∩ B(y,d) for x in s_1,
                             y in s_2 with d_H(x,y) <= 2d, filtered against
                             s_3..s_n; never chosen by AUTO; needs n >= 2
                             and 2d <= 20 */
};

typedef struct pms_ctx pms_ctx;

typedef struct {
    int device;               /* HIP device ordinal */
    int path;                 /* PMS_PATH_*; 0 = auto */
    size_t mem_budget_bytes;  /* device memory the context may hold for
                                 per-call buffers; 0 = 90% of free memory */
    const char *tune_cache;   /* autotuner cache file (read at create,
                                 written after tuning); NULL = in memory */
    int serve_slots;          /* serving: max requests on the device at
                                 once; 0 = 64 */
    int serve_queue;          /* serving: max requests waiting for
                                 admission; 0 = 4096 */
    int tile_threads;         /* tiled path: workgroup size of the tile
                                 kernel, 256 or 512; 0 = automatic (512
                                 where the tiles hold 4^8 or 4^9 codes).
                                 The result does not depend on it. */
    double serve_launch_ms;   /* serving: device time each launch aims at,
                                 in ms; 0 = 16. Shorter launches finish
                                 small requests sooner; longer ones waste
                                 less of the GPU on the host work between
                                 launches (more capacity, lower p99). The
                                 results do not depend on it. */
    int pair_partner;         /* PMS_PATH_PAIR: 0 = for every l-mer x of
                                 s_1 the string whose nearest l-mer is
                                 farthest from x (TraverStringRef's string
                                 reordering, Sec. 3.2.3: smaller pair
                                 intersections); 1 = s_2 for every x
                                 (Observation 3.3 as stated). The result
                                 does not depend on it. */
} pms_options;

/* Fill *opt with the defaults above (device 0, auto path). */
void pms_default_options(pms_options *opt);

/* Create a context on opt->device (opt may be NULL for the defaults).
 * *out receives the context, or NULL on failure (status returned). */
int pms_create(pms_ctx **out, const pms_options *opt);

/* Stop the serving engine, free every device and host buffer. NULL-safe. */
void pms_destroy(pms_ctx *ctx);

/* Detail of the last failure on ctx ("" if none); valid until the next call
 * on ctx. With ctx == NULL: the last pms_create failure of this thread. */
const char *pms_last_error(const pms_ctx *ctx);

/* Static name of a status code. */
const char *pms_status_string(int status);

/*
 * Solve one instance. seqs: n*m bytes, row-major (string i at seqs+i*m),
 * host memory. On PMS_OK *motifs points at *count ascending codes owned by
 * ctx (NULL when *count == 0).
 */
int pms_solve(pms_ctx *ctx, const char *seqs, int n, int m, int l, int d,
              const uint64_t **motifs, size_t *count);

/*
 * Solve one instance whose input already sits in device memory.
 * d_seqs: n*m ASCII bytes in device memory. stream: a hipStream_t to run
 * on (NULL = the context's own stream). d_out: device array of cap codes.
 * On PMS_OK the stream has been synchronised, *count holds the number of
 * motifs and d_out[0..*count) the ascending codes. If cap < *count the
 * call returns PMS_ENOMEM with *count set to the size needed and d_out
 * unspecified. The input buffer is only read.
 */
int pms_solve_device(pms_ctx *ctx, const uint8_t *d_seqs, int n, int m,
                     int l, int d, void *stream, uint64_t *d_out, size_t cap,
                     size_t *count);

/*
 * pms_solve_device for callers that cannot allocate device memory (code
 * being captured into a HIP graph, tight serving loops, harnesses that
 * forbid allocation): same arguments, layout, ownership, output and
 * PMS_ENOMEM-with-*count contract as pms_solve_device, but the call makes
 * no hipMalloc, hipFree or other allocation. Its device working memory is a
 * fixed 64 MiB array that each device the library runs on holds until the
 * process ends (looked up by pms_create). It always runs the tiled path,
 * so l must be at least 3 and the tiles at most 4^14 (PMS_EINVAL
 * otherwise); an instance whose index, tile arrays and output heap do not
 * fit in the array is rejected with PMS_ENOMEM before any launch (at
 * n = 20, m = 600 that admits up to l = 19, i.e. up to 4^10 tiles), and
 * PMS_ENOMEM with *count = the motif count when the motifs overflow the
 * heap. The array keeps the last call's contents; what must start at zero
 * is cleared by the call itself. All calls on one device share the one
 * array: calls that overlap in time on the same device (other threads,
 * other contexts, other streams) race and give undefined results.
 */
int pms_solve_device_noalloc(pms_ctx *ctx, const uint8_t *d_seqs, int n,
                             int m, int l, int d, void *stream,
                             uint64_t *d_out, size_t cap, size_t *count);

/*
 * Quorum motifs (Definition 5 and the qPMS definition, Sec. 1.2.5): every
 * l-mer M such that at least q of the n strings have an l-mer within
 * Hamming distance d of M. q = n is exactly pms_solve. Same arguments,
 * layout, ownership and output as pms_solve, plus q. Runs the tiled path
 * with a per-code count of strings without a d-neighbour (tile suffix at
 * most 8 bases) while its tiles fit (3 <= l <= 22); otherwise, or when the
 * context's path is forced to PMS_PATH_FILTER, the sample-driven filter
 * with a miss count per candidate: candidates from the d-spheres of the
 * l-mers of s_1..s_(n-q+1) (Observation 3.1), each kept once, from its
 * first such l-mer. PMS_EINVAL when q < 1 or q > n, when n - q > 30, when
 * the context's path is forced to PMS_PATH_BITSET or PMS_PATH_PAIR, or
 * when (n-q+1)*(m-l+1) reaches 2^27. The output can be large (a sizeable
 * fraction of 4^l codes when q is small): it is sized on the device before
 * it is copied.
 */
int pms_solve_quorum(pms_ctx *ctx, const char *seqs, int n, int m, int l,
                     int d, int q, const uint64_t **motifs, size_t *count);

/* pms_solve_quorum with input and output in device memory, as
 * pms_solve_device (PMS_ENOMEM with *count = the size needed when cap is
 * too small). */
int pms_solve_quorum_device(pms_ctx *ctx, const uint8_t *d_seqs, int n,
                            int m, int l, int d, int q, void *stream,
                            uint64_t *d_out, size_t cap, size_t *count);

/*
 * Motifs over another alphabet (Sec. 1.2.5 states the problem for any
 * alphabet; Table 3.1 sizes the spheres for any |Sigma|), e.g. the 20
 * amino-acid letters. alphabet: sigma distinct bytes (2 <= sigma <= 32);
 * the letter alphabet[i] has code i and a motif is reported as the base-sigma
 * number sum_j code(M[j]) * sigma^(l-1-j) (first letter in the top digit,
 * so numeric order is the alphabet's lexicographic order). seqs: n*m bytes
 * of those letters, row-major. Runs the sample-driven filter (candidates
 * from the spheres of s_1's l-mers, strings tested in order with early
 * exit), then sorts and drops repeats on the device. Output as pms_solve.
 * PMS_EBASE for a byte outside the alphabet; PMS_EINVAL for a bad shape, a
 * bad alphabet, sigma^l above 2^64 (codes past 64 bits; 2^64 itself, as
 * 16^16, is allowed), a sphere beyond 2^62 candidates (or 2^22 position
 * sets) or more than 2^62 candidates over all m-l+1 references. alphabet
 * "ACGT" with sigma 4 is pms_solve.
 */
int pms_solve_alphabet(pms_ctx *ctx, const char *alphabet, int sigma,
                       const char *seqs, int n, int m, int l, int d,
                       const uint64_t **motifs, size_t *count);

/* pms_solve_alphabet with input and output in device memory, as
 * pms_solve_device (PMS_ENOMEM with *count = the size needed when cap is
 * too small). */
int pms_solve_alphabet_device(pms_ctx *ctx, const char *alphabet, int sigma,
                              const uint8_t *d_seqs, int n, int m, int l,
                              int d, void *stream, uint64_t *d_out,
                              size_t cap, size_t *count);

/*
 * Long motifs, 1 <= l <= 64 (Sec. 3.3.1 keeps an l-mer that one word cannot
 * hold in ceil(l/32) words per group). The problem is pms_solve's; a code
 * takes up to 128 bits and is returned as two uint64 words, high word first:
 * motif i is (*motifs)[2i] = bits 127..64 and (*motifs)[2i+1] = bits 63..0
 * of sum_j b(M[j]) * 4^(l-1-j). Motifs ascend by that 128-bit value;
 * *count counts motifs (2 * *count words). Runs the sample-driven filter
 * with one 64-bit word per bit plane (candidates from the spheres of s_1's
 * l-mers, strings tested in order with early exit, each motif kept from the
 * first l-mer of s_1 within d of it), then sorts on the device. The words
 * belong to the context as for pms_solve. Errors as pms_solve, with the
 * domain 1 <= l <= 64; PMS_EINVAL also for a sphere beyond 2^62 candidates,
 * 2^22 position sets, or more than 2^62 candidates over all m-l+1
 * references. For l <= 32 the low words are pms_solve's codes.
 */
int pms_solve_wide(pms_ctx *ctx, const char *seqs, int n, int m, int l,
                   int d, const uint64_t **motifs, size_t *count);

/* pms_solve_wide with input and output in device memory, as
 * pms_solve_device: d_out holds 2 * cap words (cap motifs); PMS_ENOMEM with
 * *count = the number of motifs when cap is too small. */
int pms_solve_wide_device(pms_ctx *ctx, const uint8_t *d_seqs, int n, int m,
                          int l, int d, void *stream, uint64_t *d_out,
                          size_t cap, size_t *count);

/* One instance of a batch. seqs: n*m host bytes. q: quorum of an
 * (l,d,q)-motif search (1 <= q < n; see pms_solve_quorum), 0 or n for the
 * plain (l,d) search. */
typedef struct {
    const char *seqs;
    int n, m, l, d;
    int q;
} pms_instance;

/* Result of one instance. motifs: ctx-owned, ascending; status: PMS_*. */
typedef struct {
    const uint64_t *motifs;
    size_t count;
    int status;
} pms_result;

/*
 * Solve k independent instances of any sizes together: all of them run in
 * one persistent launch that drains a device work queue, replayed as a
 * captured HIP graph when the same batch shape repeats. Instances the
 * tiled kernel does not suit, and quorum instances (1 <= q < n), are solved
 * one by one after it, as pms_solve / pms_solve_quorum would. out[i]
 * receives instance i's result (status PMS_EBASE / PMS_EINVAL for a bad
 * instance, q outside 0..n included; the others still complete). Returns
 * PMS_OK if every instance succeeded, else the first failing status.
 */
int pms_solve_batch(pms_ctx *ctx, const pms_instance *in, int k,
                    pms_result *out);

/*
 * Serving (continuous batching). pms_submit copies the request and queues
 * it; the context's engine thread admits queued requests while device
 * memory and slots allow and runs admitted requests' work together, a
 * bounded slice per launch, so requests join and leave between launches.
 * Two launches are in flight: the next is queued while the current runs,
 * and finished requests are compacted and copied out beside it.
 * Each launch aims at pms_options.serve_launch_ms of device time (default
 * 16 ms), shared equally by cost among the admitted requests (processor
 * sharing): a small request finishes within a launch or two, a large one in
 * proportion to its size and load.
 * *ticket identifies the request. PMS_EBUSY if the waiting queue is full;
 * PMS_EINVAL for a bad shape, for a shape the tiled path does not suit
 * (l < 3, or more than 4^14 tiles; use pms_solve), for a quorum request
 * (in->q other than 0 or n; use pms_solve_quorum or pms_solve_batch), and
 * PMS_ENOMEM for a request larger than the serving pool (all checked
 * before queueing).
 * Bad bytes are found on the device: the result's status is PMS_EBASE.
 * While requests are in flight, do not call pms_solve* or pms_autotune on
 * the same context from another thread.
 */
int pms_submit(pms_ctx *ctx, const pms_instance *in, uint64_t *ticket);

/* PMS_PENDING until the request finished; then PMS_OK (or its error) with
 * *out filled; the result stays valid until pms_release(ticket). */
int pms_poll(pms_ctx *ctx, uint64_t ticket, pms_result *out);

/* Block until the request finished (or timeout_ms elapsed: PMS_PENDING). */
int pms_wait(pms_ctx *ctx, uint64_t ticket, int timeout_ms, pms_result *out);

/* Forget a finished request and free its result. */
int pms_release(pms_ctx *ctx, uint64_t ticket);

/* Times of a request on the library's steady clock (pms_clock_ms):
 * submission, admission to the device and completion (0 if not yet). */
int pms_ticket_times(pms_ctx *ctx, uint64_t ticket, double *t_submit_ms,
                     double *t_admit_ms, double *t_done_ms);

/* Milliseconds on the steady clock used by pms_ticket_times. */
double pms_clock_ms(void);

/* Calibration, not part of any solve: the device's rate of the Hamming
 * test of Sec. 3.3.1 as the filter computes it (XOR, OR, popcount, running
 * minimum over two bit planes), at full occupancy from registers only.
 * *tests_per_s receives the rate. Runs a kernel of tens of milliseconds on
 * the context's stream. Returns PMS_EINVAL for NULL arguments. */
int pms_test_rate(pms_ctx *ctx, double *tests_per_s);

/* Calibration, not part of any solve: the device's rate of the tile
 * kernels' mark (a single-bit 32-bit atomic OR into LDS) at their
 * occupancy, with every half wave on 32 different banks. *ors_per_s
 * receives lane ORs per second over the whole device. Runs a kernel of
 * tens of milliseconds on the context's stream. PMS_EINVAL for NULL
 * arguments. */
int pms_lds_rate(pms_ctx *ctx, double *ors_per_s);

/* Timing and work counters of the last pms_solve / pms_solve_device /
 * pms_solve_batch call. Kernel times come from HIP events recorded on the
 * stream each kernel ran on. */
typedef struct {
    int path;                 /* PMS_PATH_* actually used */
    int tile_suffix;          /* tiled/bitset: bases per tile suffix (s) */
    double ms_total;          /* host wall time of the call */
    double ms_index;          /* pack + l-mer index kernels (bitset
                                 path: and the per-tile string order) */
    double ms_main;           /* filter / tiled kernels; bitset path: its
                                 n pass launches */
    double ms_output;         /* compaction, ordering, copies */
    uint64_t main_launches;   /* launches of the main kernel */
    uint64_t hcanon;          /* filter path: Hamming tests in the
                                 canonical order of the sample-driven
                                 method; 0 for other paths */
    uint64_t tiles;           /* tiled/bitset: tiles processed */
    uint64_t tile_passes;     /* tiled/bitset: (tile, string) passes run */
    uint64_t marks;           /* tiled/bitset: 64-bit sphere-word ORs */
    uint64_t filter_tests;    /* tiled: Hamming tests of the filter stage;
                                 pair path: tests against s_3..s_n (L per
                                 string examined); filter path: tests the
                                 kernel executed, candidate slots x l-mers
                                 scanned over whole waves (a wave leaves a
                                 string once each of its live candidates
                                 has a hit), beside the canonical hcanon */
    uint64_t bytes_main;      /* bitset path: device bytes read+written */
    uint64_t retries;         /* output-capacity retries */
    uint64_t pairs;           /* pair path: pairs (x, y) with d_H <= 2d */
    uint64_t candidates;      /* pair path: sum of |B(x,d) ∩ B(y,d)| */
    int tile_threads;         /* tiled path: threads per workgroup of the
                                 tile kernel (256 or 512; unless forced by
                                 pms_options.tile_threads: 512 for tiles of
                                 4^8 or 4^9 codes, and for a batch when
                                 most of its planned work is in such
                                 tiles); 0 when no tile kernel ran */
    int graph_replayed;       /* pms_solve_batch: 1 when the call replayed
                                 the HIP graph captured by an earlier call
                                 of the same batch shape, 0 when it
                                 captured one; 0 for other calls */
} pms_stats;

int pms_last_stats(const pms_ctx *ctx, pms_stats *out);

/* Serving statistics since pms_create. */
typedef struct {
    uint64_t submitted, completed, launches;
    uint64_t max_inflight;
    double busy_ms;           /* kernel time of the engine's launches */
    uint64_t retries;         /* requests run again because their motifs
                                 overflowed the output room sized for them */
} pms_serve_stats;

int pms_serve_stats_get(const pms_ctx *ctx, pms_serve_stats *out);

/*
 * Filter path only: copy the per-reference Hamming-test counts of the last
 * solve, when it ran the plain (q = n) filter path (entry j: the tests spent
 * on candidates from the l-mer of s_1 at offset j). n_refs must be m-l+1 of
 * that solve; PMS_EINVAL otherwise, and after any solve on another path
 * (tiled, bitset, pair, quorum, another alphabet, long motifs).
 */
int pms_last_hcanon_per_ref(const pms_ctx *ctx, uint64_t *out, size_t n_refs);

/*
 * Autotuner. Times every tile configuration (suffix length, survivor
 * threshold and, for tiles of at least 4^7 codes unless
 * pms_options.tile_threads fixes it, the workgroup size 256 or 512) of the
 * tiled kernel on a synthetic planted instance shaped like (n, m, l, d),
 * keeps the fastest, and stores it in the context's tuning table (and
 * tune_cache file, if set) under the key (l, d, n-bucket, m-bucket). Every
 * configuration gives the same motif set; only speed differs. *best_s /
 * *best_t receive the suffix and threshold chosen (may be NULL); the
 * workgroup size in effect shows in pms_last_stats' tile_threads.
 */
int pms_autotune(pms_ctx *ctx, int n, int m, int l, int d, int *best_s,
                 int *best_t);

/* Override the tile configuration used for (l, d) from now on (0 = back to
 * the tuned or default choice). For testing configuration invariance. */
int pms_set_tile_config(pms_ctx *ctx, int l, int d, int s, int surv_t);

#ifdef __cplusplus
}
#endif

#endif /* PMS_H */
