// pms_host.h -- host-side state of libpms shared by the C ABI files
// (plain solves, batch, serving engine, autotuner).
#pragma once

#include "pms.h"
#include "pms_internal.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace pms {

constexpr size_t kPinnedDescBytes = 1 << 20;   // descriptor + string order
constexpr size_t kPinnedHcEntries = 1 << 16;   // per-reference test counts
constexpr int kMaxTilePrefix = 14;             // at most 4^14 tiles

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }
inline uint64_t pow4(int k) { return k <= 0 ? 1ull : (1ull << (2 * k)); }

double now_ms();
double nb_real(int l, int d);
uint64_t nb_exact(int l, int d);
int check_shape(int n, int m, int l, int d);
void cost_model(int n, int m, int l, int d, int s, int surv_t, double &cf,
                double &ct);
int default_suffix(int l);
uint64_t tune_key(int l, int d, int n, int m);

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Offsets of one instance's device arrays inside an arena.
struct InstLayout {
    size_t seqs = 0, packed = 0, phi = 0, plo = 0, planes = 0, codes = 0,
           order = 0, bad = 0, tile_cnt = 0, tile_heap_off = 0,
           tile_pos = 0, scan = 0, heap_top = 0, heap = 0, out = 0,
           total = 0;
};

InstLayout layout_instance(int n, int m, int l, uint64_t ntiles,
                           uint64_t heap_cap, bool own_seqs, bool own_tiles,
                           bool own_out);
InstDev make_desc(char *base, const InstLayout &o, const uint8_t *seqs,
                  int n, int m, int l, int d, int s, int surv_t,
                  uint64_t ntiles, uint64_t heap_cap);

// Tile shape of the tiled kernel: suffix bases s (4^s codes per tile), the
// survivor threshold, and the workgroup size (256 or 512; 0: automatic).
struct TileCfg {
    int s;
    int surv_t;
    int tpb;
};

struct Plan {
    int path;     // PMS_PATH_FILTER / PMS_PATH_TILED / PMS_PATH_BITSET
    int s;        // tile suffix bases
    int surv_t;   // survivor threshold of the tiled filter stage
    int tpb;      // tile kernel workgroup size, 0: automatic
    uint64_t ntiles;
    double cost_filter, cost_tiled;
};

// Tile kernel workgroup size: the caller's choice (pms_options.tile_threads)
// or, when that is 0, the automatic one.
inline bool pick_wide(const pms_ctx *c, bool automatic);

struct SolveOut {
    uint64_t *d_out;
    size_t count;
};

// Device memory a solve must work in instead of the context's arena: the
// tiled path only, no allocation, output in the caller's buffer.
struct FixedArena {
    char *base;
    size_t bytes;
};

struct Server;

}  // namespace pms

struct pms_ctx {
    pms_options opt{};
    int device = 0;
    std::string err;
    std::string tune_path;
    hipStream_t stream = nullptr;
    int n_cu = 0, tiled_bpc = 1, filter_bpc = 1, tiled_q_bpc = 1,
        alpha_bpc = 1, pair_bpc = 1, tiled_wide_bpc = 1, bitset_bpc = 1,
        wide_bpc = 1;
    size_t budget = 0;
    std::atomic<size_t> held{0};

    void *tables_mem = nullptr;
    pms::Tables tb{};

    pms::DevBuf arena, out, masks, hc_ref, sort_scr, bitset, alive;
    pms::DevBuf aux;              // any-alphabet path: heap, repeat removal
    int masks_l = -1, masks_d = -1;
    uint64_t masks_nb = 0;
    std::vector<uint64_t> host_out;
    pms_stats last{};
    int last_L = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    unsigned long long *pinned = nullptr;      // small D2H staging
    char *pinned_desc = nullptr;               // descriptor H2D staging
    unsigned long long *pinned_hc = nullptr;   // per-reference counts

    std::mutex tune_mu;
    std::map<uint64_t, pms::TileCfg> tune;
    std::map<std::pair<int, int>, pms::TileCfg> override_cfg;

    // batch
    pms::DevBuf b_arena;
    char *b_pinned = nullptr;
    size_t b_pinned_bytes = 0;
    std::vector<uint64_t> b_host;
    std::vector<std::vector<uint64_t>> b_solo;
    hipGraphExec_t b_graph = nullptr;
    hipGraph_t b_graph_def = nullptr;
    uint64_t b_graph_key = 0;
    uint64_t b_graph_replays = 0;
    uint64_t b_heap_key = 0;      // shape of the last batch
    uint64_t b_heap_need = 0;     // heap it needed (with slack)
    // single solves: heap entries a shape (n, m, l, d, q) last needed, so
    // that repeated calls start large enough instead of rerunning
    std::map<std::tuple<int, int, int, int, int>, uint64_t> heap_need;

    pms::Server *srv = nullptr;

    int fail(int status, const char *fmt, ...)
        __attribute__((format(printf, 3, 4)));
    int alloc(pms::DevBuf &b, size_t bytes);
    void release(pms::DevBuf &b);
    pms::TileCfg tile_config(int n, int m, int l, int d);
    pms::Plan plan(int n, int m, int l, int d, int forced);
};

#define HIPCHK(c, x)                                                         \
    do {                                                                     \
        hipError_t e_ = (x);                                                 \
        if (e_ != hipSuccess)                                                \
            return (c)->fail(PMS_EDEVICE, "%s failed: %s", #x,               \
                             hipGetErrorString(e_));                         \
    } while (0)

namespace pms {

constexpr int kWideMinSuffix = 8;  // 512-thread tile kernel from 4^8 codes

inline bool pick_wide(const pms_ctx *c, bool automatic)
{
    return c->opt.tile_threads == 512 ||
           (c->opt.tile_threads == 0 && automatic);
}

// The same for one instance's plan: the caller's choice, else the tuned
// size, else 512 for tiles of at least 4^kWideMinSuffix codes.
inline bool pick_wide(const pms_ctx *c, const Plan &p)
{
    if (c->opt.tile_threads != 0 || p.tpb == 0)
        return pick_wide(c, p.s >= kWideMinSuffix);
    return p.tpb == 512;
}
// q = 0 (or q = n): plain PMS; 1 <= q < n: (l,d,q)-motifs (tiled path).
// fixed != nullptr: work in that memory (tiled path, d_out_ext required),
// allocate nothing, PMS_ENOMEM when the instance does not fit.
int solve_core(pms_ctx *c, const char *host_seqs, const uint8_t *d_seqs,
               int n, int m, int l, int d, hipStream_t st, uint64_t *d_out_ext,
               size_t cap_ext, int forced_path, SolveOut *res, int q = 0,
               const FixedArena *fixed = nullptr);
// Device address of the fixed scratch array on the context's device,
// looked up once per device (pms_noalloc.hip); nullptr if unavailable.
char *noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
// Pair path: lists compatible pairs and filters their candidates into
// I.heap (index already built on st); *found = survivors, possibly more
// than I.heap_cap (then nothing beyond it was written).
int pair_run(pms_ctx *c, const InstDev &I, hipStream_t st, uint64_t *found,
             pms_stats &S);
void serve_shutdown(pms_ctx *c);
void load_tune_cache(pms_ctx *c);
}  // namespace pms
