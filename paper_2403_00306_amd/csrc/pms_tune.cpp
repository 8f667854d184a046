// pms_tune.cpp -- autotuner for the tiled kernel's tile shape.
//
// The tile shape decides how the 4^l code space is cut (suffix length s:
// 4^s codes per tile, 4^(l-s) tiles), when a tile stops ANDing sphere
// unions and starts filtering the codes it has left (surv_t), and the
// workgroup size of the tile kernel (256 or 512 threads). None changes the
// motif set, only the split of work between marking, prefix tests and
// Hamming tests and how it is spread over the chip. The tuner times every
// shape on a synthetic planted instance of the requested size (a random
// motif with d substitutions at a random offset of every string, as in the
// planted problem of Sec. 1.2.5), checks that every shape returns the same
// set, and keeps the fastest per (l, d, n-bucket, m-bucket).
#include "pms_host.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <random>

using namespace pms;

namespace pms {

void load_tune_cache(pms_ctx *c)
{
    if (c->tune_path.empty())
        return;
    FILE *f = fopen(c->tune_path.c_str(), "r");
    if (!f)
        return;
    // lines "key s surv_t tpb"
    char line[128];
    while (fgets(line, sizeof line, f)) {
        unsigned long long key;
        int s, t, tpb = 0;
        const int k = sscanf(line, "%llx %d %d %d", &key, &s, &t, &tpb);
        if (k < 3)
            continue;
        if (tpb != 256 && tpb != 512)
            tpb = 0;
        if (s >= kMinSuffix && s <= kMaxSuffix && t >= 1 && t <= kSurvMax)
            c->tune[key] = {s, t, tpb};
    }
    fclose(f);
}

static void save_tune_cache(pms_ctx *c)
{
    if (c->tune_path.empty())
        return;
    const std::string tmp = c->tune_path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f)
        return;
    for (auto &kv : c->tune)
        fprintf(f, "%llx %d %d %d\n", (unsigned long long)kv.first,
                kv.second.s, kv.second.surv_t, kv.second.tpb);
    fclose(f);
    rename(tmp.c_str(), c->tune_path.c_str());
}

}  // namespace pms

extern "C" int pms_autotune(pms_ctx *c, int n, int m, int l, int d,
                            int *best_s, int *best_t)
{
    if (!c)
        return PMS_EINVAL;
    int rc = check_shape(n, m, l, d);
    if (rc || l < kMinSuffix)
        return c->fail(PMS_EINVAL, "autotune: bad shape n=%d m=%d l=%d d=%d",
                       n, m, l, d);
    hipSetDevice(c->device);
    // synthetic planted instance (tuning input only): uniform DNA with a
    // random motif, d bases of it changed, at a random offset of each string
    std::mt19937_64 rng(tune_key(l, d, n, m) ^ 0x5eed5eedull);
    std::vector<char> seqs((size_t)n * m);
    for (auto &ch : seqs)
        ch = "ACGT"[rng() & 3];
    std::vector<int> motif(l);
    for (auto &b : motif)
        b = (int)(rng() & 3);
    for (int i = 0; i < n; i++) {
        std::vector<int> occ = motif;
        std::vector<int> pos(l);
        for (int j = 0; j < l; j++)
            pos[j] = j;
        for (int k = 0; k < d; k++) {   // d distinct positions, new bases
            const int r = k + (int)(rng() % (uint64_t)(l - k));
            std::swap(pos[k], pos[r]);
            occ[pos[k]] = (occ[pos[k]] + 1 + (int)(rng() % 3)) & 3;
        }
        const int at = (int)(rng() % (uint64_t)(m - l + 1));
        for (int j = 0; j < l; j++)
            seqs[(size_t)i * m + at + j] = "ACGT"[occ[j]];
    }

    // tile suffixes around the default (more tiles vs longer tiles), three
    // survivor thresholds, and both workgroup sizes where the tile holds at
    // least 4^7 codes (unless the caller fixed the size)
    std::vector<TileCfg> cand;
    const int s_def = default_suffix(l);
    const int s_hi = std::min(std::min(kMaxSuffix, l), s_def + 2);
    const int s_lo = std::max(kMinSuffix, std::max(l - kMaxTilePrefix, s_def - 2));
    for (int s = s_lo; s <= s_hi; s++)
        for (int t : {32, 64, 96}) {
            if (c->opt.tile_threads != 0 || s < 7) {
                cand.push_back({s, t, 0});
                continue;
            }
            cand.push_back({s, t, 256});
            cand.push_back({s, t, 512});
        }

    TileCfg saved{};
    bool had_override;
    {
        std::lock_guard<std::mutex> g(c->tune_mu);
        auto it = c->override_cfg.find({l, d});
        had_override = it != c->override_cfg.end();
        if (had_override)
            saved = it->second;
    }
    double best = 1e300;
    TileCfg pick = cand.front();
    std::vector<uint64_t> ref, got;
    bool have_ref = false;
    int status = PMS_OK;
    for (auto &cf : cand) {
        {
            std::lock_guard<std::mutex> g(c->tune_mu);
            c->override_cfg[{l, d}] = cf;
        }
        double t_min = 1e300;
        for (int rep = 0; rep < 2 && status == PMS_OK; rep++) {
            SolveOut r{};
            rc = solve_core(c, seqs.data(), nullptr, n, m, l, d, c->stream,
                            nullptr, 0, PMS_PATH_TILED, &r);
            if (rc) {
                status = rc;
                break;
            }
            t_min = std::min(t_min, c->last.ms_main + c->last.ms_output);
            if (rep == 0) {
                got.resize(r.count);
                if (r.count &&
                    hipMemcpy(got.data(), r.d_out, r.count * 8,
                              hipMemcpyDeviceToHost) != hipSuccess) {
                    status = c->fail(PMS_EDEVICE, "autotune: copy failed");
                    break;
                }
                if (!have_ref) {
                    ref = got;
                    have_ref = true;
                } else if (got != ref) {
                    status = c->fail(PMS_EDEVICE, "autotune: tile shape s=%d "
                                     "t=%d threads=%d changed the motif set",
                                     cf.s, cf.surv_t, cf.tpb);
                    break;
                }
            }
        }
        if (status != PMS_OK)
            break;
        if (t_min < best) {
            best = t_min;
            pick = cf;
        }
    }
    {
        std::lock_guard<std::mutex> g(c->tune_mu);
        if (had_override)
            c->override_cfg[{l, d}] = saved;
        else
            c->override_cfg.erase({l, d});
        if (status == PMS_OK) {
            c->tune[tune_key(l, d, n, m)] = pick;
            save_tune_cache(c);
        }
    }
    if (status != PMS_OK)
        return status;
    if (best_s)
        *best_s = pick.s;
    if (best_t)
        *best_t = pick.surv_t;
    return PMS_OK;
}

// Rate of the Hamming-test instruction mix on this device at full
// occupancy, from registers only (a check of the integer peak that the
// roofline figures assume).
extern "C" int pms_test_rate(pms_ctx *c, double *tests_per_s)
{
    if (!c || !tests_per_s)
        return PMS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    int rc = c->alloc(c->aux, 256);
    if (rc)
        return rc;
    const hipStream_t st = c->stream;
    const int grid = std::max(1, c->n_cu * test_rate_blocks_per_cu());
    unsigned int *sink = (unsigned int *)c->aux.p;
    HIPCHK(c, launch_test_rate(grid, 64, 1u, sink, st));   // warm-up
    // about 2e11 tests: tens of milliseconds
    const uint64_t per_iter =
        (uint64_t)grid * kTPB * test_rate_tests_per_thread(1);
    const int iters = (int)std::max<uint64_t>(
        64, std::min<uint64_t>(1u << 20, 200000000000ull / per_iter));
    HIPCHK(c, hipEventRecord(c->ev[0], st));
    HIPCHK(c, launch_test_rate(grid, iters, 2u, sink, st));
    HIPCHK(c, hipEventRecord(c->ev[1], st));
    HIPCHK(c, hipEventSynchronize(c->ev[1]));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    if (ms <= 0)
        return c->fail(PMS_EDEVICE, "test rate: no elapsed time");
    *tests_per_s = (double)per_iter * (double)iters / ((double)ms / 1e3);
    return PMS_OK;
}

extern "C" int pms_lds_rate(pms_ctx *c, double *ors_per_s)
{
    if (!c || !ors_per_s)
        return PMS_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    int rc = c->alloc(c->aux, 256);
    if (rc)
        return rc;
    const hipStream_t st = c->stream;
    const int grid = std::max(1, c->n_cu * lds_rate_blocks_per_cu());
    unsigned int *sink = (unsigned int *)c->aux.p;
    HIPCHK(c, launch_lds_rate(grid, 16, sink, st));   // warm-up
    // about 1e11 ORs: a few tens of milliseconds
    const uint64_t per_iter = (uint64_t)grid * lds_rate_ors_per_block(1);
    const int iters = (int)std::max<uint64_t>(
        16, std::min<uint64_t>(1u << 20, 100000000000ull / per_iter));
    HIPCHK(c, hipEventRecord(c->ev[0], st));
    HIPCHK(c, launch_lds_rate(grid, iters, sink, st));
    HIPCHK(c, hipEventRecord(c->ev[1], st));
    HIPCHK(c, hipEventSynchronize(c->ev[1]));
    float ms = 0;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
    if (ms <= 0)
        return c->fail(PMS_EDEVICE, "lds rate: no elapsed time");
    *ors_per_s = (double)per_iter * (double)iters / ((double)ms / 1e3);
    return PMS_OK;
}
