// pms_noalloc.hip -- pms_solve_device_noalloc: the device-resident tiled
// solve with all of its device working memory (l-mer index, tile arrays,
// output heap, descriptor, counters) in one file-scope device array instead
// of context allocations, for callers that cannot allocate.
//
// The array is a device symbol: its host-side name is a stand-in, not a
// device address. Each device's copy is looked up once, with that device
// current, by hipGetSymbolAddress when a context is created on it (or, if
// that failed, at the entry point's first call there); only the address
// found that way is ever handed to kernels or copies.
#include "pms_host.h"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
char *g_ptr[kMaxDevices] = {};

}  // namespace

namespace pms {

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Caller has made `device` current.
char *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess ||
            !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[device] = (char *)p;
    }
    return g_ptr[device];
}

}  // namespace pms

using namespace pms;

extern "C" int pms_solve_device_noalloc(pms_ctx *c, const uint8_t *d_seqs,
                                        int n, int m, int l, int d,
                                        void *stream, uint64_t *d_out,
                                        size_t cap, size_t *count)
{
    if (!c)
        return PMS_EINVAL;
    if (!d_seqs || !count || !d_out)
        return c->fail(PMS_EINVAL, "NULL argument");
    *count = 0;
    if (hipSetDevice(c->device) != hipSuccess)
        return c->fail(PMS_EDEVICE, "hipSetDevice(%d) failed", c->device);
    char *base = noalloc_scratch(c->device);
    if (!base)
        return c->fail(PMS_EDEVICE, "no address for the scratch array on "
                       "device %d", c->device);
    const FixedArena fa{base, kScratchBytes};
    hipStream_t st = stream ? (hipStream_t)stream : c->stream;
    SolveOut r{};
    const int rc = solve_core(c, nullptr, d_seqs, n, m, l, d, st, d_out, cap,
                              PMS_PATH_TILED, &r, 0, &fa);
    *count = r.count;
    return rc;
}
