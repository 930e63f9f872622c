// h-degrees without any device allocation: khdeg_compute_noalloc.
//
// The multi-source BFS of khdeg_compute needs scratch memory (visited and
// frontier words, frontier maps and lists, counters).  This entry point
// takes all of it from one file-scope device array, `scratch`, that the
// code object holds on every GPU the library runs on until the process
// ends.  In host code the array's name is only a host-side stand-in, so
// the device address is looked up once per device with hipGetSymbolAddress
// (from khc_create, with the device current) and only that address is used
// afterwards.  Every call on a GPU shares that GPU's array: overlapping
// calls on one device race, and each call clears the parts that must start
// at zero with a fill kernel.
#include <mutex>

#include "khc_internal.h"

namespace khc {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

int noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return KHC_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return KHC_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return KHC_EHIP;
    }
    g_scratch_ptr[device] = ptr;
    return KHC_OK;
}

}  // namespace khc

using namespace khc;

extern "C" int khdeg_compute_noalloc(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                                     uint32_t *deg) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !deg) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h == 0) return set_error(ctx, KHC_EINVAL, "h must be >= 1");
    if (h > kMaxRoundH) return set_error(ctx, KHC_EINVAL, "h above 1024");
    (void)hipSetDevice(ctx->device);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
    }
    if (!base) return set_error(ctx, KHC_EHIP, "no static scratch address for this device");
    if (g->n == 0) return KHC_OK;
    // the widest batch (up to the context's maximum width) whose buffers,
    // plus the source list and its counter, fit the scratch array
    const size_t fixed = (((size_t)g->n * 4 + 255) & ~(size_t)255) + 256 + 256;
    int W = 0;
    for (int w = ctx->max_width; w >= 1; w >>= 1)
        if (fixed + msbfs_arena_bytes(g, h, w) <= kScratchBytes) {
            W = w;
            break;
        }
    if (!W)
        return set_error(ctx, KHC_ENOMEM,
                         "graph too large for the static scratch of khdeg_compute_noalloc (" +
                             std::to_string(fixed + msbfs_arena_bytes(g, h, 1)) + " bytes needed at width 1, " +
                             std::to_string(kScratchBytes) + " available)");
    Arena arena;
    arena.base = (char *)base;
    arena.bytes = kScratchBytes;
    return khdeg_compute_impl(ctx, g, alive, h, deg, &arena, W);
}
