// C ABI entry points: context, workspace, graph store and h-degrees.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "khc_internal.h"

namespace khc {

int set_error(khc_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int prof_begin(khc_ctx *ctx, int cls, double bytes) {
    if (!ctx->profile) return -1;
    khc_ctx::ProfRec r;
    for (int i = 0; i < 2; ++i) {
        hipEvent_t ev;
        if (!ctx->prof_pool.empty()) {
            ev = ctx->prof_pool.back();
            ctx->prof_pool.pop_back();
        } else if (hipEventCreate(&ev) != hipSuccess) {
            (void)hipGetLastError();
            return -1;
        }
        (i == 0 ? r.a : r.b) = ev;
    }
    r.cls = cls;
    r.bytes = bytes;
    (void)hipEventRecord(r.a, ctx->stream);
    ctx->prof_pending.push_back(r);
    return (int)ctx->prof_pending.size() - 1;
}

void prof_end(khc_ctx *ctx, int rec) {
    if (rec < 0) return;
    (void)hipEventRecord(ctx->prof_pending[rec].b, ctx->stream);
}

int check_hip(khc_ctx *ctx, hipError_t e, const char *what) {
    if (e == hipSuccess) return KHC_OK;
    if (ctx) ctx->sticky = 1;
    return set_error(ctx, KHC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int ws_get(khc_ctx *ctx, int slot, size_t bytes, void **out) {
    if (bytes == 0) bytes = 8;
    DevBuf &b = ctx->bufs[slot];
    if (b.bytes >= bytes) {
        *out = b.ptr;
        return KHC_OK;
    }
    size_t want = bytes + bytes / 8;  // some headroom for growth
    uint64_t total = ctx->ws_bytes - b.bytes + want;
    if (ctx->ws_limit && total > ctx->ws_limit) {
        want = bytes;
        total = ctx->ws_bytes - b.bytes + want;
        if (total > ctx->ws_limit)
            return set_error(ctx, KHC_ENOMEM, "workspace limit exceeded (" + std::to_string(total) +
                                                  " > " + std::to_string(ctx->ws_limit) + " bytes)");
    }
    if (b.ptr) {
        // captured persistent launches hold the old address
        drop_persist_graphs(ctx, nullptr);
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return check_hip(ctx, e, "stream sync before workspace growth");
        (void)hipFree(b.ptr);
        ctx->ws_bytes -= b.bytes;
        b.ptr = nullptr;
        b.bytes = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, KHC_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
    }
    // zero on allocation: kernels rely on some buffers starting cleared
    e = hipMemsetAsync(p, 0, want, ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "workspace clear");
    b.ptr = p;
    b.bytes = want;
    ctx->ws_bytes += want;
    *out = p;
    return KHC_OK;
}

namespace {

// Error bits of the CSR validator.
enum : uint32_t {
    VBAD_OFFSETS = 1,
    VBAD_RANGE = 2,
    VSELF_LOOP = 4,
    VUNSORTED = 8,
    VASYMMETRIC = 16,
};

__global__ void validate_rows_kernel(uint32_t n, uint64_t nnz, const uint64_t *row_ptr,
                                     uint32_t *flags) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 && (row_ptr[0] != 0 || row_ptr[n] != nnz)) atomicOr(flags, VBAD_OFFSETS);
    if (v < n && row_ptr[v + 1] < row_ptr[v]) atomicOr(flags, VBAD_OFFSETS);
}

// One thread per arc: range, self-loop, strict order within the row, and
// the reverse arc (binary search in the target row).
__global__ void validate_arcs_kernel(uint32_t n, uint64_t nnz, const uint64_t *row_ptr,
                                     const uint32_t *col, uint32_t *flags) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    // row of arc e: last v with row_ptr[v] <= e
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (row_ptr[mid] <= e) lo = mid; else hi = mid;
    }
    const uint32_t v = lo;
    const uint32_t u = col[e];
    if (u >= n) {
        atomicOr(flags, VBAD_RANGE);
        return;
    }
    if (u == v) atomicOr(flags, VSELF_LOOP);
    if (e > row_ptr[v] && col[e - 1] >= u) atomicOr(flags, VUNSORTED);
    uint64_t a = row_ptr[u], b = row_ptr[u + 1];
    bool found = false;
    while (a < b) {
        uint64_t mid = a + (b - a) / 2;
        uint32_t c = col[mid];
        if (c == v) { found = true; break; }
        if (c < v) a = mid + 1; else b = mid;
    }
    if (!found) atomicOr(flags, VASYMMETRIC);
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// flags |= 1 if some listed vertex id is >= n.
__global__ void check_ids_kernel(const uint32_t *verts, uint32_t count, uint32_t n, uint32_t *flags) {
    bool bad = false;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        bad |= verts[i] >= n;
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 1u);
}

// Append every live vertex that has a live neighbour (the others have
// h-degree 0 and need no BFS), walking the row schedule: heavy rows, then
// light rows with arcs, each by descending degree.  Wave-aggregated atomic
// append, so the list is close to that order.  Sources of similar degree
// then share a BFS batch: the balls of a batch of hubs cover most of the
// graph and saturate their rows' words early (the pull stops gathering
// there), and batches of low-degree sources keep small frontiers.
__global__ void compact_sources_kernel(const uint32_t *heavy_rows, uint32_t n_heavy, const uint32_t *light_rows,
                                       uint32_t n_light_nz, const uint64_t *row_ptr, const uint32_t *col,
                                       const uint8_t *alive, uint32_t *out, uint32_t *count) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    bool keep = false;
    uint32_t v = 0;
    if (i < n_heavy + n_light_nz) v = i < n_heavy ? heavy_rows[i] : light_rows[i - n_heavy];
    if (i < n_heavy + n_light_nz && (!alive || alive[v])) {
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            if (!alive || alive[col[e]]) {
                keep = true;
                break;
            }
        }
    }
    const uint64_t m = __ballot(keep);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__builtin_popcountll(m));
    base = __shfl(base, leader, 64);
    if (keep) out[base + __builtin_popcountll(m & ((1ull << lane) - 1ull))] = v;
}

int grid_for(uint64_t count, int threads, int cap) {
    uint64_t g = (count + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

}  // namespace

void launch_compact(hipStream_t st, const khc_graph *g, const uint8_t *alive, uint32_t *out, uint32_t *count) {
    const uint32_t rows = g->n_heavy + g->n_light_nz;
    hipLaunchKernelGGL(compact_sources_kernel, dim3(rows / 256 + 1), dim3(256), 0, st, g->heavy_rows, g->n_heavy,
                       g->light_rows, g->n_light_nz, g->row_ptr, g->col, alive, out, count);
}

namespace {

int check_csr_args(khc_ctx *ctx, const khc_csr *g) {
    if (!g) return set_error(ctx, KHC_EINVAL, "csr is null");
    if (g->n == 0xFFFFFFFFu) return set_error(ctx, KHC_EINVAL, "n must be below 2^32-1");
    if (!g->row_ptr) return set_error(ctx, KHC_EINVAL, "row_ptr is null");
    if (g->nnz > 0 && !g->col) return set_error(ctx, KHC_EINVAL, "col is null");
    return KHC_OK;
}

int validate_impl(khc_ctx *ctx, const khc_csr *g) {
    int rc = check_csr_args(ctx, g);
    if (rc) return rc;
    void *flags;
    if ((rc = ws_get(ctx, WS_FLAGS, 64, &flags))) return rc;
    uint32_t *f = (uint32_t *)flags;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, f, 0u, (uint64_t)1);
    hipLaunchKernelGGL(validate_rows_kernel, dim3(grid_for((uint64_t)g->n + 1, 256, 1 << 20)),
                       dim3(256), 0, st, g->n, g->nnz, g->row_ptr, f);
    uint32_t host = 0;
    hipError_t e = hipMemcpyAsync(&host, f, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "validate rows");
    if (!host && g->nnz) {
        hipLaunchKernelGGL(validate_arcs_kernel, dim3((unsigned)((g->nnz + 255) / 256)), dim3(256), 0,
                           st, g->n, g->nnz, g->row_ptr, g->col, f);
        e = hipMemcpyAsync(&host, f, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return check_hip(ctx, e, "validate arcs");
    }
    if (host) {
        std::string m = "CSR is not a simple undirected graph:";
        if (host & VBAD_OFFSETS) m += " bad row offsets (row_ptr[0] != 0, row_ptr[n] != nnz or decreasing);";
        if (host & VBAD_RANGE) m += " column id >= n;";
        if (host & VSELF_LOOP) m += " self-loop;";
        if (host & VUNSORTED) m += " row not strictly increasing (unsorted or duplicate arc);";
        if (host & VASYMMETRIC) m += " arc without its reverse;";
        return set_error(ctx, KHC_EGRAPH, m);
    }
    return KHC_OK;
}

template <typename T>
int upload(khc_ctx *ctx, const std::vector<T> &v, T **out) {
    size_t bytes = std::max<size_t>(v.size() * sizeof(T), 8);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(ctx, KHC_ENOMEM, "hipMalloc for graph schedule failed");
    }
    if (!v.empty()) {
        hipError_t e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return check_hip(ctx, e, "graph schedule upload");
        }
    }
    *out = (T *)p;
    return KHC_OK;
}

}  // namespace

int graph_create_impl(khc_ctx *ctx, const khc_csr *g, khc_graph **out, const std::vector<uint64_t> *vbase);

}  // namespace khc

using namespace khc;

extern "C" {

int khc_set_progress(khc_ctx *ctx, khc_progress_fn fn, void *user, uint32_t interval_ms) {
    if (!ctx) return KHC_EINVAL;
    ctx->progress_fn = fn;
    ctx->progress_user = user;
    ctx->progress_ms = interval_ms;
    return KHC_OK;
}

int khc_create(khc_ctx **out, int device, void *hip_stream) {
    if (!out) return KHC_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return KHC_EHIP;
    }
    if (device < 0 || device >= ndev) return KHC_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return KHC_EHIP;
    khc_ctx *c = new khc_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->bufs.resize(WS_NUM_SLOTS);
    // the device address of the static scratch of khdeg_compute_noalloc,
    // looked up once per device while it is current (a failure here only
    // disables that entry point, which then reports it)
    (void)noalloc_init(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        c->capture_stream = nullptr;
    }
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate_khz > 0)
        c->wall_clock_khz = (uint64_t)rate_khz;
    (void)hipGetLastError();
    if (hipHostMalloc((void **)&c->host_scalars, kHostScalarBytes, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return KHC_ENOMEM;
    }
    // progress of the persistent kernel, written by the device while it runs
    if (hipHostMalloc((void **)&c->persist_progress, 64, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess ||
        hipHostGetDevicePointer((void **)&c->persist_progress_dev, (void *)c->persist_progress, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (c->persist_progress) (void)hipHostFree((void *)c->persist_progress);
        (void)hipHostFree(c->host_scalars);
        delete c;
        return KHC_ENOMEM;
    }
    *out = c;
    return KHC_OK;
}

int khc_destroy(khc_ctx *ctx) {
    if (!ctx) return KHC_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    drop_persist_graphs(ctx, nullptr);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto &b : ctx->bufs)
        if (b.ptr) (void)hipFree(b.ptr);
    for (auto &r : ctx->prof_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto ev : ctx->prof_pool) (void)hipEventDestroy(ev);
    if (ctx->host_scalars) (void)hipHostFree(ctx->host_scalars);
    if (ctx->persist_progress) (void)hipHostFree((void *)ctx->persist_progress);
    delete ctx;
    return KHC_OK;
}

const char *khc_last_error(const khc_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

int khc_set_option(khc_ctx *ctx, int option, int64_t value) {
    if (!ctx) return KHC_EINVAL;
    switch (option) {
        case KHC_OPT_MAX_WIDTH:
            if (value < 1 || value > kMaxWidth || (value & (value - 1)))
                return set_error(ctx, KHC_EINVAL, "max width must be a power of two in [1, 32]");
            ctx->max_width = (int)value;
            return KHC_OK;
        case KHC_OPT_SCHEDULE:
            if (value < 0 || value > 3) return set_error(ctx, KHC_EINVAL, "schedule must be 0, 1, 2 or 3");
            ctx->schedule = (int)value;
            return KHC_OK;
        case KHC_OPT_WORKSPACE_LIMIT:
            if (value < 0) return set_error(ctx, KHC_EINVAL, "workspace limit must be >= 0");
            ctx->ws_limit = (uint64_t)value;
            return KHC_OK;
        case KHC_OPT_VALIDATE:
            ctx->validate = value ? 1 : 0;
            return KHC_OK;
        case KHC_OPT_WAVES_PER_CU:
            if (value < 4 || value > 32) return set_error(ctx, KHC_EINVAL, "waves per CU must be in [4, 32]");
            ctx->waves_per_cu = (int)value;
            return KHC_OK;
        case KHC_OPT_PROFILE:
            ctx->profile = value ? 1 : 0;
            return KHC_OK;
        case KHC_OPT_DRIVER:
            if (value != 0 && value != 1) return set_error(ctx, KHC_EINVAL, "driver must be 0 or 1");
            ctx->driver = (int)value;
            return KHC_OK;
        case KHC_OPT_PERSIST_WIDTH:
            if (value != 8 && value != 16 && value != 32)
                return set_error(ctx, KHC_EINVAL, "persistent width must be 8, 16 or 32 words");
            ctx->persist_width = (int)value;
            return KHC_OK;
        case KHC_OPT_BARRIER_TIMEOUT:
            if (value < 1 || value > 600) return set_error(ctx, KHC_EINVAL, "barrier timeout must be 1..600 s");
            ctx->barrier_timeout_s = (int)value;
            return KHC_OK;
        case KHC_OPT_PUSH_COST:
            if (value < 0 || value > 4096) return set_error(ctx, KHC_EINVAL, "push cost must be in [0, 4096]");
            ctx->push_cost = (int)value;
            return KHC_OK;
        case KHC_OPT_TUNE_REPEATS:
            if (value < 1 || value > 15) return set_error(ctx, KHC_EINVAL, "tune repeats must be in [1, 15]");
            ctx->tune_repeats = (int)value;
            return KHC_OK;
        case KHC_OPT_TUNE_CACHE:
            ctx->tune_cache_on = value ? 1 : 0;
            if (!value) ctx->tune_cache.clear();
            return KHC_OK;
        case KHC_OPT_ROUND_LIMIT:
            if (value < 0 || value > 0xFFFFFFFFll) return set_error(ctx, KHC_EINVAL, "round limit must be >= 0");
            ctx->round_limit = (uint32_t)value;
            return KHC_OK;
        default:
            return set_error(ctx, KHC_EINVAL, "unknown option " + std::to_string(option));
    }
}

int khc_profile_read(khc_ctx *ctx, khc_profile *out, int reset) {
    if (!ctx) return KHC_EINVAL;
    (void)hipSetDevice(ctx->device);
    for (auto &r : ctx->prof_pending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return check_hip(ctx, e, "profile event");
        ctx->prof_acc.launches[r.cls] += 1;
        ctx->prof_acc.ms[r.cls] += ms;
        ctx->prof_acc.bytes[r.cls] += r.bytes;
        ctx->prof_pool.push_back(r.a);
        ctx->prof_pool.push_back(r.b);
    }
    ctx->prof_pending.clear();
    if (out) {
        for (int c = 0; c < 4; ++c) {
            out->launches[c] += ctx->prof_acc.launches[c];
            out->ms[c] += ctx->prof_acc.ms[c];
            out->bytes[c] += ctx->prof_acc.bytes[c];
        }
    }
    if (reset) ctx->prof_acc = khc_profile{};
    return KHC_OK;
}

int khc_validate_csr(khc_ctx *ctx, const khc_csr *g) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return KHC_EHIP;
    (void)hipSetDevice(ctx->device);
    return validate_impl(ctx, g);
}

int khc_graph_create(khc_ctx *ctx, const khc_csr *g, khc_graph **out) {
    if (!ctx) return KHC_EINVAL;
    if (!out) return set_error(ctx, KHC_EINVAL, "out is null");
    *out = nullptr;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    (void)hipSetDevice(ctx->device);
    return graph_create_impl(ctx, g, out, nullptr);
}

}  // extern "C"

namespace khc {
namespace {

__global__ void graph_id_kernel(uint32_t n, uint32_t G, const uint64_t *vtx_base, uint32_t *gid) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = G;  // last g with vtx_base[g] <= v
        while (hi - lo > 1) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (vtx_base[mid] <= v) lo = mid; else hi = mid;
        }
        gid[v] = lo;
    }
}

// Local ids to global ids; an id outside its own graph sets flag bit 2.
__global__ void union_col_kernel(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                                 const uint32_t *gid, const uint64_t *vtx_base, uint32_t *out,
                                 uint32_t *flags) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t g = gid[v];
        const uint64_t base = vtx_base[g], ng = vtx_base[g + 1] - base;
        for (uint64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            const uint32_t c = col[e];
            if (c >= ng) {
                atomicOr(flags, 2u);
                out[e] = 0;
            } else {
                out[e] = (uint32_t)(base + c);
            }
        }
    }
}

}  // namespace
}  // namespace khc

extern "C" {

int khc_graph_create_batched(khc_ctx *ctx, uint32_t G, const uint64_t *vtx_base, const uint64_t *row_ptr,
                             const uint32_t *col, uint64_t nnz, khc_graph **out) {
    if (!ctx) return KHC_EINVAL;
    if (!out) return set_error(ctx, KHC_EINVAL, "out is null");
    *out = nullptr;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (G == 0 || !vtx_base || !row_ptr || (nnz && !col))
        return set_error(ctx, KHC_EINVAL, "batched graph: G == 0 or null pointer");
    (void)hipSetDevice(ctx->device);
    hipStream_t st = ctx->stream;
    std::vector<uint64_t> vb(G + 1);
    hipError_t e = hipMemcpyAsync(vb.data(), vtx_base, (G + 1) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "vtx_base download");
    if (vb[0] != 0) return set_error(ctx, KHC_EINVAL, "vtx_base[0] must be 0");
    for (uint32_t g = 0; g < G; ++g)
        if (vb[g + 1] < vb[g]) return set_error(ctx, KHC_EINVAL, "vtx_base must be non-decreasing");
    if (vb[G] >= 0xFFFFFFFFull) return set_error(ctx, KHC_EINVAL, "too many vertices in the batch");
    const uint32_t n = (uint32_t)vb[G];
    uint32_t *gid = nullptr, *ucol = nullptr, *flags = nullptr;
    uint64_t *vbd = nullptr;
    auto cleanup = [&]() {
        if (gid) (void)hipFree(gid);
        if (ucol) (void)hipFree(ucol);
        if (vbd) (void)hipFree(vbd);
    };
    if (hipMalloc(&gid, (size_t)n * 4 + 4) != hipSuccess || hipMalloc(&ucol, nnz * 4 + 4) != hipSuccess ||
        hipMalloc(&vbd, (G + 1) * 8) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return set_error(ctx, KHC_ENOMEM, "batched graph allocation failed");
    }
    int rc;
    void *fl;
    if ((rc = ws_get(ctx, WS_FLAGS, 64, &fl))) {
        cleanup();
        return rc;
    }
    flags = (uint32_t *)fl;
    e = hipMemcpyAsync(vbd, vtx_base, (G + 1) * 8, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
        cleanup();
        return check_hip(ctx, e, "vtx_base copy");
    }
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, flags, 0u, (uint64_t)1);
    const int grid = grid_for(n, 256, ctx->num_cu * 8);
    hipLaunchKernelGGL(graph_id_kernel, dim3(grid), dim3(256), 0, st, n, G, (const uint64_t *)vbd, gid);
    hipLaunchKernelGGL(union_col_kernel, dim3(grid), dim3(256), 0, st, n, row_ptr, col, gid,
                       (const uint64_t *)vbd, ucol, flags);
    uint32_t hf = 0;
    e = hipMemcpyAsync(&hf, flags, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        cleanup();
        return check_hip(ctx, e, "batched graph build");
    }
    if (hf & 2u) {
        cleanup();
        return set_error(ctx, KHC_EGRAPH, "batched graph: a column id lies outside its own graph");
    }
    khc_csr u{n, nnz, row_ptr, ucol};
    khc_graph *gr = nullptr;
    if ((rc = graph_create_impl(ctx, &u, &gr, &vb))) {
        cleanup();
        return rc;
    }
    gr->ngraphs = G;
    gr->gid = gid;
    gr->col_owned = ucol;
    gr->vtx_base = vbd;
    *out = gr;
    return KHC_OK;
}

int khcore_decompose_batched(khc_ctx *ctx, uint32_t G, const uint64_t *vtx_base, const uint64_t *row_ptr,
                             const uint32_t *col, uint64_t nnz, uint32_t h, uint32_t *core,
                             uint32_t *peel_round, khc_stats *stats) {
    khc_graph *g = nullptr;
    int rc = khc_graph_create_batched(ctx, G, vtx_base, row_ptr, col, nnz, &g);
    if (rc) return rc;
    rc = khcore_decompose(ctx, g, h, core, peel_round, stats);
    khc_graph_destroy(g);
    return rc;
}

}  // extern "C"

namespace khc {

void report_progress(khc_ctx *ctx, std::chrono::steady_clock::time_point *last, uint32_t rounds, uint64_t removed,
                     uint32_t level) {
    if (!ctx->progress_fn) return;
    const auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration<double, std::milli>(now - *last).count() < (double)ctx->progress_ms) return;
    *last = now;
    ctx->progress_fn(ctx->progress_user, rounds, removed, level);
}

int graph_create_impl(khc_ctx *ctx, const khc_csr *g, khc_graph **out, const std::vector<uint64_t> *vbase) {
    int rc = check_csr_args(ctx, g);
    if (rc) return rc;
    if (ctx->validate && (rc = validate_impl(ctx, g))) return rc;

    // Row schedule: light rows (<= kHeavyRowArcs arcs) by descending degree,
    // heavy rows by descending degree and cut into chunks.  Several graphs
    // packed together (vbase) are scheduled graph by graph, so the rows of
    // consecutive graphs form one range of each list.
    const uint32_t n = g->n;
    std::vector<uint64_t> rp(n + 1);
    hipError_t e = hipMemcpyAsync(rp.data(), g->row_ptr, (n + 1) * sizeof(uint64_t),
                                  hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return check_hip(ctx, e, "row_ptr download");
    if (rp[n] != g->nnz) return set_error(ctx, KHC_EGRAPH, "row_ptr[n] != nnz");
    const uint32_t G = vbase ? (uint32_t)(vbase->size() - 1) : 1u;
    auto deg = [&](uint32_t v) { return rp[v + 1] - rp[v]; };
    std::vector<uint32_t> light, heavy, chunk_heavy, chunk_first, light_first(G + 1, 0), gchunk_first(G + 1, 0);
    light.reserve(n);
    uint32_t maxdeg = 0;
    std::vector<uint32_t> bucket(kHeavyRowArcs + 2), start(kHeavyRowArcs + 2);
    for (uint32_t gi = 0; gi < G; ++gi) {
        const uint32_t v0 = vbase ? (uint32_t)(*vbase)[gi] : 0u, v1 = vbase ? (uint32_t)(*vbase)[gi + 1] : n;
        light_first[gi] = (uint32_t)light.size();
        gchunk_first[gi] = (uint32_t)chunk_heavy.size();
        std::fill(bucket.begin(), bucket.end(), 0u);
        const size_t heavy0 = heavy.size();
        for (uint32_t v = v0; v < v1; ++v) {
            const uint64_t d = deg(v);
            if (d > maxdeg) maxdeg = (uint32_t)std::min<uint64_t>(d, 0xFFFFFFFFu);
            if (d > kHeavyRowArcs) heavy.push_back(v);
            else bucket[kHeavyRowArcs - d]++;  // descending degree order
        }
        start[0] = (uint32_t)light.size();
        for (uint32_t i = 1; i < start.size(); ++i) start[i] = start[i - 1] + bucket[i - 1];
        light.resize(light.size() + (v1 - v0) - (heavy.size() - heavy0));
        for (uint32_t v = v0; v < v1; ++v) {
            const uint64_t d = deg(v);
            if (d <= kHeavyRowArcs) light[start[kHeavyRowArcs - d]++] = v;
        }
        std::sort(heavy.begin() + heavy0, heavy.end(), [&](uint32_t a, uint32_t b) {
            return deg(a) != deg(b) ? deg(a) > deg(b) : a < b;
        });
        for (size_t i = heavy0; i < heavy.size(); ++i) {
            const uint32_t nch = (uint32_t)((deg(heavy[i]) + kChunkArcs - 1) / kChunkArcs);
            chunk_first.push_back((uint32_t)chunk_heavy.size());
            for (uint32_t c = 0; c < nch; ++c) chunk_heavy.push_back((uint32_t)i);
        }
    }
    light_first[G] = (uint32_t)light.size();
    gchunk_first[G] = (uint32_t)chunk_heavy.size();
    chunk_first.push_back((uint32_t)chunk_heavy.size());

    khc_graph *gr = new khc_graph();
    gr->ctx = ctx;
    gr->n = n;
    gr->nnz = g->nnz;
    gr->row_ptr = g->row_ptr;
    gr->col = g->col;
    gr->n_light = (uint32_t)light.size();
    if (!vbase) {
        for (uint32_t v : light) {
            const uint64_t d = rp[v + 1] - rp[v];
            gr->n_light_mid += d > kMidDeg;
            gr->n_light_nz += d > 0;
        }
    } else {
        // not one descending-degree order: every light row on the one-lane path
        gr->n_light_mid = 0;
        gr->n_light_nz = gr->n_light;
    }
    gr->n_heavy = (uint32_t)heavy.size();
    gr->n_chunks = (uint32_t)chunk_heavy.size();
    gr->max_degree = maxdeg;
    if ((rc = upload(ctx, light, &gr->light_rows)) || (rc = upload(ctx, heavy, &gr->heavy_rows)) ||
        (rc = upload(ctx, chunk_heavy, &gr->chunk_heavy)) ||
        (rc = upload(ctx, chunk_first, &gr->chunk_first)) ||
        (vbase && ((rc = upload(ctx, light_first, &gr->light_first)) ||
                   (rc = upload(ctx, gchunk_first, &gr->graph_chunk_first))))) {
        khc_graph_destroy(gr);
        return rc;
    }
    *out = gr;
    return KHC_OK;
}

}  // namespace khc

extern "C" {

int khc_graph_destroy(khc_graph *g) {
    if (!g) return KHC_EINVAL;
    if (g->ctx) {
        (void)hipStreamSynchronize(g->ctx->stream);
        drop_persist_graphs(g->ctx, g);
    }
    if (g->gid) (void)hipFree(g->gid);
    if (g->col_owned) (void)hipFree(g->col_owned);
    if (g->vtx_base) (void)hipFree(g->vtx_base);
    if (g->light_rows) (void)hipFree(g->light_rows);
    if (g->heavy_rows) (void)hipFree(g->heavy_rows);
    if (g->chunk_heavy) (void)hipFree(g->chunk_heavy);
    if (g->chunk_first) (void)hipFree(g->chunk_first);
    if (g->light_first) (void)hipFree(g->light_first);
    if (g->graph_chunk_first) (void)hipFree(g->graph_chunk_first);
    delete g;
    return KHC_OK;
}

}  // extern "C"

namespace khc {
int compact_sources(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t **srcs_out,
                    uint32_t *count) {
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    int rc;
    void *srcs, *cnt;
    if ((rc = ws_get(ctx, WS_SRCS, (size_t)n * 4 + 4, &srcs)) || (rc = ws_get(ctx, WS_FLAGS, 64, &cnt)))
        return rc;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, (uint32_t *)cnt, 0u, (uint64_t)1);
    launch_compact(st, g, alive, (uint32_t *)srcs, (uint32_t *)cnt);
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, cnt, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "source compaction");
    *srcs_out = (uint32_t *)srcs;
    *count = ctx->host_scalars[0];
    return KHC_OK;
}

void fill_u32(khc_ctx *ctx, uint32_t *p, uint32_t value, uint64_t count) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(count, 256, 4096)), dim3(256), 0, ctx->stream, p, value,
                       count);
}
}  // namespace khc

extern "C" {

int khdeg_compute(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                  uint32_t *deg) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !deg) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h == 0) return set_error(ctx, KHC_EINVAL, "h must be >= 1");
    (void)hipSetDevice(ctx->device);
    return khc::khdeg_compute_impl(ctx, g, alive, h, deg, nullptr, 0);
}

}  // extern "C"

namespace khc {

int khdeg_compute_impl(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h, uint32_t *deg,
                       Arena *arena, int arena_width) {
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    if (n == 0) return KHC_OK;
    int rc;
    void *srcs, *cnt;
    if (arena) {
        srcs = arena->take((size_t)n * 4);
        cnt = arena->take(64);
        if (!srcs || !cnt) return set_error(ctx, KHC_ENOMEM, "source list exceeds the caller's scratch region");
    } else if ((rc = ws_get(ctx, WS_SRCS, (size_t)n * 4, &srcs)) || (rc = ws_get(ctx, WS_FLAGS, 64, &cnt))) {
        return rc;
    }
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, deg, 0u,
                       (uint64_t)n);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, (uint32_t *)cnt, 0u, (uint64_t)1);
    launch_compact(st, g, alive, (uint32_t *)srcs, (uint32_t *)cnt);
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, cnt, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "source compaction");
    const uint32_t nsrc = ctx->host_scalars[0];
    return msbfs_degrees(ctx, g, alive, h, (const uint32_t *)srcs, nsrc, nullptr, 1, deg, arena, arena_width);
}

}  // namespace khc

extern "C" {

int khdeg_scanned_arcs(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                       uint64_t *te) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || !te) return set_error(ctx, KHC_EINVAL, "graph or output is null");
    if (h == 0) return set_error(ctx, KHC_EINVAL, "h must be >= 1");
    (void)hipSetDevice(ctx->device);
    hipStream_t st = ctx->stream;
    const uint32_t n = g->n;
    if (n == 0) return KHC_OK;
    int rc;
    void *srcs, *cnt;
    if ((rc = ws_get(ctx, WS_SRCS, (size_t)n * 4, &srcs)) || (rc = ws_get(ctx, WS_FLAGS, 64, &cnt)))
        return rc;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for((uint64_t)n * 2, 256, 4096)), dim3(256), 0, st,
                       (uint32_t *)te, 0u, (uint64_t)n * 2);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, (uint32_t *)cnt, 0u, (uint64_t)1);
    launch_compact(st, g, alive, (uint32_t *)srcs, (uint32_t *)cnt);
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, cnt, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "source compaction");
    return msbfs_scanned_arcs(ctx, g, alive, h, (const uint32_t *)srcs, ctx->host_scalars[0], te);
}

int khdeg_compute_list(khc_ctx *ctx, const khc_graph *g, const uint8_t *alive, uint32_t h,
                       const uint32_t *verts, uint32_t count, uint32_t *deg) {
    if (!ctx) return KHC_EINVAL;
    if (ctx->sticky) return set_error(ctx, KHC_EHIP, "context has a sticky HIP error");
    if (!g || (count && (!verts || !deg))) return set_error(ctx, KHC_EINVAL, "null argument");
    if (h == 0) return set_error(ctx, KHC_EINVAL, "h must be >= 1");
    if (count == 0) return KHC_OK;
    (void)hipSetDevice(ctx->device);
    // ids are read on the device: check the range before any kernel uses them
    int rc;
    void *flags;
    if ((rc = ws_get(ctx, WS_FLAGS, 64, &flags))) return rc;
    hipStream_t st = ctx->stream;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, (uint32_t *)flags, 0u, (uint64_t)1);
    hipLaunchKernelGGL(check_ids_kernel, dim3(grid_for(count, 256, 1024)), dim3(256), 0, st, verts, count, g->n,
                       (uint32_t *)flags);
    hipError_t e = hipMemcpyAsync(ctx->host_scalars, flags, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return check_hip(ctx, e, "vertex id check");
    if (ctx->host_scalars[0]) return set_error(ctx, KHC_EINVAL, "a listed vertex id is >= n");
    return msbfs_degrees(ctx, g, alive, h, verts, count, deg, 0, nullptr);
}

}  // extern "C"
