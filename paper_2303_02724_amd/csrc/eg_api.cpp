// eg_api.cpp -- the C ABI: argument checks, workspace carving and the kernel
// sequence on the caller's stream.  Nothing here allocates or synchronises.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "eg_internal.h"

using namespace eg;

namespace {

constexpr int64_t kMaxIndex = (int64_t(1) << 31) - 1;

bool grid_from(int ndim, const int64_t* dims, Grid* g)
{
    if (ndim < 1 || ndim > EG_MAX_NDIM || !dims) return false;
    std::memset(g, 0, sizeof(*g));
    g->ndim = ndim;
    int64_t N = 1;
    for (int i = 0; i < ndim; ++i) {
        if (dims[i] < 1) return false;
        if (dims[i] > kMaxIndex) return false;
        N *= dims[i];
        if (N > kMaxIndex) return false;
        g->dims[i] = (int32_t)dims[i];
    }
    g->N = (int32_t)N;
    return true;
}

bool caps_ok(int64_t cap_max, int64_t cap_sad, int64_t cap_arc)
{
    auto ok = [](int64_t c) { return c >= 0 && c < kMaxIndex; };
    return ok(cap_max) && ok(cap_sad) && ok(cap_arc);
}

eg_status too_large_or_arg(int ndim, const int64_t* dims)
{
    if (ndim < 1 || ndim > EG_MAX_NDIM || !dims) return EG_ERR_ARG;
    // distinguish an oversized grid from a malformed one
    long double N = 1;
    for (int i = 0; i < ndim; ++i) {
        if (dims[i] < 1) return EG_ERR_ARG;
        N *= (long double)dims[i];
    }
    return N > (long double)kMaxIndex ? EG_ERR_TOO_LARGE : EG_ERR_ARG;
}

// Validate one field's arguments; fill g and w.
eg_status check_one(const float* field, int ndim, const int64_t* dims, const eg_out* o, Grid* g, Work* w)
{
    if (!o || !field) return EG_ERR_ARG;
    Tuning tu;
    if (!decode_tuning(o->tuning, &tu)) return EG_ERR_ARG;
    if (!grid_from(ndim, dims, g)) return too_large_or_arg(ndim, dims);
    if (o->flags & ~uint32_t(EG_MINIMA)) return EG_ERR_ARG;
    if (!caps_ok(o->cap_max, o->cap_sad, o->cap_arc)) return EG_ERR_TOO_LARGE;
    if (!o->labels || !o->header || !o->arc_offsets) return EG_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(o->labels) & 15u) return EG_ERR_ARG;
    if ((o->cap_max > 0 && !o->maxima) || (o->cap_sad > 0 && !o->saddles) || (o->cap_arc > 0 && !o->arc_maxima))
        return EG_ERR_ARG;
    const int64_t X = g->dims[g->ndim - 1];
    const Work need = carve(nullptr, g->ndim, g->N, X, o->cap_sad, tu.exit_cap);
    if (!o->workspace || (reinterpret_cast<uintptr_t>(o->workspace) & 255u) || o->ws_bytes < need.bytes)
        return EG_ERR_WORKSPACE;
    *w = carve(o->workspace, g->ndim, g->N, X, o->cap_sad, tu.exit_cap);
    return EG_OK;
}

// Stage (a) + (c): pointers, maxima and saddle candidates (resets counters).
hipError_t stage_classify(const float* field, const Grid& g, const LinkTable& t, const eg_out& o, const Work& w,
                          const Tuning& tu, hipStream_t s)
{
    const bool minima = (o.flags & EG_MINIMA) != 0;
    hipError_t e = launch_init(w.ctr, o.header, s);
    if (e != hipSuccess) return e;
    return launch_classify(field, g, t, minima, o.labels, o.ptr, w, tu, s);
}

// Stage (b): labels by pointer jumping, in place.
hipError_t stage_label(const Grid& g, const eg_out& o, const Work& w, const Tuning& tu, hipStream_t s)
{
    return launch_labels(g, o.labels, w, tu, s);
}

// Stage (d) and the canonical outputs: ascending maxima and saddles, the
// arcs of every saddle as a CSR, and the header (which also reports labels
// left unresolved by the last label pass).
hipError_t stage_arcs(const float* field, const Grid& g, const eg_out& o, const Work& w, const Tuning& tu,
                      hipStream_t s)
{
    ArcArgs a = arc_args(field, g, o, w);
    a.last_flag = gptr<const uint32_t>(w.ctr + C_FINAL + tu.passes - 1);
    return launch_arcs(a, s);
}

enum Stage { S_CLASSIFY = 1, S_LABEL = 2, S_ARCS = 4, S_ALL = 7 };

eg_status run_stages(int stages, const float* field, int ndim, const int64_t* dims, void* stream,
                     const eg_out* out)
{
    Grid g;
    Work w;
    const eg_status st = check_one(field, ndim, dims, out, &g, &w);
    if (st != EG_OK) return st;
    LinkTable t;
    make_table(g, &t);
    Tuning tu;
    decode_tuning(out->tuning, &tu);
    tu.passes = passes_for(tu, g.N);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (stages & S_CLASSIFY) e = stage_classify(field, g, t, *out, w, tu, s);
    if (e == hipSuccess && (stages & S_LABEL)) e = stage_label(g, *out, w, tu, s);
    if (e == hipSuccess && (stages & S_ARCS)) e = stage_arcs(field, g, *out, w, tu, s);
    return e == hipSuccess ? EG_OK : EG_ERR_HIP;
}

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct BatchLayout {
    size_t o_plan, o_fields, o_bctr, bytes, plan_bytes;
};

BatchLayout batch_layout(int count)
{
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t at = off;
        off = align_up(off + n);
        return at;
    };
    L.o_plan = take(sizeof(BatchPlan));
    L.o_fields = take(sizeof(BatchField) * (size_t)count);
    L.plan_bytes = off;
    L.o_bctr = take(sizeof(uint32_t) * C_SLOTS);
    L.bytes = off;
    return L;
}

eg_status batch_check(int count, const int* ndims, const int64_t* dims, const eg_out* outs)
{
    if (count < 1 || !ndims || !dims || !outs) return EG_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        Grid g;
        if (ndims[i] != 2 && ndims[i] != 3) return EG_ERR_ARG;
        if (!grid_from(ndims[i], dims + (size_t)i * EG_MAX_NDIM, &g))
            return too_large_or_arg(ndims[i], dims + (size_t)i * EG_MAX_NDIM);
        const eg_out& o = outs[i];
        if (!caps_ok(o.cap_max, o.cap_sad, o.cap_arc)) return EG_ERR_TOO_LARGE;
    }
    return EG_OK;
}

}  // namespace

// ------------------------------------------------------------------ scratch

// The workspace of eg_build_noalloc: one file-scope device array, so that the
// entry point never allocates.  Each device that runs the library holds its
// own copy until the process ends.  In host code `scratch` is only a handle:
// its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is ever passed to kernels.
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of the current device's scratch array, or nullptr.
void* scratch_address()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    void* p = g_scratch[dev].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
        void* q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return nullptr;
        g_scratch[dev].store(q, std::memory_order_release);
        p = q;
    }
    return p;
}

}  // namespace

extern "C" {

size_t eg_batch_plan_bytes(int count)
{
    if (count < 1) return 0;
    return batch_layout(count).plan_bytes;
}

size_t eg_batch_workspace_bytes(int count, const int* ndims, const int64_t* dims, const eg_out* outs)
{
    if (batch_check(count, ndims, dims, outs) != EG_OK) return 0;
    return batch_layout(count).bytes;
}

eg_status eg_batch_plan(int count, const float* const* fields, const int* ndims, const int64_t* dims,
                        const eg_out* outs, void* batch_ws, size_t batch_ws_bytes, void* host_plan,
                        size_t host_plan_bytes)
{
    eg_status st = batch_check(count, ndims, dims, outs);
    if (st != EG_OK) return st;
    if (!fields || !host_plan) return EG_ERR_ARG;
    const BatchLayout L = batch_layout(count);
    if (host_plan_bytes < L.plan_bytes) return EG_ERR_ARG;
    if (!batch_ws || (reinterpret_cast<uintptr_t>(batch_ws) & 255u) || batch_ws_bytes < L.bytes)
        return EG_ERR_WORKSPACE;
    char* dbase = (char*)batch_ws;
    std::memset(host_plan, 0, L.plan_bytes);
    BatchPlan* P = (BatchPlan*)host_plan;
    BatchField* F = (BatchField*)((char*)host_plan + L.o_fields);
    P->count = count;
    if (!decode_tuning(outs[0].tuning, &P->tuning)) return EG_ERR_ARG;
    P->bctr = gptr((uint32_t*)(dbase + L.o_bctr));
    P->fields = gptr((BatchField*)(dbase + L.o_fields));
    P->dev = (const BatchPlan*)(dbase + L.o_plan);
    P->plan_bytes = (int64_t)L.plan_bytes;
    // plan order: by class (2D max, 2D min, 3D max, 3D min), stable
    std::vector<int> order;
    order.reserve(count);
    for (int c = 0; c < 4; ++c) {
        P->class_field[c] = (int32_t)order.size();
        for (int i = 0; i < count; ++i) {
            const int ci = (ndims[i] == 3 ? 2 : 0) + ((outs[i].flags & EG_MINIMA) ? 1 : 0);
            if (ci == c) order.push_back(i);
        }
    }
    P->class_field[4] = count;
    int64_t tiles = 0, arc_blocks_total = 0;
    int cls = 0;
    for (int k = 0; k < count; ++k) {
        while (cls < 4 && P->class_field[cls + 1] <= k) {
            P->class_tile[cls + 1] = tiles;
            ++cls;
        }
        const int i = order[k];
        Grid g;
        Work w;
        const eg_out& o = outs[i];
        st = check_one(fields[i], ndims[i], dims + (size_t)i * EG_MAX_NDIM, &o, &g, &w);
        if (st != EG_OK) return st;
        int ty, tz;
        tile_shape(P->tuning, g.ndim, &ty, &tz);
        BatchField& B = F[k];
        B.ta = tile_args(fields[i], g, o.labels, o.ptr, w, ty, tz);
        B.arc = arc_args(fields[i], g, o, w);
        B.ndim = g.ndim;
        B.minima = (o.flags & EG_MINIMA) ? 1 : 0;
        B.N = g.N;
        B.tile_base = tiles;
        B.arc_base = arc_blocks_total;
        B.exres = gptr(w.exres);
        tiles += B.ta.ntiles;
        arc_blocks_total += B.arc.arc_blocks;
    }
    while (cls < 4) {
        P->class_tile[cls + 1] = tiles;
        ++cls;
    }
    P->class_tile[0] = 0;
    int64_t max_n = 1;
    for (int i = 0; i < count; ++i) max_n = std::max<int64_t>(max_n, F[i].N);
    P->tuning.passes = passes_for(P->tuning, max_n);
    for (int k = 0; k < count; ++k)
        F[k].arc.last_flag = gptr<const uint32_t>((const uint32_t*)P->bctr + C_FINAL + P->tuning.passes - 1);
    P->total_tiles = tiles;
    P->total_arc_blocks = arc_blocks_total;
    return EG_OK;
}

eg_status eg_build_batched(const void* host_plan, void* stream)
{
    if (!host_plan) return EG_ERR_ARG;
    const BatchPlan& P = *(const BatchPlan*)host_plan;
    if (P.count < 1 || !P.dev) return EG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_batched_init(P.dev, P, s);
    if (e == hipSuccess) e = launch_classify_batched(P.dev, P, s);
    if (e == hipSuccess) e = launch_batched_rest(P.dev, P, s);
    return e == hipSuccess ? EG_OK : EG_ERR_HIP;
}

eg_status eg_paths(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out,
                   const eg_paths_out* paths)
{
    Grid g;
    Work w;
    const eg_status st = check_one(field, ndim, dims, out, &g, &w);
    if (st != EG_OK) return st;
    if (!paths || !out->ptr || !paths->pair_offsets || !paths->path_offsets || !paths->header) return EG_ERR_ARG;
    if (paths->cap_paths < 0 || paths->cap_vertices < 0) return EG_ERR_TOO_LARGE;
    if (paths->cap_paths >= kMaxIndex || paths->cap_vertices >= kMaxIndex) return EG_ERR_TOO_LARGE;
    if (paths->cap_vertices > 0 && !paths->path_vertices) return EG_ERR_ARG;
    PathArgs p{};
    p.ptr = gptr<const int32_t>(out->ptr);
    p.pair_offsets = gptr(paths->pair_offsets);
    p.path_offsets = gptr(paths->path_offsets);
    p.vertices = gptr(paths->path_vertices);
    p.header = gptr(paths->header);
    p.cap_paths = (uint32_t)paths->cap_paths;
    p.cap_vertices = (uint32_t)paths->cap_vertices;
    const hipError_t e = launch_paths(arc_args(field, g, *out, w), p, (hipStream_t)stream);
    return e == hipSuccess ? EG_OK : EG_ERR_HIP;
}

size_t eg_workspace_bytes(int ndim, const int64_t* dims, int64_t cap_sad)
{
    Grid g;
    if (!grid_from(ndim, dims, &g)) return 0;
    if (!caps_ok(0, cap_sad, 0)) return 0;
    return carve(nullptr, ndim, g.N, g.dims[ndim - 1], cap_sad).bytes;
}

eg_status eg_build(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out)
{
    return run_stages(S_ALL, field, ndim, dims, stream, out);
}

eg_status eg_build_noalloc(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out)
{
    if (!out) return EG_ERR_ARG;
    Grid g;
    if (!grid_from(ndim, dims, &g)) return too_large_or_arg(ndim, dims);
    if (!caps_ok(out->cap_max, out->cap_sad, out->cap_arc)) return EG_ERR_TOO_LARGE;
    Tuning tu;
    if (!decode_tuning(out->tuning, &tu)) return EG_ERR_ARG;
    const Work need = carve(nullptr, g.ndim, g.N, g.dims[g.ndim - 1], out->cap_sad, tu.exit_cap);
    if (need.bytes > kScratchBytes) return EG_ERR_SCRATCH;
    void* ws = scratch_address();
    if (!ws) return EG_ERR_HIP;
    eg_out o = *out;
    o.workspace = ws;
    o.ws_bytes = kScratchBytes;
    return run_stages(S_ALL, field, ndim, dims, stream, &o);
}

size_t eg_noalloc_scratch_bytes(void) { return kScratchBytes; }

eg_status eg_build_streamed(const float* host_field, float* dev_field, int ndim, const int64_t* dims,
                            int64_t slab_planes, void* stream, void* copy_stream, void* const* events,
                            int64_t nevents, const eg_out* out)
{
    if (!host_field || !dev_field || !events || slab_planes < 1) return EG_ERR_ARG;
    if (ndim != 2 && ndim != 3) return EG_ERR_ARG;
    Grid g;
    Work w;
    const eg_status st = check_one(dev_field, ndim, dims, out, &g, &w);
    if (st != EG_OK) return st;
    Tuning tu;
    decode_tuning(out->tuning, &tu);
    tu.passes = passes_for(tu, g.N);
    int ty, tz;
    tile_shape(tu, ndim, &ty, &tz);
    // slabs are whole tile rows along axis 0 (the slowest)
    const int64_t depth = ndim == 3 ? tz : ty;
    const int64_t D0 = g.dims[0];
    const int64_t plane = (int64_t)g.N / D0;
    const int64_t slab = (slab_planes + depth - 1) / depth * depth;
    const int64_t nslabs = (D0 + slab - 1) / slab;
    const int64_t rows = (D0 + depth - 1) / depth;
    if (nevents < nslabs + 1) return EG_ERR_ARG;
    for (int64_t k = 0; k <= nslabs; ++k)
        if (!events[k]) return EG_ERR_ARG;
    const TileArgs ta = tile_args(dev_field, g, out->labels, out->ptr, w, ty, tz);
    const int64_t tiles_per_row = (int64_t)ta.tiles_x * (ndim == 3 ? ta.tiles_y : 1);
    hipStream_t s = (hipStream_t)stream, cs = (hipStream_t)copy_stream;
    // the copies overwrite dev_field: they wait for the work already queued
    // on the compute stream (an earlier build may still read it)
    if (hipEventRecord((hipEvent_t)events[nslabs], s) != hipSuccess) return EG_ERR_HIP;
    if (hipStreamWaitEvent(cs, (hipEvent_t)events[nslabs], 0) != hipSuccess) return EG_ERR_HIP;
    // every copy first, each slab followed by its event, so the copy engine
    // streams while the compute stream classifies the slabs that have landed
    for (int64_t k = 0; k < nslabs; ++k) {
        const int64_t p0 = k * slab, p1 = std::min(D0, p0 + slab);
        if (hipMemcpyAsync(dev_field + p0 * plane, host_field + p0 * plane, (size_t)((p1 - p0) * plane) * sizeof(float),
                           hipMemcpyHostToDevice, cs) != hipSuccess)
            return EG_ERR_HIP;
        if (hipEventRecord((hipEvent_t)events[k], cs) != hipSuccess) return EG_ERR_HIP;
    }
    const bool minima = (out->flags & EG_MINIMA) != 0;
    hipError_t e = launch_init(w.ctr, out->header, s);
    for (int64_t k = 0; k < nslabs && e == hipSuccess; ++k) {
        // the tiles of slab k read one plane past it: wait for the next slab too
        e = hipStreamWaitEvent(s, (hipEvent_t)events[std::min(k + 1, nslabs - 1)], 0);
        const int64_t r0 = k * slab / depth, r1 = std::min(rows, (k + 1) * slab / depth);
        if (e == hipSuccess)
            e = launch_classify_tiled(dev_field, g, minima, out->labels, out->ptr, w, tu, s, r0 * tiles_per_row,
                                      (r1 - r0) * tiles_per_row);
    }
    if (e == hipSuccess) e = stage_label(g, *out, w, tu, s);
    if (e == hipSuccess) e = stage_arcs(dev_field, g, *out, w, tu, s);
    return e == hipSuccess ? EG_OK : EG_ERR_HIP;
}

eg_status eg_classify(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out)
{
    return run_stages(S_CLASSIFY, field, ndim, dims, stream, out);
}

eg_status eg_label(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out)
{
    return run_stages(S_LABEL, field, ndim, dims, stream, out);
}

eg_status eg_arcs(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out)
{
    return run_stages(S_ARCS, field, ndim, dims, stream, out);
}

const char* eg_status_string(int status)
{
    switch (status) {
        case EG_OK: return "ok";
        case EG_ERR_ARG: return "invalid argument";
        case EG_ERR_TOO_LARGE: return "grid or capacity too large (2^31 limit)";
        case EG_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case EG_ERR_NAN: return "field contains NaN";
        case EG_ERR_CAPACITY: return "output capacity too small (header holds required counts)";
        case EG_ERR_HIP: return "HIP launch failed";
        case EG_ERR_SCRATCH: return "field needs more workspace than eg_build_noalloc's fixed scratch holds";
        case EG_ERR_UNRESOLVED: return "labels left unresolved by the last label pass (internal error)";
        default: return "unknown status";
    }
}

int eg_link_table(int ndim, int8_t* offsets, uint64_t* adjacency)
{
    int8_t off[kMaxNb][EG_MAX_NDIM];
    uint64_t adj[kMaxNb * 2];
    const int k = make_rows(ndim, off, adj);
    if (k < 0) return -1;
    const int W = (k + 63) / 64;
    for (int j = 0; j < k; ++j) {
        if (offsets)
            for (int i = 0; i < ndim; ++i) offsets[j * ndim + i] = off[j][i];
        if (adjacency)
            for (int w = 0; w < W; ++w) adjacency[j * W + w] = adj[j * W + w];
    }
    return k;
}

}  // extern "C"
