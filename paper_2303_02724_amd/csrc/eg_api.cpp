// eg_api.cpp -- the C ABI: argument checks, workspace carving and the kernel
// sequence on the caller's stream.  Nothing here allocates or synchronises.
#include <cstring>

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

bool caps_ok(int64_t cap_max, int64_t cap_sad, int64_t cap_pairs, int64_t cap_arc)
{
    auto ok = [](int64_t c) { return c >= 0 && c < kMaxIndex; };
    return ok(cap_max) && ok(cap_sad) && ok(cap_pairs) && ok(cap_arc) && cap_pairs + cap_sad < kMaxIndex;
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

// Validate one field's arguments; fill g and t.
eg_status check_one(const float* field, int ndim, const int64_t* dims, const eg_out* o, Grid* g, Work* w)
{
    if (!o || !field) return EG_ERR_ARG;
    if (!grid_from(ndim, dims, g)) return too_large_or_arg(ndim, dims);
    if (o->flags & ~uint32_t(EG_MINIMA)) return EG_ERR_ARG;
    if (!caps_ok(o->cap_max, o->cap_sad, o->cap_pairs, o->cap_arc)) return EG_ERR_TOO_LARGE;
    if (!o->labels || !o->header || !o->arc_offsets) return EG_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(o->labels) & 15u) return EG_ERR_ARG;
    if ((o->cap_max > 0 && !o->maxima) || (o->cap_sad > 0 && !o->saddles) || (o->cap_arc > 0 && !o->arc_maxima))
        return EG_ERR_ARG;
    const Work need = carve(nullptr, o->cap_max, o->cap_sad, o->cap_pairs);
    if (!o->workspace || (reinterpret_cast<uintptr_t>(o->workspace) & 255u) || o->ws_bytes < need.bytes)
        return EG_ERR_WORKSPACE;
    *w = carve(o->workspace, o->cap_max, o->cap_sad, o->cap_pairs);
    return EG_OK;
}

// Stage (a) + (c): pointers, maxima and saddle candidates (resets counters).
hipError_t stage_classify(const float* field, const Grid& g, const LinkTable& t, const eg_out& o, const Work& w,
                          hipStream_t s)
{
    const bool minima = (o.flags & EG_MINIMA) != 0;
    hipError_t e = launch_init(w.ctr, o.header, s);
    if (e != hipSuccess) return e;
    return launch_classify(field, g, t, minima, o.labels, o.ptr, w, o.cap_max, o.cap_sad, s);
}

// Stage (b): labels by pointer jumping, in place.
hipError_t stage_label(const Grid& g, const eg_out& o, const Work& w, hipStream_t s)
{
    return launch_jump(o.labels, g.N, w.ctr, s);
}

// Stage (d) and the canonical outputs: ascending maxima; reps -> (saddle,
// maximum) keys -> radix sort -> unique -> CSR; the header.
hipError_t stage_arcs(const float* field, const Grid& g, const LinkTable& t, const eg_out& o, const Work& w,
                      hipStream_t s)
{
    const bool minima = (o.flags & EG_MINIMA) != 0;
    const int b = id_bits(g.N);
    hipError_t e;
    if ((e = launch_load_maxima(w, o.cap_max, s)) != hipSuccess) return e;
    if ((e = launch_sort(w.keysA, w.keysB, &w.ctr[C_NMAX], o.cap_max, b, w.hist, o.maxima, nullptr, s)) !=
        hipSuccess)
        return e;
    if ((e = launch_reps(field, g, t, minima, o.labels, w, o.cap_sad, b, s)) != hipSuccess) return e;
    uint64_t* sorted = nullptr;
    if ((e = launch_sort(w.keysA, w.keysB, &w.ctr[C_NKEYS], w.cap_keys, 2 * b + 1, w.hist, nullptr, &sorted, s)) !=
        hipSuccess)
        return e;
    if ((e = launch_csr(sorted, w, b, o, s)) != hipSuccess) return e;
    return launch_finalize(w, o, s);
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
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (stages & S_CLASSIFY) e = stage_classify(field, g, t, *out, w, s);
    if (e == hipSuccess && (stages & S_LABEL)) e = stage_label(g, *out, w, s);
    if (e == hipSuccess && (stages & S_ARCS)) e = stage_arcs(field, g, t, *out, w, s);
    return e == hipSuccess ? EG_OK : EG_ERR_HIP;
}

}  // namespace

extern "C" {

size_t eg_workspace_bytes(int ndim, const int64_t* dims, int64_t cap_max, int64_t cap_sad, int64_t cap_pairs)
{
    Grid g;
    if (!grid_from(ndim, dims, &g)) return 0;
    if (!caps_ok(cap_max, cap_sad, cap_pairs, 0)) return 0;
    return carve(nullptr, cap_max, cap_sad, cap_pairs).bytes;
}

eg_status eg_build(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out)
{
    return run_stages(S_ALL, field, ndim, dims, stream, out);
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
        default: return "unknown status";
    }
}

int eg_link_table(int ndim, int8_t* offsets, uint64_t* adjacency)
{
    int8_t off[kMaxNb][EG_MAX_NDIM];
    uint64_t adj[kMaxNb];
    const int k = make_rows(ndim, off, adj);
    if (k < 0) return -1;
    for (int j = 0; j < k; ++j) {
        if (offsets)
            for (int i = 0; i < ndim; ++i) offsets[j * ndim + i] = off[j][i];
        if (adjacency) adjacency[j] = adj[j];
    }
    return k;
}

}  // extern "C"
