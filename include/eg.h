/*
 * eg.h -- C ABI of the MI355X extremum-graph library (libeg_hip.so).
 *
 * Computes the extremum graph of a piecewise-linear scalar field sampled on an
 * n-dimensional grid (n = 1..6; float32 samples, other sample types through
 * eg_order_field), following Ande, Subhash and Natarajan,
 * "TACHYON: Efficient Shared Memory Parallel Computation of Extremum Graphs":
 *
 *   - grid vertices are the integer points of the box dims[0] x ... x dims[n-1],
 *     stored in row-major (C) order: dims[0] is the slowest axis and the linear
 *     index of a vertex is its array index (Sec. 3.2, Sec. 4);
 *   - the grid is split by the Freudenthal tessellation: two vertices are
 *     adjacent iff their coordinate difference is nonzero with every component
 *     in {0,1}, or every component in {0,-1} (Alg. 1), giving 2(2^n - 1)
 *     neighbours; vertices outside the box are absent (the link is truncated);
 *   - ties are broken by simulated perturbation (Sec. 3.3): u is below v iff
 *     f[u] < f[v], or f[u] == f[v] and u < v.  IEEE comparison (-0 == +0);
 *     infinities are ordered normally; NaN is an error;
 *   - a vertex is a maximum iff its upper link is empty and an (n-1)-saddle iff
 *     its upper link has at least two connected components (Table 1);
 *   - the steepest-ascent pointer of a vertex is the highest vertex of its
 *     upper link, or the vertex itself at a maximum (Sec. 3.3);
 *   - the label of a vertex is the maximum at the end of its steepest-ascent
 *     path: the descending manifold containing it (Sec. 2, Alg. 2);
 *   - for each saddle s and each upper-link component, the path from the
 *     component's highest vertex ends at a maximum m; the arcs (s, m) form a
 *     set (Sec. 2, Sec. 3.4 Alg. 2, UpperLinkRep).
 *
 * With EG_MINIMA the same is computed for the reversed order (u below v iff v
 * is below u in the order above): the minimum graph, whose "maxima" are the
 * minima of f and whose saddles are its 1-saddles (Sec. 2, Sec. 5).
 *
 * Conventions shared by every entry point:
 *   - every buffer named "device" is HIP device memory owned by the caller;
 *     the library never allocates, frees or synchronises; all work is queued
 *     on the caller's stream (a hipStream_t passed as void*, NULL = default);
 *   - argument errors are detected on the host and returned synchronously,
 *     before anything is queued;
 *   - data-dependent conditions (NaN in the field, an output buffer that is
 *     too small) are written to the device header (EG_H_* slots) together
 *     with the counts that a retry needs; read it after synchronising.
 */
#ifndef EG_H
#define EG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum eg_status {
    EG_OK = 0,
    EG_ERR_ARG = 1,       /* host: bad ndim, dims, flags, a NULL buffer, or labels not 16-byte aligned */
    EG_ERR_TOO_LARGE = 2, /* host: N >= 2^31 vertices, or a capacity >= 2^31 */
    EG_ERR_WORKSPACE = 3, /* host: workspace NULL, misaligned or smaller than eg_workspace_bytes */
    EG_ERR_NAN = 4,       /* device header: the field holds a NaN (outputs undefined) */
    EG_ERR_CAPACITY = 5,  /* device header: an output capacity was too small; counts are the required sizes */
    EG_ERR_HIP = 6,       /* host: a HIP launch failed */
    EG_ERR_SCRATCH = 7,   /* host: eg_build_noalloc: the field needs more than its fixed scratch */
    EG_ERR_UNRESOLVED = 8 /* device header: a label was still a code after the last label pass
                             (an internal error: the pass count covers every path; outputs undefined) */
} eg_status;

/* eg_out.flags */
#define EG_MINIMA 0x1u /* build the minimum graph instead of the maximum graph */

#define EG_MAX_NDIM 6

/* Slots of the device header (int32 each, EG_H_SLOTS in total). */
#define EG_H_STATUS 0 /* eg_status of the device-side work */
#define EG_H_NMAX 1   /* number of maxima (required size of maxima[]) */
#define EG_H_NSAD 2   /* number of saddles (required size of saddles[], saddle_beta[]) */
#define EG_H_NARC 3   /* number of arcs (required size of arc_maxima[]); -1 if unknown */
#define EG_H_NPAIRS 4 /* number of (saddle, upper-link component) pairs, the sum of beta; -1 if unknown */
#define EG_H_PASSES 5 /* per-vertex label passes that ran */
#define EG_H_EXITS 6  /* tile exit-list entries the labels used (diagnostic) */
#define EG_H_SLOTS 8

/*
 * Output description for one field.  All pointers are device pointers.
 *
 *   labels       [N]            label (vertex id of the maximum) of every vertex;
 *                               16-byte aligned
 *   ptr          [N] or NULL    steepest-ascent pointer of every vertex (optional)
 *   maxima       [cap_max]      ascending vertex ids of the maxima
 *   saddles      [cap_sad]      ascending vertex ids of the saddles
 *   saddle_beta  [cap_sad] or NULL   upper-link component count of each saddle
 *   arc_offsets  [cap_sad + 1]  CSR row offsets: saddle i owns arc_maxima[arc_offsets[i] ..
 *                               arc_offsets[i+1]), ascending and distinct
 *   arc_maxima   [cap_arc]      maxima ids of the arcs
 *   workspace    device scratch of at least eg_workspace_bytes(...) bytes,
 *                256-byte aligned; contents need not be initialised
 *   header       [EG_H_SLOTS] int32 device; written by the library
 */
typedef struct eg_out {
    uint32_t flags;
    int32_t* labels;
    int32_t* ptr;
    int32_t* maxima;
    int64_t cap_max;
    int32_t* saddles;
    int32_t* saddle_beta;
    int32_t* arc_offsets;
    int64_t cap_sad;
    int32_t* arc_maxima;
    int64_t cap_arc;
    void* workspace;
    size_t ws_bytes;
    int32_t* header;
    uint32_t tuning; /* launch configuration (EG_TUNE_*), 0 = defaults; never changes results */
} eg_out;

/*
 * eg_out.tuning: launch choices an autotuner may vary.  Every choice gives
 * bit-identical results.
 *   EG_TUNE_TILE3(v)  3D tile: 0 = 64x8x8, 1 = 64x4x16, 2 = 64x8x4
 *   EG_TUNE_TILE2(v)  2D tile: 0 = 64x32, 1 = 64x16
 *   EG_TUNE_HOPS(h)   links followed per label pass: 0 = 64; 16, 32, 64 or 128
 *   EG_TUNE_EXITS(e)  most exit-list entries: 0 = the default capacity, e = 1..30
 *                     caps it at 2^e (a test hook for the path that tiles whose
 *                     exits do not fit take: labels by vertex codes instead)
 * Other values are EG_ERR_ARG.  A batch uses outs[0].tuning for its launch
 * choices and each field's own EG_TUNE_EXITS.
 */
#define EG_TUNE_TILE3(v) ((uint32_t)(v) & 0xFu)
#define EG_TUNE_TILE2(v) (((uint32_t)(v) & 0xFu) << 4)
#define EG_TUNE_HOPS(h) (((uint32_t)(h) & 0xFFu) << 8)
#define EG_TUNE_EXITS(e) (((uint32_t)(e) & 0x1Fu) << 16)

/*
 * Workspace bytes that eg_build needs for a field of the given shape and the
 * given saddle capacity (eg_out.cap_sad; the other capacities do not enter):
 * about 4.25 bytes per vertex (more when the last axis is much shorter than
 * 64; 4 more for 1D, 4D, 5D and 6D grids) plus 16 bytes per saddle slot (32
 * for 4D, 5D and 6D grids).  Pure,
 * host-only.  Returns 0 on invalid arguments (ndim outside [1, EG_MAX_NDIM],
 * a dim < 1, N >= 2^31, a capacity outside [0, 2^31)).
 */
size_t eg_workspace_bytes(int ndim, const int64_t* dims, int64_t cap_sad);

/*
 * Extremum graph of one field (Sec. 3: classification, then path tracing).
 *
 *   field   device, float32[N], C order, read-only
 *   ndim    1..EG_MAX_NDIM
 *   dims    host, int64[ndim], each >= 1, product N < 2^31
 *   stream  hipStream_t (as void*) on which all work is queued
 *   out     host struct describing the caller's device buffers (see eg_out)
 *
 * Returns EG_OK once the work is queued; the device header then carries the
 * final status and the counts.  On EG_ERR_CAPACITY every count in the header
 * is the size needed, except EG_H_NARC and EG_H_NPAIRS, which are -1 when the
 * saddles overflowed (retry with cap_sad >= EG_H_NSAD first).  Entries below
 * each capacity are written even then.  Outputs are bit-identical for
 * identical inputs and independent of launch configuration.
 */
eg_status eg_build(const float* field, int ndim, const int64_t* dims, void* stream,
                   const eg_out* out);

/*
 * eg_build for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * Same arguments, outputs and results as eg_build, except that out->workspace
 * and out->ws_bytes are ignored: the workspace is a fixed device array inside
 * the library, eg_noalloc_scratch_bytes() bytes (64 MiB) on each device,
 * reserved when the library's code is loaded on that device and held until the
 * process ends.  The caller still owns every output buffer and the header.
 * The array of the device current at the call is used, so `stream` must
 * belong to that device.  Nothing is allocated, freed or synchronised; the
 * first call on a device looks up the array's address once (no allocation).
 *
 * Errors: as eg_build, plus EG_ERR_SCRATCH (synchronous, nothing queued) when
 * eg_workspace_bytes(ndim, dims, out->cap_sad) exceeds the scratch size (about
 * 15 M vertices of a 2D or 3D field with modest saddle capacity), and EG_ERR_HIP
 * when the array's address cannot be found.
 *
 * Every call on one device shares that device's array (its contents are left
 * from the last call; every call clears what it needs): calls that overlap on
 * one device, from several streams or threads, race and give undefined
 * results.  Serialise them, e.g. on one stream.
 */
eg_status eg_build_noalloc(const float* field, int ndim, const int64_t* dims, void* stream,
                           const eg_out* out);
size_t eg_noalloc_scratch_bytes(void);

/*
 * eg_build of a field that sits in host memory, with the copy to the device
 * overlapped with classification (the paper's slab decomposition along the
 * slowest axis, Sec. 4, re-thought for one GPU whose memory holds the field):
 * the field is copied slab by slab (slab_planes planes of axis 0, rounded up
 * to whole tile rows) on copy_stream, each slab followed by events[k]; on
 * stream, the tiles of slab k are classified once slab k + 1 has landed (one
 * plane of it is their ghost layer); labels and arcs follow for the whole
 * field.  Results equal eg_build's on the same field.
 *
 *   host_field   host, float32[N], C order; page-locked (pinned) memory for
 *                the copies to overlap (pageable memory works, but the runtime
 *                may then copy synchronously)
 *   dev_field    device, float32[N]: receives the field (caller-owned)
 *   ndim         2 or 3
 *   slab_planes  >= 1
 *   stream       compute stream; copy_stream: a different stream for the copies
 *   events       hipEvent_t[nevents] created by the caller, nevents >= the
 *                number of slabs, ceil(dims[0] / slab planes), plus one: the
 *                last is recorded on stream first, and the copies wait for it
 *                (work already queued there may still read dev_field)
 *   out          as for eg_build
 *
 * Errors: as eg_build, plus EG_ERR_ARG for a NULL host or device field, ndim
 * outside {2, 3}, slab_planes < 1 or too few events; EG_ERR_HIP when a copy
 * or an event call fails.  Nothing is allocated or synchronised.
 */
eg_status eg_build_streamed(const float* host_field, float* dev_field, int ndim, const int64_t* dims,
                            int64_t slab_planes, void* stream, void* copy_stream, void* const* events,
                            int64_t nevents, const eg_out* out);

/*
 * The three stages of eg_build, callable one at a time with the same
 * arguments (eg_build = eg_classify, then eg_label, then eg_arcs, on one
 * stream).  Each validates its arguments like eg_build.
 *
 * eg_classify  Sec. 3.3 / Table 1: resets the header and the workspace
 *              counters, then for every vertex its steepest-ascent pointer
 *              (into labels[], and ptr[] when given), the maxima (empty upper
 *              link) and the saddle candidates (>= 2 upper-link components),
 *              kept in the workspace as bitmasks.
 * eg_label     Sec. 2 / Alg. 2 (the walk to a maximum): pointer jumping on
 *              labels[] in place until every entry names its maximum.  Needs
 *              eg_classify's labels[] and workspace.
 * eg_arcs      Sec. 3.4 Alg. 2 / UpperLinkRep: the ascending maxima and
 *              saddles (compaction of the bitmasks), the highest vertex of
 *              every upper-link component of every saddle, its label, the
 *              distinct (saddle, maximum) arcs as a CSR, and the header.
 *              Needs the labels and workspace of the two stages before it.
 */
eg_status eg_classify(const float* field, int ndim, const int64_t* dims, void* stream,
                      const eg_out* out);
eg_status eg_label(const float* field, int ndim, const int64_t* dims, void* stream,
                   const eg_out* out);
eg_status eg_arcs(const float* field, int ndim, const int64_t* dims, void* stream,
                  const eg_out* out);

/*
 * Gradient-path geometry (Sec. 3.4, Alg. 2): for every saddle s and every
 * component of its upper link, the vertex list of the path that Alg. 2 walks:
 * s, r, ptr(r), ptr(ptr(r)), ..., m, where r is the component's highest vertex
 * (UpperLinkRep) and m the maximum it reaches (ptr(m) = m).  Saddles come in
 * the order of eg_out.saddles; the components of a saddle in ascending order
 * of their smallest vertex id.  There are beta+ paths per saddle; the set of
 * their last vertices is the saddle's arc row.
 *
 *   pair_offsets   [cap_sad + 1]  saddle i owns paths pair_offsets[i] .. pair_offsets[i+1]
 *   path_offsets   [cap_paths + 1] path k is path_vertices[path_offsets[k] .. path_offsets[k+1])
 *   path_vertices  [cap_vertices] vertex ids
 *   header         [EG_P_SLOTS] int32 device: status, number of paths, number of vertices
 *
 * eg_paths(field, ndim, dims, stream, out, paths) reads the outputs of an
 * eg_build (or eg_classify + eg_label + eg_arcs) with the same `out`, queued
 * earlier on the same stream: out->ptr must be given.
 * Host errors as eg_build, plus EG_ERR_ARG for a missing ptr, saddle_beta or
 * paths buffer.  Device: EG_ERR_CAPACITY with the required counts when a
 * capacity is short (entries below each capacity are written), or when the
 * saddles themselves exceeded out->cap_sad; EG_ERR_ARG when out->ptr does not
 * hold this field's pointers (a step that leaves the grid or does not rise
 * ends that walk).
 */
#define EG_P_STATUS 0
#define EG_P_PATHS 1
#define EG_P_VERTICES 2
#define EG_P_SLOTS 4

typedef struct eg_paths_out {
    int32_t* pair_offsets;
    int32_t* path_offsets;
    int64_t cap_paths;
    int32_t* path_vertices;
    int64_t cap_vertices;
    int32_t* header;
} eg_paths_out;

eg_status eg_paths(const float* field, int ndim, const int64_t* dims, void* stream, const eg_out* out,
                   const eg_paths_out* paths);

/*
 * Simplification of a finished extremum graph (Sec. 3.5), on the host: the
 * graph has one node per critical point and the cancellations depend on one
 * another, as in the paper's serial implementation.
 *
 *   EG_SIMPLIFY_BUNDLE  arc bundling: for every pair of maxima that share
 *                       saddles, the highest shared saddle represents the pair
 *                       and the pair's other saddles are discarded; a saddle
 *                       survives iff it represents one of its pairs or has
 *                       fewer than two distinct maxima (no pair shares it).
 *   EG_SIMPLIFY_CANCEL  persistence-directed cancellation: saddles are taken in
 *                       order of cost = height of the second-highest of their
 *                       maxima - height of the saddle (for a simple saddle the
 *                       lower of its two maxima; ties: the lower saddle first),
 *                       costs recomputed when a saddle comes up: above the
 *                       threshold it is discarded, above the cost stored at
 *                       the top of the queue it is queued again, else it is
 *                       cancelled: every one of its maxima except the highest
 *                       merges into the highest and the saddle leaves the
 *                       graph.  Applied after bundling when both are set.
 *
 * Heights are the field values in the graph's order (ties by vertex id),
 * reversed for a minimum graph (flags = EG_MINIMA), passed as doubles (exact
 * for every sample type except 64-bit integers of magnitude above 2^53).  All pointers are host
 * memory.  Inputs: the graph as eg_build returns it (ascending maxima and
 * saddles, CSR arcs of maxima ids) and the field value at every maximum and
 * saddle.  Outputs:
 *   out_offsets [nsad + 1], out_arcs [arc_offsets[nsad]]  the simplified arcs of
 *       every saddle (an empty row for a saddle removed by bundling or
 *       cancelled), the ascending distinct representatives of its maxima (one
 *       entry when they all merged into one)
 *   max_rep [nmax]     index of the maximum each maximum merged into (its own
 *                      index if it survives)
 *   pair_saddle, pair_max [arc_offsets[nsad]], pair_cost   the cancellations in
 *                      order, one row per merged maximum (saddle index,
 *                      maximum index, the cancellation's cost; the maxima of
 *                      one cancellation from the highest down); *n_pairs rows
 * EG_ERR_ARG for NULL pointers, unknown ops, a NaN threshold, unsorted maxima,
 * malformed offsets or an arc to a vertex that is not in maxima.
 */
#define EG_SIMPLIFY_BUNDLE 0x1u
#define EG_SIMPLIFY_CANCEL 0x2u

typedef struct eg_graph_host {
    uint32_t flags;
    int64_t nmax;
    const int32_t* maxima;
    const double* max_values;
    int64_t nsad;
    const int32_t* saddles;
    const double* sad_values;
    const int32_t* arc_offsets;
    const int32_t* arc_maxima;
} eg_graph_host;

eg_status eg_simplify(const eg_graph_host* graph, uint32_t ops, double threshold, int32_t* out_offsets,
                      int32_t* out_arcs, int32_t* max_rep, int32_t* pair_saddle, int32_t* pair_max,
                      double* pair_cost, int64_t* n_pairs);

/*
 * Batches: the extremum graphs of `count` independent 2D or 3D fields in one
 * launch sequence.  Classification runs one launch per class of fields (2D or
 * 3D, maximum or minimum graph) over a work list of (field, tile) items;
 * labels, compaction, arcs and the per-field CSR outputs are computed for all
 * fields together, each launch split over the fields in proportion to their
 * size.  Results equal eg_build's for every field.
 *
 * Field i is described exactly as for eg_build: fields[i] (device float32),
 * ndims[i] (2 or 3), dims[i * EG_MAX_NDIM + 0 .. ndims[i]-1], outs[i] (its own
 * output buffers, header and workspace of eg_workspace_bytes).
 * The batch also needs a batch workspace (device, 256-byte aligned, at least
 * eg_batch_workspace_bytes) and a plan:
 *
 *   1. eg_batch_plan() validates everything (host only) and writes the plan
 *      into host memory of eg_batch_plan_bytes(count) bytes;
 *   2. the caller copies those bytes to the start of the batch workspace
 *      (any stream-ordered or synchronous host-to-device copy);
 *   3. eg_build_batched(host_plan, stream) queues the work.  It never
 *      allocates or synchronises, so a plan can be replayed, e.g. from a HIP
 *      graph, as long as the fields and buffers it names stay in place.
 *
 * Errors: EG_ERR_ARG for ndim outside {2, 3}, NULL pointers or a short host
 * plan buffer; EG_ERR_TOO_LARGE when a field or a capacity is too large;
 * EG_ERR_WORKSPACE for a missing, misaligned or short workspace.  Device-side
 * conditions go to each field's header.
 */
size_t eg_batch_plan_bytes(int count);
size_t eg_batch_workspace_bytes(int count, const int* ndims, const int64_t* dims, const eg_out* outs);
eg_status eg_batch_plan(int count, const float* const* fields, const int* ndims, const int64_t* dims,
                        const eg_out* outs, void* batch_ws, size_t batch_ws_bytes, void* host_plan,
                        size_t host_plan_bytes);
eg_status eg_build_batched(const void* host_plan, void* stream);

/*
 * Sample types (Sec. 4: the input may hold 8- to 64-bit signed or unsigned
 * integers, or 32- or 64-bit floats).  The graph depends on the samples only
 * through the simulated-perturbation order (Sec. 3.3: u below v iff f[u] <
 * f[v] compared in the sample type, or equal and u < v), so a field of any
 * type is first turned into a float32 field with exactly the same order, its
 * order surrogate, and eg_build then runs unchanged on that:
 *
 *   EG_F32                  a copy
 *   EG_I8, EG_U8, EG_I16,   the value converted to float32 (exact, ties kept)
 *   EG_U16
 *   EG_I32, EG_U32, EG_I64, the rank of (value, index) in the order, encoded
 *   EG_U64, EG_F64          as a strictly increasing float32 (no ties left):
 *                           a stable LSD radix sort of order-preserving
 *                           integer keys of the values
 *
 * For float types -0 equals +0 and infinities order normally; a NaN in the
 * field leaves NaN in the surrogate (every entry, for EG_F64), so eg_build then
 * reports EG_ERR_NAN.
 */
typedef enum eg_dtype {
    EG_F32 = 0,
    EG_F64 = 1,
    EG_I8 = 2,
    EG_U8 = 3,
    EG_I16 = 4,
    EG_U16 = 5,
    EG_I32 = 6,
    EG_U32 = 7,
    EG_I64 = 8,
    EG_U64 = 9
} eg_dtype;

/*
 * Workspace bytes eg_order_field needs for n samples of the given type: 0 for
 * EG_F32 and the 8- and 16-bit types; about 2(sizeof key + 4) bytes per sample
 * for the ranked types (the key is 4 bytes for 32-bit types, 8 for 64-bit
 * ones) plus a fixed part.  Host-only; 0 also for invalid arguments (unknown
 * dtype, n < 1 or n >= 2^31).
 */
size_t eg_order_workspace_bytes(int dtype, int64_t n);

/*
 * Order surrogate of a field of n samples (any shape: the order does not
 * depend on it).
 *
 *   dtype      an eg_dtype
 *   field      device, n samples of that type, read-only
 *   out        device, float32[n]: for all u, v, (out[u], u) is below
 *              (out[v], v) in the simulated-perturbation order iff (field[u],
 *              u) is below (field[v], v); may not overlap field
 *   workspace  device, 256-byte aligned, eg_order_workspace_bytes(dtype, n)
 *              bytes (may be NULL when that is 0)
 *   stream     hipStream_t (as void*) on which the work is queued
 *
 * Host errors: EG_ERR_ARG (unknown dtype, NULL field/out, n < 1, out
 * overlapping field), EG_ERR_TOO_LARGE (n >= 2^31), EG_ERR_WORKSPACE, EG_ERR_HIP.
 * Never allocates or synchronises.
 */
eg_status eg_order_field(int dtype, const void* field, int64_t n, float* out, void* workspace, size_t ws_bytes,
                         void* stream);

/* Human-readable name of a status code (static string). */
const char* eg_status_string(int status);

/*
 * Host-only: the neighbour table the kernels use for an n-dimensional grid
 * (Alg. 1).  Writes k = 2(2^n - 1) rows sorted so that, for any in-bounds
 * neighbours, row order equals linear-index order: offsets[j * ndim + i] in
 * {-1,0,1} is the coordinate difference on axis i; the adjacency of row j is
 * W = (k + 63) / 64 words (1 up to n = 5, 2 for n = 6), adjacency[j * W + l / 64]
 * bit l % 64 set iff neighbours j and l are adjacent to each other (a link
 * edge).  Returns k, or -1 for ndim outside [1, EG_MAX_NDIM].  Buffers may be
 * NULL to query k.
 */
int eg_link_table(int ndim, int8_t* offsets, uint64_t* adjacency);

#ifdef __cplusplus
}
#endif

#endif /* EG_H */
