// eg_internal.h -- shared definitions of the HIP extremum-graph library.
//
// Vertex order.  The simulated-perturbation order of Sec. 3.3 (u below v iff
// f[u] < f[v], or f[u] == f[v] and u < v) is evaluated with a 32-bit
// order-preserving integer image of the float (order_key): after -0 is mapped
// to +0, x < y as floats iff key(x) < key(y) as unsigned integers.  Ties
// between equal keys are decided by linear index.  For the minimum graph the
// order is reversed, which equals using ~key with the tie-break reversed.
//
// Neighbour rows.  The 2(2^n - 1) Freudenthal neighbours (Alg. 1) are stored
// as rows sorted lexicographically by coordinate offset: the {0,-1}^n rows
// first, then the {0,1}^n rows.  For any in-bounds neighbours this row order is
// the order of their linear indices, and the vertex itself sits between the
// two halves.  So a scan of the closed neighbourhood in row order visits
// vertices in increasing index order, and "later wins ties" is a single >=.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "eg.h"

namespace eg {

constexpr int kMaxNb = 126;         // 2(2^6 - 1)
constexpr int kJumpHops = 64;       // default links per pointer-jumping pass
constexpr int kMaxPasses = 8;       // flag slots per pass sequence
constexpr int kArcBlocks = 8192;    // most blocks per field of the stage (d) kernels
constexpr int kArcVertsPerBlock = 8192;  // stage (d) blocks: one per this many vertices
constexpr int kTile3Y = 8, kTile3Z = 8;  // default 3D tile: 64 x 8 x 8 vertices
constexpr int kTile2Y = 32;             // default 2D tile: 64 x 32 vertices

// Decoded eg_out.tuning.
struct Tuning {
    int tile3;  // 0: 64x8x8, 1: 64x4x16, 2: 64x8x4
    int tile2;  // 0: 64x32, 1: 64x16
    int hops;   // links per label pass
    int passes; // passes that cover any path of fewer than 2^31 links
    int64_t exit_cap;  // most exit-list entries (0: the default capacity)
};
bool decode_tuning(uint32_t t, Tuning* out);
// Label passes for a grid of n vertices: a steepest-ascent path has fewer
// than n links and pass p leaves every entry hops^(p+1) links further on or
// final, so the smallest p with hops^p >= n suffices (at most t.passes).
int passes_for(const Tuning& t, int64_t n);
inline void tile_shape(const Tuning& t, int ndim, int* ty, int* tz)
{
    if (ndim == 3) {
        static const int ys[3] = {8, 4, 8}, zs[3] = {8, 16, 4};
        *ty = ys[t.tile3];
        *tz = zs[t.tile3];
    } else {
        static const int ys[2] = {32, 16};
        *ty = ys[t.tile2];
        *tz = 1;
    }
}

// counter slots in the workspace (uint32 each)
enum : int {
    C_NAN = 0,
    C_NMAX = 1,
    C_NSAD = 2,
    C_NPAIRS = 3,
    C_NARC = 4,
    C_PASSES = 6,
    C_PATHS = 40,     // paths (sum of beta over the saddles) for eg_paths
    C_PVERTS = 41,    // their vertices
    C_PBAD = 42,      // eg_paths met a pointer that leaves the grid or does not rise
    C_NEXIT = 7,  // exit-list entries requested by the tiles
    C_JUMP = 8,   // kMaxPasses "not converged" flags of the exit-list passes
    C_FINAL = 16, // kMaxPasses "not converged" flags of the per-vertex passes
    C_SLOTS = 64,
};

// Neighbour table for one grid, passed by value as a kernel argument (the
// rows' mutual adjacency is a compile-time table, eg_rows.h).
struct LinkTable {
    int32_t k;                 // number of rows, 2(2^n - 1)
    int32_t lin[kMaxNb];       // linear index offset of row j
    uint32_t forb[kMaxNb];     // boundary bits that rule row j out (see boundary_bits)
};

struct Grid {
    int32_t ndim;
    int32_t N;
    int32_t dims[EG_MAX_NDIM];
};

// Critical vertices between classification and stage (d) are kept as two
// bitmasks (maxima, saddles) in a row-padded layout: the grid is cut into
// rows along its fastest axis (X vertices each), every row takes XW =
// ceil(X / 64) 64-bit words, and vertex (row, x) is bit x % 64 of word
// row * XW + x / 64.  A wave of a 64-wide tile writes exactly one word per
// row, and a scan over the words lists the vertices in ascending order.
inline int64_t mask_words(int64_t N, int64_t X) { return (N / X) * ((X + 63) / 64); }

// Carved workspace.
struct Work {
    uint32_t* ctr;    // [C_SLOTS]
    uint64_t* mmask;  // [words] maxima
    uint64_t* smask;  // [words] saddles
    uint32_t* bsum;   // [4 * kArcBlocks] per-block counts of stage (d)
    uint4* atmp;      // [cap_sad] the first four arcs of every saddle ([2 cap_sad], eight, from 4D on)
    uint32_t* exits;  // [cap_exit] exit vertices published by the tiles
    int32_t* exres;   // [cap_exit] their labels while being resolved
    uint32_t* keys;   // [N] order keys of the untiled grids (1D, 4D, 5D); else null
    int64_t words;
    int64_t cap_exit;
    size_t bytes;
};

// Pointers to device memory in the structs below are typed as global-memory
// pointers in device code (same 64-bit layout as the host's plain pointers).
// Structs read from a batch plan would otherwise give the compiler generic
// pointers, whose flat instructions also wait on the LDS counter.
#if defined(__HIP_DEVICE_COMPILE__)
#define EG_GPTR(T) __attribute__((address_space(1))) T*
#else
#define EG_GPTR(T) T*
#endif
template <class T>
__host__ __device__ inline EG_GPTR(T) gptr(T* p)
{
    return (EG_GPTR(T))p;
}

// Everything a classification tile needs to know about its field.
struct TileArgs {
    EG_GPTR(const float) f;
    EG_GPTR(int32_t) lab;
    EG_GPTR(int32_t) ptr;
    EG_GPTR(uint32_t) ctr;
    EG_GPTR(uint64_t) mmask;
    EG_GPTR(uint64_t) smask;
    EG_GPTR(uint32_t) exits;
    int32_t X, Y, Z, tiles_x, tiles_y, ntiles;
    uint32_t cap_exit, pad0;
};

// Everything stage (d) needs to know about its field.
struct ArcArgs {
    EG_GPTR(const float) f;
    EG_GPTR(const uint32_t) keys;  // order keys when classification stored them, else null
    EG_GPTR(const int32_t) lab;
    EG_GPTR(const uint64_t) mmask;
    EG_GPTR(const uint64_t) smask;
    EG_GPTR(uint32_t) bsum;
    EG_GPTR(uint4) atmp;
    EG_GPTR(uint32_t) ctr;
    EG_GPTR(int32_t) header;
    EG_GPTR(int32_t) maxima;
    EG_GPTR(int32_t) saddles;
    EG_GPTR(int32_t) beta;  // may be null
    EG_GPTR(int32_t) offsets;
    EG_GPTR(int32_t) arcs;
    int32_t ndim, minima, N, X, XW, words;
    int32_t dims[EG_MAX_NDIM];
    uint32_t cap_max, cap_sad, cap_arc;
    int32_t arc_blocks;  // blocks of this field in the stage (d) kernels (<= kArcBlocks)
    int32_t pad0;
    // "not converged" flag of the last label pass (set: some label is still
    // a code, the header reports EG_ERR_UNRESOLVED); null: not checked
    EG_GPTR(const uint32_t) last_flag;
};

// The outputs of eg_paths for one field.
struct PathArgs {
    EG_GPTR(const int32_t) ptr;
    EG_GPTR(int32_t) pair_offsets;
    EG_GPTR(int32_t) path_offsets;
    EG_GPTR(int32_t) vertices;
    EG_GPTR(int32_t) header;
    uint32_t cap_paths, cap_vertices;
};

// One field of a batch (device-resident plan, built on the host).
struct BatchField {
    TileArgs ta;
    ArcArgs arc;
    int32_t ndim, minima, N, pad0;
    int64_t tile_base;   // exclusive prefix over fields of tiles
    int64_t arc_base;    // ... of stage (d) blocks
    EG_GPTR(int32_t) exres;
};

struct BatchPlan {
    int32_t count, pad0;
    Tuning tuning;
    int64_t total_tiles, total_arc_blocks;
    // fields are ordered by class (2D max, 2D min, 3D max, 3D min); class c
    // owns fields [class_field[c], class_field[c + 1]) and tiles
    // [class_tile[c], class_tile[c + 1])
    int32_t class_field[5];
    int32_t pad1;
    int64_t class_tile[5];
    EG_GPTR(uint32_t) bctr;      // [C_SLOTS] batch counters (label pass flags)
    EG_GPTR(BatchField) fields;  // device address of fields[] (right after this header)
    const BatchPlan* dev; // device address of this plan (start of the batch workspace)
    int64_t plan_bytes;
};

// Host: table rows for ndim (Alg. 1), independent of dims.  Returns k.  The
// adjacency of row j is adj[j * W .. j * W + W), W = (k + 63) / 64 words.
int make_rows(int ndim, int8_t (*off)[EG_MAX_NDIM], uint64_t* adj);
// Host: full kernel table for a grid.
void make_table(const Grid& g, LinkTable* t);
// Host: carve (or size, when base == nullptr) the workspace of a grid with N
// vertices.
Work carve(void* base, int ndim, int64_t N, int64_t X, int64_t cap_sad, int64_t exit_cap = 0);
// Exit-list capacity for a grid of N vertices (label codes need N + cap < 2^31).
int64_t exit_capacity(int64_t N);
// Bits needed to hold any vertex id of a grid with N vertices.
inline int id_bits(int64_t N)
{
    int b = 1;
    while ((int64_t(1) << b) < N) ++b;
    return b;
}

// ------------------------------------------------------------------ device

// Keys lie in [1, 0xFFFFFFFE] in both modes (non-NaN values map into
// [0x007FFFFF, 0xFF800000]; NaN patterns, reported as an error, are clamped),
// so 0 is a sentinel below every vertex, used for positions outside the grid:
// no pointer can ever leave the grid.
// Adding +0.0 turns -0 into +0 (round to nearest) and leaves every other
// value unchanged; the sign-dependent flip makes unsigned order equal float
// order; the clamp keeps NaN patterns off the sentinel.
__device__ __forceinline__ uint32_t order_key(float x)
{
    const uint32_t b = __float_as_uint(x + 0.0f);
    const uint32_t k = b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
    return min(max(k, 1u), 0xFFFFFFFEu);
}

template <bool MINMODE>
__device__ __forceinline__ uint32_t mode_key(float x)
{
    const uint32_t k = order_key(x);
    return MINMODE ? ~k : k;
}

// Boundary bits of a vertex: bit 2i set if coordinate i is 0, bit 2i+1 set if
// it is dims[i]-1.  Row j exists iff (bits & forb[j]) == 0.
__device__ __forceinline__ uint32_t boundary_bit(int c, int d, int axis)
{
    return (uint32_t(c == 0) << (2 * axis)) | (uint32_t(c == d - 1) << (2 * axis + 1));
}

// Whether row j beats an equal key (it lies later in visiting order).  In the
// maximum graph later = larger index = the {0,1} half; in the minimum graph
// the roles swap.
template <bool MINMODE>
__device__ __forceinline__ bool row_wins_tie(int j, int k)
{
    return (j >= k / 2) != MINMODE;
}

// f(std::integral_constant<int, i>) for i in [I, N): compile-time row indices.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Upper-link masks, one 32-bit word per 32 rows, built from the highest row
// down: up = 2 up + (u above c), where the comparison's lane mask is the carry
// of an add that doubles the word (two instructions per row); a row that wins
// ties is above at equal keys.
template <bool WINS_TIE>
__device__ __forceinline__ uint32_t push_above(uint32_t up, uint32_t u, uint32_t c)
{
    uint32_t r;
    if constexpr (WINS_TIE)
        asm("v_cmp_ge_u32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %3, %3, vcc" : "=v"(r) : "v"(u), "v"(c), "v"(up) : "vcc");
    else
        asm("v_cmp_gt_u32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, %3, %3, vcc" : "=v"(r) : "v"(u), "v"(c), "v"(up) : "vcc");
    return r;
}
// The first row's comparison as the mask's lowest bit (no zero to double).
template <bool WINS_TIE>
__device__ __forceinline__ uint32_t first_above(uint32_t u, uint32_t c)
{
    uint32_t r;
    if constexpr (WINS_TIE)
        asm("v_cmp_ge_u32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, 0, 0, vcc" : "=v"(r) : "v"(u), "v"(c) : "vcc");
    else
        asm("v_cmp_gt_u32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, 0, 0, vcc" : "=v"(r) : "v"(u), "v"(c) : "vcc");
    return r;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_init(uint32_t* ctr, int32_t* header, hipStream_t s);
hipError_t launch_classify(const float* f, const Grid& g, const LinkTable& t, bool minima, int32_t* lab,
                           int32_t* ptr, const Work& w, const Tuning& tu, hipStream_t s);
// Classification of the 2D/3D tiles [first, first + count) (tiles in C order:
// tile rows along axis 0 are contiguous ranges); count < 0: every tile.
hipError_t launch_classify_tiled(const float* f, const Grid& g, bool minima, int32_t* lab, int32_t* ptr,
                                 const Work& w, const Tuning& tu, hipStream_t s, int64_t first = 0,
                                 int64_t count = -1);
TileArgs tile_args(const float* f, const Grid& g, int32_t* lab, int32_t* ptr, const Work& w, int ty, int tz);
ArcArgs arc_args(const float* f, const Grid& g, const eg_out& o, const Work& w);
uint32_t arc_blocks(int64_t N);
hipError_t launch_classify_batched(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s);
hipError_t launch_batched_init(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s);
hipError_t launch_batched_rest(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s);

// Label codes between classification and the label pass (int32):
//   x >= 0            final: the maximum x
//   -N <= x <= -1     "same label as vertex -x-1" (a later vertex of the path)
//   x < -N            "same label as exit-list entry -x-1-N"
__device__ __forceinline__ int exit_list_code(int N, uint32_t idx) { return -(N + 1 + (int)idx); }
hipError_t launch_labels(const Grid& g, int32_t* lab, const Work& w, const Tuning& tu, hipStream_t s);
// Tile-ordered first per-vertex label pass (2D/3D grids); raises ctr[flag_slot]
// if some vertex is not final yet.
hipError_t launch_final_tiled(const Grid& g, int32_t* lab, const Work& w, const Tuning& tu, int flag_slot,
                              hipStream_t s);
// The tile-ordered pass over every field of a batch; raises bctr[C_FINAL].
hipError_t launch_final_tiled_batched(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s);
// Stage (d) of one field: ascending maxima and saddles from the bitmasks,
// the arcs of every saddle, the CSR and the header.
hipError_t launch_arcs(const ArcArgs& a, hipStream_t s);
// Gradient-path geometry of one field (after stage (d)).
hipError_t launch_paths(const ArcArgs& a, const PathArgs& p, hipStream_t s);
// Stage (d) of every field of a batch (fields are blockIdx.y).
hipError_t launch_arcs_batched(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s);

}  // namespace eg
