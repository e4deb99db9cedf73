/*
 * eg_oracle.c -- plain CPU reference for the extremum graph of a PL scalar
 * field on an n-dimensional grid (Ande, Subhash, Natarajan, "TACHYON:
 * Efficient Shared Memory Parallel Computation of Extremum Graphs").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke entry point and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header, table or helper
 * with the GPU library and must never serve as a fallback for it.
 *
 * It computes the definitions written out, slowly and plainly:
 *
 *   adjacency   Freudenthal tessellation, GridAdjacency test (Sec. 3.2, Alg. 1):
 *               p ~ q iff p != q and every p_i - q_i lies in {0,1}, or every one
 *               lies in {0,-1}.  Neighbours are found by trying all 3^n - 1
 *               offset vectors and applying that test literally; vertices
 *               outside the grid simply do not exist (truncated link).
 *   order       simulated perturbation (Sec. 3.3): a strict total order,
 *               u below v iff f[u] < f[v], or f[u] == f[v] and u < v, with u, v
 *               row-major linear indices (C order, dims[0] slowest).  Samples
 *               are compared as values of the field's own type (8- to 64-bit
 *               signed or unsigned integers, float32, float64: the input types
 *               of Sec. 4); IEEE comparison makes -0 equal to +0.  The minima
 *               graph uses the reversed order.
 *   upper link  U(v) = link vertices above v; link edges are pairs of link
 *               vertices that are themselves adjacent (Sec. 3.3).
 *   beta+       number of connected components of U(v), found by BFS over the
 *               link edges (the textbook traversal the paper names in Sec. 3.3;
 *               the paper replaces it by union-find for the GPU, which counts
 *               the same components).  Table 1: maximum iff beta+ = 0,
 *               (n-1)-saddle iff beta+ >= 2.
 *   gradient    highest vertex of the upper link (Sec. 3.3), here for every
 *               vertex; a maximum points to itself.
 *   reps        UpperLinkRep (Sec. 3.4): the highest vertex of each upper link
 *               component of a saddle.
 *   labels      the maximum at the end of the gradient path from v (the walk
 *               of Alg. 2), i.e. the descending manifold that contains v.
 *   arcs        for every saddle s and rep r: the arc (s, label(r)); arcs form
 *               a set (Sec. 2), so duplicates are dropped.
 *   paths       the geometry of Alg. 2: for every saddle s and every upper-link
 *               component, the vertex list s, r, grad(r), grad(grad(r)), ...,
 *               up to the maximum, r being the component's rep.  A saddle's
 *               components are listed in ascending order of their smallest
 *               vertex id (the order a BFS seeded at the lowest unvisited
 *               upper-link vertex finds them).
 *
 * Parallelism: OpenMP over vertices for the per-vertex classification; the
 * label walk is serial with memoisation.  Nothing is blocked, fused or
 * reordered beyond that.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EGO_MAXDIM 8
#define EGO_MAXNB 512 /* 3^8 offsets bound the neighbour count */

enum { EGO_OK = 0, EGO_ERR_ARG = 1, EGO_ERR_NAN = 4, EGO_ERR_CAPACITY = 5, EGO_ERR_NOMEM = 7 };

/* sample types */
enum { EGO_F32 = 0, EGO_F64 = 1, EGO_I8 = 2, EGO_U8 = 3, EGO_I16 = 4, EGO_U16 = 5, EGO_I32 = 6, EGO_U32 = 7,
       EGO_I64 = 8, EGO_U64 = 9, EGO_NTYPES = 10 };

typedef struct {
    const void* f;
    int dtype;
    int n;
    int64_t dims[EGO_MAXDIM];
    int64_t N;
    int minima;
} grid_t;

static void to_coords(const grid_t* g, int64_t v, int64_t* c)
{
    for (int i = g->n - 1; i >= 0; --i) {
        c[i] = v % g->dims[i];
        v /= g->dims[i];
    }
}

static int64_t to_index(const grid_t* g, const int64_t* c)
{
    int64_t v = 0;
    for (int i = 0; i < g->n; ++i) v = v * g->dims[i] + c[i];
    return v;
}

/* Alg. 1, GridAdjacency: collect the coordinate differences; adjacent iff
 * they all lie in {0,1} or all lie in {0,-1} (and p != q). */
static int grid_adjacent(int n, const int64_t* p, const int64_t* q)
{
    int in01 = 1, in0m1 = 1, same = 1;
    for (int i = 0; i < n; ++i) {
        int64_t d = p[i] - q[i];
        if (d != 0) same = 0;
        if (!(d == 0 || d == 1)) in01 = 0;
        if (!(d == 0 || d == -1)) in0m1 = 0;
    }
    return !same && (in01 || in0m1);
}

/* Sign of f[a] - f[b], comparing the samples as values of their own type. */
#define EGO_CMP(T)                                                   \
    {                                                                \
        const T x = ((const T*)g->f)[a], y = ((const T*)g->f)[b];    \
        return (x > y) - (x < y);                                    \
    }
static int value_cmp(const grid_t* g, int64_t a, int64_t b)
{
    switch (g->dtype) {
        case EGO_F32: EGO_CMP(float)
        case EGO_F64: EGO_CMP(double)
        case EGO_I8: EGO_CMP(int8_t)
        case EGO_U8: EGO_CMP(uint8_t)
        case EGO_I16: EGO_CMP(int16_t)
        case EGO_U16: EGO_CMP(uint16_t)
        case EGO_I32: EGO_CMP(int32_t)
        case EGO_U32: EGO_CMP(uint32_t)
        case EGO_I64: EGO_CMP(int64_t)
        default: EGO_CMP(uint64_t)
    }
}
#undef EGO_CMP

static int is_nan(const grid_t* g, int64_t v)
{
    if (g->dtype == EGO_F32) return isnan(((const float*)g->f)[v]);
    if (g->dtype == EGO_F64) return isnan(((const double*)g->f)[v]);
    return 0;
}

/* a above b in the order that defines the graph (maxima: the simulated
 * perturbation order; minima: its reverse). */
static int above(const grid_t* g, int64_t a, int64_t b)
{
    const int c = value_cmp(g, a, b);
    if (!g->minima) return c > 0 || (c == 0 && a > b);
    return c < 0 || (c == 0 && b > a);
}

/* All neighbours of v: every offset in {-1,0,1}^n \ {0} whose target lies in
 * the grid and passes Alg. 1.  Returns the count; ids and coordinates out. */
static int neighbours(const grid_t* g, int64_t v, int64_t* ids, int64_t (*coords)[EGO_MAXDIM])
{
    int64_t c[EGO_MAXDIM], q[EGO_MAXDIM];
    to_coords(g, v, c);
    int n = g->n, cnt = 0;
    int64_t total = 1;
    for (int i = 0; i < n; ++i) total *= 3;
    for (int64_t t = 0; t < total; ++t) {
        int64_t r = t;
        int inside = 1;
        for (int i = 0; i < n; ++i) {
            int64_t d = (r % 3) - 1;
            r /= 3;
            q[i] = c[i] + d;
            if (q[i] < 0 || q[i] >= g->dims[i]) inside = 0;
        }
        if (!inside || !grid_adjacent(n, c, q)) continue;
        ids[cnt] = to_index(g, q);
        memcpy(coords[cnt], q, sizeof(int64_t) * (size_t)n);
        ++cnt;
    }
    return cnt;
}

/* Classify one vertex: gradient target, beta+, and the highest vertex of each
 * upper-link component (reps, in order of discovery; caller sorts if needed).
 * Returns the number of reps (= beta+). */
static int classify_vertex_mins(const grid_t* g, int64_t v, int64_t* ptr_out, int64_t* reps, int64_t* mins);
static int classify_vertex(const grid_t* g, int64_t v, int64_t* ptr_out, int64_t* reps)
{
    return classify_vertex_mins(g, v, ptr_out, reps, NULL);
}

/* The same, also giving the smallest vertex id of each component (mins may
 * be NULL). */
static int classify_vertex_mins(const grid_t* g, int64_t v, int64_t* ptr_out, int64_t* reps, int64_t* mins)
{
    int64_t ids[EGO_MAXNB];
    int64_t coords[EGO_MAXNB][EGO_MAXDIM];
    int k = neighbours(g, v, ids, coords);

    /* upper link vertices */
    int up[EGO_MAXNB], nu = 0;
    for (int j = 0; j < k; ++j)
        if (above(g, ids[j], v)) up[nu++] = j;

    /* gradient: highest upper-link vertex; v itself when the upper link is empty */
    int64_t best = v;
    for (int a = 0; a < nu; ++a)
        if (above(g, ids[up[a]], best)) best = ids[up[a]];
    *ptr_out = best;

    /* BFS over the upper link; edges are link-vertex pairs that are adjacent */
    int comp[EGO_MAXNB];
    for (int a = 0; a < nu; ++a) comp[a] = -1;
    int queue[EGO_MAXNB];
    int ncomp = 0;
    for (int a = 0; a < nu; ++a) {
        if (comp[a] >= 0) continue;
        int head = 0, tail = 0;
        queue[tail++] = a;
        comp[a] = ncomp;
        int64_t rep = ids[up[a]], lo = ids[up[a]];
        while (head < tail) {
            int x = queue[head++];
            if (above(g, ids[up[x]], rep)) rep = ids[up[x]];
            if (ids[up[x]] < lo) lo = ids[up[x]];
            for (int b = 0; b < nu; ++b) {
                if (comp[b] >= 0) continue;
                if (grid_adjacent(g->n, coords[up[x]], coords[up[b]])) {
                    comp[b] = ncomp;
                    queue[tail++] = b;
                }
            }
        }
        reps[ncomp] = rep;
        if (mins) mins[ncomp] = lo;
        ++ncomp;
    }
    return ncomp;
}

static int setup(grid_t* g, const void* f, int dtype, int ndim, const int64_t* dims, int minima)
{
    if (!f || dtype < 0 || dtype >= EGO_NTYPES || ndim < 1 || ndim > EGO_MAXDIM || !dims) return EGO_ERR_ARG;
    g->f = f;
    g->dtype = dtype;
    g->n = ndim;
    g->minima = minima ? 1 : 0;
    g->N = 1;
    for (int i = 0; i < ndim; ++i) {
        if (dims[i] < 1) return EGO_ERR_ARG;
        g->dims[i] = dims[i];
        g->N *= dims[i];
    }
    return EGO_OK;
}

/* ------------------------------------------------------------------ API */

int ego_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops that follow (n < 1: leave unchanged); returns
   the previous count.  Used to time the oracle on one core and on all. */
int ego_set_threads(int n)
{
#ifdef _OPENMP
    const int before = omp_get_max_threads();
    if (n >= 1) omp_set_num_threads(n);
    return before;
#else
    (void)n;
    return 1;
#endif
}

/* Neighbour ids of vertex v (count returned; at most 3^ndim - 1). */
int ego_neighbours(const void* f, int dtype, int ndim, const int64_t* dims, int64_t v, int64_t* out)
{
    grid_t g;
    if (setup(&g, f, dtype, ndim, dims, 0) != EGO_OK || v < 0 || v >= g.N) return -1;
    int64_t coords[EGO_MAXNB][EGO_MAXDIM];
    return neighbours(&g, v, out, coords);
}

/* One vertex: gradient target, beta+ and the reps (highest vertex of each
 * upper-link component, in ascending vertex order). */
int ego_vertex(const void* f, int dtype, int ndim, const int64_t* dims, int minima, int64_t v,
               int64_t* ptr_out, int64_t* reps_out)
{
    grid_t g;
    if (setup(&g, f, dtype, ndim, dims, minima) != EGO_OK || v < 0 || v >= g.N) return -1;
    int64_t reps[EGO_MAXNB];
    int b = classify_vertex(&g, v, ptr_out, reps);
    /* ascending order for a canonical result */
    for (int i = 1; i < b; ++i)
        for (int j = i; j > 0 && reps[j - 1] > reps[j]; --j) {
            int64_t t = reps[j];
            reps[j] = reps[j - 1];
            reps[j - 1] = t;
        }
    if (reps_out) memcpy(reps_out, reps, sizeof(int64_t) * (size_t)b);
    return b;
}

/* Label of one vertex: walk the gradient until it stops at a maximum. */
int64_t ego_label_of(const void* f, int dtype, int ndim, const int64_t* dims, int minima, int64_t v)
{
    grid_t g;
    if (setup(&g, f, dtype, ndim, dims, minima) != EGO_OK || v < 0 || v >= g.N) return -1;
    int64_t reps[EGO_MAXNB];
    for (;;) {
        int64_t nxt;
        classify_vertex(&g, v, &nxt, reps);
        if (nxt == v) return v;
        v = nxt;
    }
}

/* Whole-field pass 1: per-vertex gradient target and beta+.
 * Returns EGO_ERR_NAN if any sample is NaN (outputs then undefined). */
int ego_classify(const void* f, int dtype, int ndim, const int64_t* dims, int minima,
                 int32_t* ptr, int32_t* beta)
{
    grid_t g;
    int st = setup(&g, f, dtype, ndim, dims, minima);
    if (st != EGO_OK) return st;
    for (int64_t v = 0; v < g.N; ++v)
        if (is_nan(&g, v)) return EGO_ERR_NAN;
    int64_t N = g.N;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t v = 0; v < N; ++v) {
        int64_t reps[EGO_MAXNB], p;
        int b = classify_vertex(&g, v, &p, reps);
        ptr[v] = (int32_t)p;
        beta[v] = b;
    }
    return EGO_OK;
}

/* Whole-field pass 2: labels by walking ptr to its fixed point.  Each walk
 * stops at the first vertex whose label is already known and writes the
 * label back along the walked path (memoisation). */
int ego_labels(const int32_t* ptr, int64_t N, int32_t* labels)
{
    int32_t* path = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
    if (!path) return EGO_ERR_NOMEM;
    for (int64_t v = 0; v < N; ++v) labels[v] = -1;
    for (int64_t v = 0; v < N; ++v) {
        if (labels[v] >= 0) continue;
        int64_t len = 0;
        int32_t u = (int32_t)v;
        while (labels[u] < 0 && ptr[u] != u) {
            path[len++] = u;
            u = ptr[u];
        }
        int32_t m = labels[u] >= 0 ? labels[u] : u;
        labels[u] = m;
        for (int64_t i = 0; i < len; ++i) labels[path[i]] = m;
    }
    free(path);
    return EGO_OK;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Whole-field pass 3: arcs.  For each saddle (ascending list), the set of
 * labels of its reps, sorted: CSR offsets[n_sad+1] and arc_maxima.
 * Two sweeps over the saddles (count, then fill) keep the memory bounded.
 * Returns EGO_ERR_CAPACITY (with *n_arc = required count) if cap_arc is too
 * small. */
static int saddle_row(const grid_t* g, const int32_t* labels, int64_t s, int32_t* row)
{
    int64_t reps[EGO_MAXNB], p;
    int b = classify_vertex(g, s, &p, reps);
    for (int j = 0; j < b; ++j) row[j] = labels[reps[j]];
    qsort(row, (size_t)b, sizeof(int32_t), cmp_i32);
    int len = 0;
    for (int j = 0; j < b; ++j)
        if (len == 0 || row[len - 1] != row[j]) row[len++] = row[j];
    return len;
}

int ego_arcs(const void* f, int dtype, int ndim, const int64_t* dims, int minima,
             const int32_t* labels, const int32_t* saddles, int64_t n_sad,
             int32_t* offsets, int32_t* arc_maxima, int64_t cap_arc, int64_t* n_arc)
{
    grid_t g;
    int st = setup(&g, f, dtype, ndim, dims, minima);
    if (st != EGO_OK) return st;
    /* sweep 1: row lengths into offsets[i+1] */
    offsets[0] = 0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n_sad; ++i) {
        int32_t row[EGO_MAXNB];
        offsets[i + 1] = saddle_row(&g, labels, saddles[i], row);
    }
    int64_t total = 0;
    for (int64_t i = 0; i < n_sad; ++i) {
        total += offsets[i + 1];
        offsets[i + 1] = (int32_t)total;
    }
    *n_arc = total;
    if (total > cap_arc) return EGO_ERR_CAPACITY;
    /* sweep 2: fill the rows */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n_sad; ++i) {
        int32_t row[EGO_MAXNB];
        int len = saddle_row(&g, labels, saddles[i], row);
        memcpy(arc_maxima + offsets[i], row, sizeof(int32_t) * (size_t)len);
    }
    return EGO_OK;
}

/* Whole-field pass 4: gradient-path geometry (Alg. 2).  For each saddle (the
 * ascending list) and each of its upper-link components, in ascending order of
 * the component's smallest vertex id: the path s, rep, grad(rep), ..., m.
 * pair_offsets[i] .. pair_offsets[i+1] index the paths of saddle i;
 * path_offsets (CSR over all paths) index vertices.  Two sweeps (count, then
 * fill).  Returns EGO_ERR_CAPACITY with the required counts in *n_pairs and
 * *n_vertices if a capacity is too small. */
typedef struct {
    int64_t rep, lo;
} comp_t;

static int cmp_comp(const void* a, const void* b)
{
    int64_t x = ((const comp_t*)a)->lo, y = ((const comp_t*)b)->lo;
    return (x > y) - (x < y);
}

static int saddle_paths(const grid_t* g, int64_t s, comp_t* comps)
{
    int64_t reps[EGO_MAXNB], mins[EGO_MAXNB], p;
    int b = classify_vertex_mins(g, s, &p, reps, mins);
    for (int j = 0; j < b; ++j) {
        comps[j].rep = reps[j];
        comps[j].lo = mins[j];
    }
    qsort(comps, (size_t)b, sizeof(comp_t), cmp_comp);
    return b;
}

static int64_t path_length(const int32_t* ptr, int64_t r)
{
    int64_t len = 2; /* s and r */
    while (ptr[r] != r) {
        r = ptr[r];
        ++len;
    }
    return len;
}

int ego_paths(const void* f, int dtype, int ndim, const int64_t* dims, int minima, const int32_t* ptr,
              const int32_t* saddles, int64_t n_sad, int32_t* pair_offsets, int32_t* path_offsets,
              int64_t cap_pairs, int32_t* vertices, int64_t cap_vertices, int64_t* n_pairs,
              int64_t* n_vertices)
{
    grid_t g;
    int st = setup(&g, f, dtype, ndim, dims, minima);
    if (st != EGO_OK) return st;
    int64_t* vcount = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_sad > 0 ? n_sad : 1));
    if (!vcount) return EGO_ERR_NOMEM;
    /* sweep 1: components and path vertices per saddle */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_sad; ++i) {
        comp_t comps[EGO_MAXNB];
        int b = saddle_paths(&g, saddles[i], comps);
        int64_t nv = 0;
        for (int j = 0; j < b; ++j) nv += path_length(ptr, comps[j].rep);
        pair_offsets[i + 1] = b;
        vcount[i] = nv;
    }
    pair_offsets[0] = 0;
    int64_t tp = 0, tv = 0;
    for (int64_t i = 0; i < n_sad; ++i) {
        tp += pair_offsets[i + 1];
        pair_offsets[i + 1] = (int32_t)tp;
        const int64_t nv = vcount[i];
        vcount[i] = tv; /* first vertex of the saddle's paths */
        tv += nv;
    }
    *n_pairs = tp;
    *n_vertices = tv;
    if (tp > cap_pairs || tv > cap_vertices) {
        free(vcount);
        return EGO_ERR_CAPACITY;
    }
    /* sweep 2: fill */
    path_offsets[0] = 0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_sad; ++i) {
        comp_t comps[EGO_MAXNB];
        int b = saddle_paths(&g, saddles[i], comps);
        int64_t at = vcount[i];
        for (int j = 0; j < b; ++j) {
            int64_t r = comps[j].rep;
            vertices[at++] = saddles[i];
            vertices[at++] = (int32_t)r;
            while (ptr[r] != r) {
                r = ptr[r];
                vertices[at++] = (int32_t)r;
            }
            path_offsets[pair_offsets[i] + j + 1] = (int32_t)at;
        }
    }
    free(vcount);
    return EGO_OK;
}
