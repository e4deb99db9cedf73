// eg_arcs.hip -- stage (d) and the canonical outputs, for one field or a batch.
//
// Classification leaves the maxima and the saddles as two row-padded bitmasks.
// Here:
//   1. k_mask_count / k_scan_rows / k_mask_emit: an order-preserving
//      compaction of each mask (block counts, their scan, then every block
//      expands its words), so maxima[] and saddles[] come out in ascending
//      vertex order without a sort;
//   2. k_arc_count: for every saddle, the highest vertex of each upper-link
//      component (UpperLinkRep, Sec. 3.4), the label it reaches, and the
//      number of distinct labels: the saddle's arcs (arcs form a set,
//      Sec. 2); the smallest are kept in registers and stored (four in 2D
//      and 3D, eight from 4D on);
//   3. k_scan_rows / k_arc_write: the CSR offsets from a scan of the counts,
//      then the arcs (a saddle with more distinct arcs than were stored,
//      rare, finds the rest in ascending order by one more pass over its
//      components per arc);
//   4. k_finalize: status and counts into the header.
// No step uses an atomic: every position comes from a scan, so results do
// not depend on scheduling.
//
// Every kernel is written against a field selector: OneField (the field is
// the kernel argument, blocks are blockIdx.x) or BatchFields (the plan lists
// the fields; a flat grid is split over them in proportion to their size).
#include <algorithm>

#include "eg_internal.h"
#include "eg_rows.h"
#include "eg_link.h"

namespace eg {

// ------------------------------------------------------------------ selectors

struct OneField {
    ArcArgs a;
    // the field of this block, the block's index among the field's blocks and
    // their number
    __device__ __forceinline__ const ArcArgs& locate(uint32_t& blk, uint32_t& nb) const
    {
        blk = blockIdx.x;
        nb = gridDim.x;
        return a;
    }
    // kernels with one block per field
    __device__ __forceinline__ const ArcArgs& field() const { return a; }
};

struct BatchFields {
    EG_GPTR(const BatchPlan) plan;
    __device__ __forceinline__ const ArcArgs& locate(uint32_t& blk, uint32_t& nb) const
    {
        const EG_GPTR(BatchField) fs = plan->fields;
        const int64_t b = blockIdx.x;
        int lo = 0, hi = plan->count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (fs[mid].arc_base <= b)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int f = __builtin_amdgcn_readfirstlane(lo);
        blk = (uint32_t)(b - fs[f].arc_base);
        nb = (uint32_t)fs[f].arc.arc_blocks;
        return fs[f].arc;
    }
    __device__ __forceinline__ const ArcArgs& field() const { return plan->fields[blockIdx.x].arc; }
};

// ------------------------------------------------------------------ helpers

// Contiguous chunk [lo, hi) of [0, n) for block blk of nb: whole rounds of
// 256 items, so every block but the last has full rounds.
__device__ __forceinline__ void chunk(uint32_t n, uint32_t nb, uint32_t blk, uint32_t& lo, uint32_t& hi)
{
    uint32_t per = (uint32_t)(((uint64_t)n + nb - 1u) / nb);
    per = (per + 255u) & ~255u;
    if (per == 0) per = 256u;
    const uint64_t l = (uint64_t)blk * per;
    lo = (uint32_t)(l < n ? l : n);
    const uint64_t h = (uint64_t)lo + per;
    hi = (uint32_t)(h < n ? h : n);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan of x over the 256 threads of the block; total gets the sum.
// Uses tmp[0..3]; every thread must call it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* tmp, uint32_t& total)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int k = 0; k < w; ++k) pre += tmp[k];
    total = tmp[0] + tmp[1] + tmp[2] + tmp[3];
    __syncthreads();
    return pre + inc - x;
}

__device__ __forceinline__ uint32_t block_sum(uint32_t x, uint32_t* tmp)
{
    uint32_t total;
    block_excl_scan(x, tmp, total);
    return total;
}

__device__ __forceinline__ uint32_t saddle_count(const ArcArgs& A)
{
    const uint32_t n = A.ctr[C_NSAD];
    return n < A.cap_sad ? n : A.cap_sad;
}

// ------------------------------------------------------------------ masks

template <class Sel>
__global__ __launch_bounds__(256) void k_mask_count(Sel sel)
{
    __shared__ uint32_t tmp[4];
    uint32_t blk, nb;
    const ArcArgs A = sel.locate(blk, nb);  // a copy: loop loads cannot alias it
    uint32_t lo, hi;
    chunk((uint32_t)A.words, nb, blk, lo, hi);
    uint32_t cm = 0, cs = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) {
        cm += (uint32_t)__popcll(A.mmask[i]);
        cs += (uint32_t)__popcll(A.smask[i]);
    }
    cm = block_sum(cm, tmp);
    cs = block_sum(cs, tmp);
    if (threadIdx.x == 0) {
        A.bsum[blk] = cm;
        A.bsum[kArcBlocks + blk] = cs;
    }
}

// Exclusive scan, in place, of rows `row` and `row + 1` of a field's block
// counts (nb <= kArcBlocks entries each); the row totals go to the counter
// slots.  One block of 1024 threads per field, kArcBlocks / 1024 entries per
// thread staged through LDS.
template <class Sel>
__global__ __launch_bounds__(1024) void k_scan_rows(Sel sel, int row, int slot0, int slot1)
{
    constexpr int PER = kArcBlocks / 1024;
    __shared__ uint32_t buf[kArcBlocks];
    __shared__ uint32_t wsum[16];
    const ArcArgs A = sel.field();
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int nb = A.arc_blocks;
    for (int r = 0; r < 2; ++r) {
        EG_GPTR(uint32_t) a = A.bsum + (row + r) * kArcBlocks;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = k * 1024 + tid;
            buf[i] = i < nb ? a[i] : 0u;
        }
        __syncthreads();
        uint32_t x[PER], sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            x[k] = buf[tid * PER + k];
            sum += x[k];
        }
        const uint32_t inc = wave_incl_scan(sum);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        if (w == 0) {
            uint32_t y = lane < 16 ? wsum[lane] : 0u;
            y = wave_incl_scan(y);
            if (lane < 16) wsum[lane] = y;
        }
        __syncthreads();
        uint32_t ex = (w > 0 ? wsum[w - 1] : 0u) + inc - sum;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            buf[tid * PER + k] = ex;
            ex += x[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = k * 1024 + tid;
            if (i < nb) a[i] = buf[i];
        }
        if (tid == 0) A.ctr[r == 0 ? slot0 : slot1] = wsum[15];
        __syncthreads();
    }
}

// Write the vertex ids of the set bits of one round of 256 words (one per
// thread) to out[run + j], j < total (entries at or past cap are dropped);
// local is the exclusive count of set bits before this thread's word.  The
// ids are staged in LDS so that the global stores are whole-wave and
// contiguous; a round with more ids than the stage (a very dense mask) writes
// directly.  Every thread of the block must call it.
constexpr int kStage = 4096;
__device__ __forceinline__ void emit_round(uint64_t word, uint32_t local, uint32_t total, int32_t vbase,
                                           uint32_t run, EG_GPTR(int32_t) out, uint32_t cap, int32_t* stage)
{
    if (total == 0) return;
    if (total <= (uint32_t)kStage) {
        for (uint32_t j = local; word; ++j) {
            stage[j] = vbase + (__ffsll((unsigned long long)word) - 1);
            word &= word - 1ull;
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < total; j += 256)
            if (run + j < cap) out[run + j] = stage[j];
        __syncthreads();
    } else {
        for (uint32_t p = run + local; word; ++p) {
            if (p < cap) out[p] = vbase + (__ffsll((unsigned long long)word) - 1);
            word &= word - 1ull;
        }
    }
}

template <class Sel>
__global__ __launch_bounds__(256) void k_mask_emit(Sel sel)
{
    __shared__ uint32_t tmp[4];
    __shared__ int32_t stage[kStage];
    uint32_t blk, nb;
    const ArcArgs A = sel.locate(blk, nb);  // a copy: loop loads cannot alias it
    uint32_t lo, hi;
    chunk((uint32_t)A.words, nb, blk, lo, hi);
    uint32_t rm = A.bsum[blk], rs = A.bsum[kArcBlocks + blk];
    const uint32_t XW = (uint32_t)A.XW, X = (uint32_t)A.X;
    for (uint32_t base = lo; base < hi; base += 256) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t m = i < hi ? A.mmask[i] : 0ull;
        const uint64_t sd = i < hi ? A.smask[i] : 0ull;
        uint32_t tm, ts;
        const uint32_t lm = block_excl_scan((uint32_t)__popcll(m), tmp, tm);
        const uint32_t ls = block_excl_scan((uint32_t)__popcll(sd), tmp, ts);
        const uint32_t row = i / XW, xw = i - row * XW;
        const int32_t vbase = (int32_t)(row * X + xw * 64u);
        emit_round(m, lm, tm, vbase, rm, A.maxima, A.cap_max, stage);
        emit_round(sd, ls, ts, vbase, rs, A.saddles, A.cap_sad, stage);
        rm += tm;
        rs += ts;
    }
}

// ------------------------------------------------------------------ arcs

// The neighbourhood of saddle v: order keys (0 outside the grid, below every
// vertex) and linear offsets of the K Freudenthal rows, and the upper-link
// mask (Alg. 1, Sec. 3.3).
// From 4D on (30 to 126 rows) the rows' offsets come from a per-block table
// in LDS when a rep is found (only the rep's offset is needed).  In 6D (126
// rows) the keys are not kept either: holding them costs more registers, and
// waves, than reloading the few keys of one component when its rep is sought.
template <int NDIM>
constexpr bool kLazyNbhd = NDIM >= 6;
template <int NDIM>
constexpr bool kOffsInLds = NDIM >= 4;

template <int NDIM, bool MINMODE>
struct Nbhd {
    static constexpr int K = Rows<NDIM>::K;
    uint32_t us[kLazyNbhd<NDIM> ? 1 : K];
    int offs[kOffsInLds<NDIM> ? 1 : K];
    Mask<NDIM> up;
    EG_GPTR(const uint32_t) keys;  // the order keys (lazy neighbourhoods)
};

// Linear offset of every row, per block (lazy neighbourhoods).
template <int NDIM>
__device__ __forceinline__ int* row_offsets()
{
    __shared__ int s_off[Rows<NDIM>::K];
    return s_off;
}

template <int NDIM, bool MINMODE>
__device__ __forceinline__ void load_nbhd(const ArcArgs& A, int v, Nbhd<NDIM, MINMODE>& nb)
{
    constexpr Rows<NDIM> R = make_rows_ce<NDIM>();
    constexpr int K = Rows<NDIM>::K;
    int c[NDIM], st[NDIM];
    {
        int rem = v, stride = 1;
#pragma unroll
        for (int i = NDIM - 1; i >= 0; --i) {
            const int d = A.dims[i];
            c[i] = rem % d;
            rem /= d;
            st[i] = stride;
            stride *= d;
        }
    }
    // keys stored by classification already carry the reversal of the
    // minimum graph
    const bool stored = A.keys != nullptr;
    const uint32_t uv = stored ? A.keys[v] : mode_key<MINMODE>(A.f[v]);
    nb.up = 0;
    nb.keys = A.keys;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        bool in = true;
        int off = 0;
#pragma unroll
        for (int i = 0; i < NDIM; ++i) {
            const int d = R.d[j][i];
            if (d != 0) {
                in = in && (unsigned)(c[i] + d) < (unsigned)A.dims[i];
                off += d * st[i];
            }
        }
        uint32_t u;
        if constexpr (NDIM >= 4 && !kLazyNbhd<NDIM>) {
            // no branch around the load: every row's load is in flight at once
            const int w = in ? v + off : v;
            const uint32_t x = stored ? A.keys[w] : mode_key<MINMODE>(A.f[w]);
            u = in ? x : 0u;
        } else {
            u = !in ? 0u : stored ? A.keys[v + off] : mode_key<MINMODE>(A.f[v + off]);
        }
        if constexpr (!kLazyNbhd<NDIM>) nb.us[j] = u;
        if constexpr (!kOffsInLds<NDIM>) nb.offs[j] = off;
        const bool wins_tie = (j >= K / 2) != MINMODE;
        nb.up |= Mask<NDIM>(wins_tie ? (u >= uv) : (u > uv)) << j;
    }
}

// Calls f(rep) for every upper-link component of saddle v, with rep the
// component's highest vertex (UpperLinkRep, Sec. 3.4), found by scanning in
// the order in which the later of two equal vertices wins.  Components are
// grown from the lowest remaining row (a bit-parallel BFS over the link
// edges; from 4D on by set algebra on the link's rows, eg_link.h); rows are
// in linear-index order, so components come in ascending order of their
// smallest vertex.
template <int NDIM, bool MINMODE, class F>
__device__ __forceinline__ void for_each_rep(int v, const Nbhd<NDIM, MINMODE>& nb, const Mask<NDIM>* s_adj, F&& f)
{
    constexpr int K = Rows<NDIM>::K;
    for (Mask<NDIM> rem = nb.up; rem != 0;) {
        Mask<NDIM> comp;
        if constexpr (NDIM >= 4)
            comp = link_component<NDIM>(rem);
        else
            comp = closure(rem & (~rem + 1), rem, s_adj);
        rem &= ~comp;
        uint32_t best_u = 0;
        int best_off = 0;
        if constexpr (kLazyNbhd<NDIM>) {
            // the component's rows in scan order: ascending rows, descending in
            // the minimum graph; every row of the mask lies in the grid
            const int* s_off = row_offsets<NDIM>();
            for (Mask<NDIM> c = comp; c != 0;) {
                const int j = MINMODE ? highest_bit(c) : lowest_bit(c);
                c &= ~(Mask<NDIM>(1) << j);
                const int off = s_off[j];
                const uint32_t u = nb.keys[v + off];
                if (u >= best_u) {
                    best_u = u;
                    best_off = off;
                }
            }
        } else if constexpr (kOffsInLds<NDIM>) {
            int best_j = 0;
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const int j = MINMODE ? K - 1 - s : s;
                if ((uint32_t)(comp >> j) & 1u && nb.us[j] >= best_u) {
                    best_u = nb.us[j];
                    best_j = j;
                }
            }
            best_off = row_offsets<NDIM>()[best_j];
        } else {
#pragma unroll
            for (int s = 0; s < K; ++s) {
                const int j = MINMODE ? K - 1 - s : s;
                if ((uint32_t)(comp >> j) & 1u && nb.us[j] >= best_u) {
                    best_u = nb.us[j];
                    best_off = nb.offs[j];
                }
            }
        }
        f(v + best_off);
    }
}

// f(label) for every component: the label its rep reaches.
template <int NDIM, bool MINMODE, class F>
__device__ __forceinline__ void for_each_arc_label(const ArcArgs& A, int v, const Nbhd<NDIM, MINMODE>& nb,
                                                   const Mask<NDIM>* s_adj, F&& f)
{
    for_each_rep<NDIM, MINMODE>(v, nb, s_adj, [&](int rep) { f((uint32_t)A.lab[rep]); });
}

// The S smallest distinct arc labels of a saddle, ascending (unused entries
// ~0u; labels are vertex ids below 2^31).  `more` is set when the saddle has
// further distinct labels above lo[S-1].  S = 4 in 2D/3D (at most 3 and 6
// components), 8 from 4D on, where more components are common.
template <int NDIM>
struct ArcList {
    static constexpr int S = NDIM >= 4 ? 8 : 4;
    uint32_t lo[S];
    bool more;
};

template <int NDIM, bool MINMODE>
__device__ __forceinline__ ArcList<NDIM> first_arcs(const ArcArgs& A, int v, const Nbhd<NDIM, MINMODE>& nb,
                                                    const Mask<NDIM>* s_adj, int& beta)
{
    constexpr int S = ArcList<NDIM>::S;
    ArcList<NDIM> r;
#pragma unroll
    for (int k = 0; k < S; ++k) r.lo[k] = ~0u;
    r.more = false;
    beta = 0;
    for_each_arc_label<NDIM, MINMODE>(A, v, nb, s_adj, [&](uint32_t L) {
        ++beta;
        bool dup = false;
#pragma unroll
        for (int k = 0; k < S; ++k) dup |= L == r.lo[k];
        if (dup) return;
        if (L > r.lo[S - 1]) {  // a distinct label above a full list
            r.more = true;
            return;
        }
        if (r.lo[S - 1] != ~0u) r.more = true;  // the list is full: its largest moves out
        r.lo[S - 1] = L;
        // one insertion step keeps the list sorted
#pragma unroll
        for (int k = S - 1; k > 0; --k)
            if (r.lo[k] < r.lo[k - 1]) {
                const uint32_t t = r.lo[k - 1];
                r.lo[k - 1] = r.lo[k];
                r.lo[k] = t;
            }
    });
    return r;
}

// Distinct labels above `last`, ascending, one pass over the components
// each: for saddles with more than four distinct arcs (rare).  Calls
// emit(k, label) for the k-th of them and returns their number.
template <int NDIM, bool MINMODE, class E>
__device__ __forceinline__ uint32_t labels_above(const ArcArgs& A, int v, const Nbhd<NDIM, MINMODE>& nb,
                                                 const Mask<NDIM>* s_adj, uint32_t last, E&& emit)
{
    uint32_t k = 0;
    for (;;) {
        uint32_t next = ~0u;
        for_each_arc_label<NDIM, MINMODE>(A, v, nb, s_adj, [&](uint32_t L) {
            if (L > last && L < next) next = L;
        });
        if (next == ~0u) return k;
        emit(k, next);
        ++k;
        last = next;
    }
}

template <int NDIM>
__device__ __forceinline__ void load_adj(const ArcArgs& A, Mask<NDIM>* s_adj)
{
    constexpr int K = Rows<NDIM>::K;
    if constexpr (NDIM < 4) {  // from 4D on components come from set algebra
        const Mask<NDIM>* t = adj_table<NDIM>();
        for (int i = threadIdx.x; i < K; i += blockDim.x) s_adj[i] = t[i];
    }
    if constexpr (kOffsInLds<NDIM>) {
        constexpr Rows<NDIM> R = make_rows_ce<NDIM>();
        int* s_off = row_offsets<NDIM>();
        int st[NDIM];
        st[NDIM - 1] = 1;
#pragma unroll
        for (int i = NDIM - 2; i >= 0; --i) st[i] = st[i + 1] * A.dims[i + 1];
        for (int j = threadIdx.x; j < K; j += blockDim.x) {
            int off = 0;
#pragma unroll
            for (int i = 0; i < NDIM; ++i) off += R.d[j][i] * st[i];
            s_off[j] = off;
        }
    }
    __syncthreads();
}

// Distinct-arc count, beta and the first four (eight from 4D on) arcs of every saddle of the
// block's chunk; the block's sums of both counts go to rows 2 and 3.
template <int NDIM, bool MINMODE>
__device__ __forceinline__ void arc_count_body(const ArcArgs& A, uint32_t blk, uint32_t nb, Mask<NDIM>* s_adj,
                                               uint32_t* tmp)
{
    load_adj<NDIM>(A, s_adj);
    uint32_t lo, hi;
    chunk(saddle_count(A), nb, blk, lo, hi);
    const int tid = threadIdx.x;
    uint32_t sc = 0, sb = 0;
    for (uint32_t i = lo + tid; i < hi; i += 256) {
        // saddle ids come from the compaction; the check keeps a stage run
        // on a workspace without classification inside the grid
        const int v = min(max(A.saddles[i], 0), A.N - 1);
        Nbhd<NDIM, MINMODE> h;
        load_nbhd<NDIM, MINMODE>(A, v, h);
        int beta;
        const ArcList<NDIM> r = first_arcs<NDIM, MINMODE>(A, v, h, s_adj, beta);
        constexpr int S = ArcList<NDIM>::S;
        uint32_t n = 0;
#pragma unroll
        for (int k = 0; k < S; ++k) n += r.lo[k] != ~0u;
        if (r.more) n += labels_above<NDIM, MINMODE>(A, v, h, s_adj, r.lo[S - 1], [](uint32_t, uint32_t) {});
        if (A.beta) A.beta[i] = beta;
        A.offsets[i + 1] = (int32_t)n;  // the count until k_arc_write turns it into an offset
        A.atmp[i] = make_uint4(r.lo[0], r.lo[1], r.lo[2], r.lo[3]);
        if constexpr (S > 4) A.atmp[A.cap_sad + i] = make_uint4(r.lo[4], r.lo[5], r.lo[6], r.lo[7]);
        sc += n;
        sb += (uint32_t)beta;
    }
    sc = block_sum(sc, tmp);
    sb = block_sum(sb, tmp);
    if (tid == 0) {
        A.bsum[2 * kArcBlocks + blk] = sc;
        A.bsum[3 * kArcBlocks + blk] = sb;
    }
}

template <int NDIM, bool MINMODE>
__device__ __forceinline__ void arc_write_body(const ArcArgs& A, uint32_t blk, uint32_t nb, Mask<NDIM>* s_adj,
                                               uint32_t* tmp)
{
    load_adj<NDIM>(A, s_adj);
    uint32_t lo, hi;
    chunk(saddle_count(A), nb, blk, lo, hi);
    const int tid = threadIdx.x;
    if (blk == 0 && tid == 0) A.offsets[0] = 0;
    uint32_t run = A.bsum[2 * kArcBlocks + blk];
    for (uint32_t base = lo; base < hi; base += 256) {
        const uint32_t i = base + tid;
        const bool valid = i < hi;
        const uint32_t n = valid ? (uint32_t)A.offsets[i + 1] : 0u;
        uint32_t total;
        const uint32_t pos = run + block_excl_scan(n, tmp, total);
        if (valid) {
            const uint4 t = A.atmp[i];
            const uint32_t a4[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k)
                if (k < n && pos + k < A.cap_arc) A.arcs[pos + k] = (int32_t)a4[k];
            constexpr int S = ArcList<NDIM>::S;
            uint32_t last = t.w;
            if constexpr (S > 4) {
                // the next four stored arcs
                if (n > 4) {
                    const uint4 u = A.atmp[A.cap_sad + i];
                    const uint32_t b4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (uint32_t k = 0; k < 4; ++k)
                        if (4 + k < n && pos + 4 + k < A.cap_arc) A.arcs[pos + 4 + k] = (int32_t)b4[k];
                    last = u.w;
                }
            }
            if (n > (uint32_t)S) {
                // past the stored arcs: ascending selection over the components
                const int v = min(max(A.saddles[i], 0), A.N - 1);
                Nbhd<NDIM, MINMODE> h;
                load_nbhd<NDIM, MINMODE>(A, v, h);
                labels_above<NDIM, MINMODE>(A, v, h, s_adj, last, [&](uint32_t k, uint32_t L) {
                    if (pos + S + k < A.cap_arc) A.arcs[pos + S + k] = (int32_t)L;
                });
            }
            A.offsets[i + 1] = (int32_t)(pos + n);
        }
        run += total;
    }
}

// Four waves per SIMD for the 5D rows, in the arc and the path kernels alike
// (the compiler's own choice, 133 to 150 registers, leaves three and stalls
// on the gathers; the few spilled values cost less); 6D keeps its registers,
// since there the spills cost more.
template <int NDIM>
constexpr int kArcWaves = NDIM == 5 ? 4 : 1;

template <int NDIM, bool MINMODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kArcWaves<NDIM>, 8))) void k_arc_count(
    OneField sel)
{
    __shared__ Mask<NDIM> s_adj[Rows<NDIM>::K];
    __shared__ uint32_t tmp[4];
    uint32_t blk, nb;
    const ArcArgs A = sel.locate(blk, nb);  // a copy: loop loads cannot alias it
    arc_count_body<NDIM, MINMODE>(A, blk, nb, s_adj, tmp);
}

template <int NDIM, bool MINMODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kArcWaves<NDIM>, 8))) void k_arc_write(
    OneField sel)
{
    __shared__ Mask<NDIM> s_adj[Rows<NDIM>::K];
    __shared__ uint32_t tmp[4];
    uint32_t blk, nb;
    const ArcArgs A = sel.locate(blk, nb);  // a copy: loop loads cannot alias it
    arc_write_body<NDIM, MINMODE>(A, blk, nb, s_adj, tmp);
}

// Batches hold 2D and 3D fields of either graph: the body is chosen per
// field (a uniform branch).
template <bool WRITE>
__global__ __launch_bounds__(256) void k_arc_batched(BatchFields sel)
{
    __shared__ uint64_t s_adj[14];
    __shared__ uint32_t tmp[4];
    uint32_t blk, nb;
    const ArcArgs A = sel.locate(blk, nb);  // a copy: loop loads cannot alias it
    const int kind = __builtin_amdgcn_readfirstlane((A.ndim == 3 ? 2 : 0) + (A.minima ? 1 : 0));
#define EG_BODY(ND, MM)                                                  \
    if (WRITE)                                                           \
        arc_write_body<ND, MM>(A, blk, nb, s_adj, tmp);                  \
    else                                                                 \
        arc_count_body<ND, MM>(A, blk, nb, s_adj, tmp);
    switch (kind) {
        case 0: EG_BODY(2, false) break;
        case 1: EG_BODY(2, true) break;
        case 2: EG_BODY(3, false) break;
        default: EG_BODY(3, true) break;
    }
#undef EG_BODY
}

// ------------------------------------------------------------------ paths

template <bool MINMODE>
__device__ __forceinline__ uint32_t key_of(const ArcArgs& A, int x)
{
    return A.keys != nullptr ? A.keys[x] : mode_key<MINMODE>(A.f[x]);
}

// The walk of Alg. 2 from rep: visit(r) for rep and every vertex after it, up
// to the maximum (ptr(m) = m).  Every step must stay in the grid and rise in
// the order; a pointer that does not (out->ptr not holding this field's
// pointers) ends the walk and returns false, so no input can make it leave
// the grid or loop.
template <bool MINMODE, class V>
__device__ __forceinline__ bool walk(const ArcArgs& A, EG_GPTR(const int32_t) const ptr, int r, V&& visit)
{
    visit(r);
    uint32_t ur = key_of<MINMODE>(A, r);
    for (;;) {
        const int q = ptr[r];
        if (q == r) return true;
        if ((unsigned)q >= (unsigned)A.N) return false;
        const uint32_t uq = key_of<MINMODE>(A, q);
        if (!(uq > ur || (uq == ur && (MINMODE ? q < r : q > r)))) return false;
        visit(q);
        r = q;
        ur = uq;
    }
}

__global__ void k_path_reset(OneField sel)
{
    if (threadIdx.x == 0) sel.field().ctr[C_PBAD] = 0;
}

// Paths and path vertices of every saddle of the block's chunk (kept for the
// write pass in the workspace), block sums into rows 0 and 1.
template <int NDIM, bool MINMODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kArcWaves<NDIM>, 8))) void k_path_count(
    OneField sel, PathArgs P)
{
    __shared__ Mask<NDIM> s_adj[Rows<NDIM>::K];
    __shared__ uint32_t tmp[4];
    uint32_t blk, nb;
    const ArcArgs A = sel.locate(blk, nb);  // a copy: loop loads cannot alias it
    load_adj<NDIM>(A, s_adj);
    uint32_t lo, hi;
    chunk(saddle_count(A), nb, blk, lo, hi);
    uint32_t sp = 0, sv = 0;
    bool bad = false;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += 256) {
        const int v = A.saddles[i];
        uint32_t np = 0, nv = 0;
        if ((unsigned)v < (unsigned)A.N) {
            Nbhd<NDIM, MINMODE> h;
            load_nbhd<NDIM, MINMODE>(A, v, h);
            for_each_rep<NDIM, MINMODE>(v, h, s_adj, [&](int rep) {
                ++np;
                ++nv;  // the saddle, then rep .. maximum
                bad |= !walk<MINMODE>(A, P.ptr, rep, [&](int) { ++nv; });
            });
        } else {
            bad = true;
        }
        A.atmp[i] = make_uint4(np, nv, 0u, 0u);
        sp += np;
        sv += nv;
    }
    if (__ballot(bad) != 0 && __lane_id() == 0) atomicOr(&A.ctr[C_PBAD], 1u);
    sp = block_sum(sp, tmp);
    sv = block_sum(sv, tmp);
    if (threadIdx.x == 0) {
        A.bsum[blk] = sp;
        A.bsum[kArcBlocks + blk] = sv;
    }
}

template <int NDIM, bool MINMODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kArcWaves<NDIM>, 8))) void k_path_write(
    OneField sel, PathArgs P)
{
    __shared__ Mask<NDIM> s_adj[Rows<NDIM>::K];
    __shared__ uint32_t tmp[4];
    uint32_t blk, nb;
    const ArcArgs A = sel.locate(blk, nb);  // a copy: loop loads cannot alias it
    load_adj<NDIM>(A, s_adj);
    uint32_t lo, hi;
    chunk(saddle_count(A), nb, blk, lo, hi);
    uint32_t runp = A.bsum[blk], runv = A.bsum[kArcBlocks + blk];
    for (uint32_t base = lo; base < hi; base += 256) {
        const uint32_t i = base + threadIdx.x;
        const bool valid = i < hi;
        const uint4 c = valid ? A.atmp[i] : make_uint4(0u, 0u, 0u, 0u);
        uint32_t tp, tv;
        uint32_t pk = runp + block_excl_scan(c.x, tmp, tp);
        uint32_t at = runv + block_excl_scan(c.y, tmp, tv);
        const int v = valid ? A.saddles[i] : 0;
        if (valid) P.pair_offsets[i] = (int32_t)pk;
        if (valid && (unsigned)v < (unsigned)A.N) {
            Nbhd<NDIM, MINMODE> h;
            load_nbhd<NDIM, MINMODE>(A, v, h);
            for_each_rep<NDIM, MINMODE>(v, h, s_adj, [&](int rep) {
                if (pk <= P.cap_paths) P.path_offsets[pk] = (int32_t)at;
                ++pk;
                if (at < P.cap_vertices) P.vertices[at] = v;
                ++at;
                walk<MINMODE>(A, P.ptr, rep, [&](int r) {
                    if (at < P.cap_vertices) P.vertices[at] = r;
                    ++at;
                });
            });
        }
        runp += tp;
        runv += tv;
    }
}

// Closing entries of both offset arrays and the header.
__global__ void k_path_finalize(OneField sel, PathArgs P)
{
    if (threadIdx.x != 0) return;
    const ArcArgs A = sel.field();
    const uint32_t nsad = A.ctr[C_NSAD], np = A.ctr[C_PATHS], nv = A.ctr[C_PVERTS];
    const uint32_t n = nsad < A.cap_sad ? nsad : A.cap_sad;
    P.pair_offsets[n] = (int32_t)np;
    if (np <= P.cap_paths) P.path_offsets[np] = (int32_t)nv;
    const bool short_ = nsad > A.cap_sad || np > P.cap_paths || nv > P.cap_vertices;
    P.header[EG_P_STATUS] = A.ctr[C_NAN] ? EG_ERR_NAN : A.ctr[C_PBAD] ? EG_ERR_ARG : short_ ? EG_ERR_CAPACITY : EG_OK;
    P.header[EG_P_PATHS] = (int32_t)np;
    P.header[EG_P_VERTICES] = (int32_t)nv;
}

template <int NDIM, bool MINMODE>
static void launch_paths_t(const OneField& sel, const PathArgs& p, uint32_t nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_path_reset, dim3(1), dim3(64), 0, s, sel);
    hipLaunchKernelGGL((k_path_count<NDIM, MINMODE>), dim3(nb), dim3(256), 0, s, sel, p);
    hipLaunchKernelGGL(k_scan_rows<OneField>, dim3(1), dim3(1024), 0, s, sel, 0, (int)C_PATHS, (int)C_PVERTS);
    hipLaunchKernelGGL((k_path_write<NDIM, MINMODE>), dim3(nb), dim3(256), 0, s, sel, p);
}

hipError_t launch_paths(const ArcArgs& a, const PathArgs& p, hipStream_t s)
{
    // walks are chains of dependent loads: one block per 256 saddle slots
    // keeps as many in flight as there are saddles
    ArcArgs ap = a;
    const int64_t want = ((int64_t)a.cap_sad + 255) / 256;
    const int64_t nbp = want < kArcBlocks ? want : kArcBlocks;
    if (nbp > ap.arc_blocks) ap.arc_blocks = (int32_t)nbp;
    const OneField sel{ap};
    const uint32_t nb = (uint32_t)ap.arc_blocks;
#define EG_CASE(N)                                    \
    case N:                                           \
        if (a.minima)                                 \
            launch_paths_t<N, true>(sel, p, nb, s);   \
        else                                          \
            launch_paths_t<N, false>(sel, p, nb, s);  \
        break;
    switch (a.ndim) {
        EG_CASE(1)
        EG_CASE(2)
        EG_CASE(3)
        EG_CASE(4)
        EG_CASE(5)
        EG_CASE(6)
        default:
            return hipErrorInvalidValue;
    }
#undef EG_CASE
    hipLaunchKernelGGL(k_path_finalize, dim3(1), dim3(64), 0, s, sel, p);
    return hipGetLastError();
}

// ------------------------------------------------------------------ header

template <class Sel>
__global__ void k_finalize(Sel sel)
{
    if (threadIdx.x != 0) return;
    const ArcArgs A = sel.field();
    const uint32_t* c = A.ctr;
    const int64_t nmax = c[C_NMAX], nsad = c[C_NSAD], narc = c[C_NARC];
    const bool sad_over = nsad > A.cap_sad;
    int status = EG_OK;
    if (c[C_NAN])
        status = EG_ERR_NAN;
    else if (A.last_flag && *A.last_flag)
        status = EG_ERR_UNRESOLVED;
    else if (nmax > A.cap_max || sad_over || narc > A.cap_arc)
        status = EG_ERR_CAPACITY;
    int32_t* h = A.header;
    h[EG_H_STATUS] = status;
    h[EG_H_NMAX] = (int32_t)nmax;
    h[EG_H_NSAD] = (int32_t)nsad;
    // with saddles cut off at the capacity, the arc and pair totals cover
    // only the first cap_sad saddles: unknown
    h[EG_H_NARC] = sad_over ? -1 : (int32_t)narc;
    h[EG_H_NPAIRS] = sad_over ? -1 : (int32_t)c[C_NPAIRS];
    h[EG_H_PASSES] = (int32_t)c[C_PASSES];
    h[EG_H_EXITS] = (int32_t)c[C_NEXIT];
}

// ------------------------------------------------------------------ launchers

// Blocks per field of the stage (d) kernels: one per kArcVertsPerBlock
// vertices; a small field still gets up to 64 blocks (one per 1024 vertices),
// so that its saddles spread over the GPU instead of queueing in a few blocks.
uint32_t arc_blocks(int64_t N)
{
    int64_t b = (N + kArcVertsPerBlock - 1) / kArcVertsPerBlock;
    if (b < 64) b = std::min<int64_t>(64, (N + 1023) / 1024);
    return (uint32_t)(b < 1 ? 1 : b > kArcBlocks ? kArcBlocks : b);
}

ArcArgs arc_args(const float* f, const Grid& g, const eg_out& o, const Work& w)
{
    ArcArgs a{};
    a.f = gptr(f);
    a.keys = gptr<const uint32_t>(w.keys);
    a.lab = gptr<const int32_t>(o.labels);
    a.mmask = gptr<const uint64_t>(w.mmask);
    a.smask = gptr<const uint64_t>(w.smask);
    a.bsum = gptr(w.bsum);
    a.atmp = gptr(w.atmp);
    a.ctr = gptr(w.ctr);
    a.header = gptr(o.header);
    a.maxima = gptr(o.maxima);
    a.saddles = gptr(o.saddles);
    a.beta = gptr(o.saddle_beta);
    a.offsets = gptr(o.arc_offsets);
    a.arcs = gptr(o.arc_maxima);
    a.ndim = g.ndim;
    a.minima = (o.flags & EG_MINIMA) ? 1 : 0;
    a.N = g.N;
    a.X = g.dims[g.ndim - 1];
    a.XW = (a.X + 63) / 64;
    a.words = (int32_t)w.words;
    for (int i = 0; i < EG_MAX_NDIM; ++i) a.dims[i] = i < g.ndim ? g.dims[i] : 1;
    a.cap_max = (uint32_t)o.cap_max;
    a.cap_sad = (uint32_t)o.cap_sad;
    a.cap_arc = (uint32_t)o.cap_arc;
    a.arc_blocks = (int32_t)arc_blocks(g.N);
    return a;
}

template <int NDIM, bool MINMODE>
static void launch_arc_pair(const OneField& sel, uint32_t nb, hipStream_t s)
{
    hipLaunchKernelGGL((k_arc_count<NDIM, MINMODE>), dim3(nb), dim3(256), 0, s, sel);
    hipLaunchKernelGGL(k_scan_rows<OneField>, dim3(1), dim3(1024), 0, s, sel, 2, (int)C_NARC, (int)C_NPAIRS);
    hipLaunchKernelGGL((k_arc_write<NDIM, MINMODE>), dim3(nb), dim3(256), 0, s, sel);
}

hipError_t launch_arcs(const ArcArgs& a, hipStream_t s)
{
    const OneField sel{a};
    const uint32_t nb = (uint32_t)a.arc_blocks;
    hipLaunchKernelGGL(k_mask_count<OneField>, dim3(nb), dim3(256), 0, s, sel);
    hipLaunchKernelGGL(k_scan_rows<OneField>, dim3(1), dim3(1024), 0, s, sel, 0, (int)C_NMAX, (int)C_NSAD);
    hipLaunchKernelGGL(k_mask_emit<OneField>, dim3(nb), dim3(256), 0, s, sel);
#define EG_CASE(N)                                  \
    case N:                                         \
        if (a.minima)                               \
            launch_arc_pair<N, true>(sel, nb, s);   \
        else                                        \
            launch_arc_pair<N, false>(sel, nb, s);  \
        break;
    switch (a.ndim) {
        EG_CASE(1)
        EG_CASE(2)
        EG_CASE(3)
        EG_CASE(4)
        EG_CASE(5)
        EG_CASE(6)
        default:
            return hipErrorInvalidValue;
    }
#undef EG_CASE
    hipLaunchKernelGGL(k_finalize<OneField>, dim3(1), dim3(64), 0, s, sel);
    return hipGetLastError();
}

hipError_t launch_arcs_batched(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    const BatchFields sel{gptr(dplan)};
    const unsigned grid = (unsigned)hplan.total_arc_blocks;
    const unsigned count = (unsigned)hplan.count;
    hipLaunchKernelGGL(k_mask_count<BatchFields>, dim3(grid), dim3(256), 0, s, sel);
    hipLaunchKernelGGL(k_scan_rows<BatchFields>, dim3(count), dim3(1024), 0, s, sel, 0, (int)C_NMAX, (int)C_NSAD);
    hipLaunchKernelGGL(k_mask_emit<BatchFields>, dim3(grid), dim3(256), 0, s, sel);
    hipLaunchKernelGGL(k_arc_batched<false>, dim3(grid), dim3(256), 0, s, sel);
    hipLaunchKernelGGL(k_scan_rows<BatchFields>, dim3(count), dim3(1024), 0, s, sel, 2, (int)C_NARC, (int)C_NPAIRS);
    hipLaunchKernelGGL(k_arc_batched<true>, dim3(grid), dim3(256), 0, s, sel);
    hipLaunchKernelGGL(k_finalize<BatchFields>, dim3(count), dim3(64), 0, s, sel);
    return hipGetLastError();
}

}  // namespace eg
