// eg_rows.h -- compile-time neighbour rows of the Freudenthal tessellation.
//
// Rows are the offsets d != 0 with every component in {0,1} or every
// component in {0,-1} (GridAdjacency, Sec. 3.2 Alg. 1), sorted
// lexicographically with axis 0 (the slowest) most significant: the {0,-1}
// half first, then the {0,1} half.  Two rows j, l are joined by a link edge
// iff d_j - d_l is itself such an offset (Sec. 3.3).  The same constexpr code
// feeds the host tables and the device kernels.
//
// A set of rows (an upper link, a component) is a bit mask: 64 bits hold the
// 62 rows of a 5D grid, a 6D grid's 126 rows take 128 bits.
#pragma once

#include <stdint.h>

namespace eg {

template <int NDIM>
struct MaskOf {
    using type = uint64_t;
};
template <>
struct MaskOf<6> {
    using type = unsigned __int128;
};
template <int NDIM>
using Mask = typename MaskOf<NDIM>::type;

template <int NDIM>
struct Rows {
    static constexpr int K = 2 * ((1 << NDIM) - 1);
    int8_t d[K][NDIM];
    Mask<NDIM> adj[K];
};

constexpr bool alg1_offset(const int* d, int n)
{
    bool in01 = true, in0m1 = true, zero = true;
    for (int i = 0; i < n; ++i) {
        if (d[i] != 0) zero = false;
        if (!(d[i] == 0 || d[i] == 1)) in01 = false;
        if (!(d[i] == 0 || d[i] == -1)) in0m1 = false;
    }
    return !zero && (in01 || in0m1);
}

template <int NDIM>
constexpr Rows<NDIM> make_rows_ce()
{
    Rows<NDIM> r{};
    int cnt = 0;
    int total = 1;
    for (int i = 0; i < NDIM; ++i) total *= 3;
    // enumerate {-1,0,1}^n in lexicographic order (axis 0 most significant)
    for (int t = 0; t < total; ++t) {
        int d[NDIM] = {};
        int x = t;
        for (int i = NDIM - 1; i >= 0; --i) {
            d[i] = x % 3 - 1;
            x /= 3;
        }
        if (alg1_offset(d, NDIM)) {
            for (int i = 0; i < NDIM; ++i) r.d[cnt][i] = (int8_t)d[i];
            ++cnt;
        }
    }
    for (int j = 0; j < Rows<NDIM>::K; ++j) {
        Mask<NDIM> m = 0;
        for (int l = 0; l < Rows<NDIM>::K; ++l) {
            int diff[NDIM] = {};
            for (int i = 0; i < NDIM; ++i) diff[i] = r.d[j][i] - r.d[l][i];
            if (alg1_offset(diff, NDIM)) m |= Mask<NDIM>(1) << l;
        }
        r.adj[j] = m;
    }
    return r;
}

// Component of `seed` in `mask` using the row adjacency (compile time).
template <int NDIM>
constexpr Mask<NDIM> closure_ce(const Rows<NDIM>& r, Mask<NDIM> seed, Mask<NDIM> mask)
{
    Mask<NDIM> comp = seed, frontier = seed;
    while (frontier) {
        int j = 0;
        while (!((frontier >> j) & 1)) ++j;
        frontier &= frontier - 1;
        const Mask<NDIM> nb = r.adj[j] & mask & ~comp;
        comp |= nb;
        frontier |= nb;
    }
    return comp;
}

// 3D: bit m of the table is set iff the upper-link mask m (14 rows) is
// non-empty and connected.
struct Conn3 {
    uint32_t w[(1 << 14) / 32];
};

// Bit m: an upper link with row mask m makes no saddle, i.e. it is empty
// (a maximum) or a single component.
constexpr Conn3 make_conn3()
{
    constexpr Rows<3> r = make_rows_ce<3>();
    Conn3 c{};
    c.w[0] = 1u;
    for (uint32_t m = 1; m < (1u << 14); ++m) {
        const uint64_t comp = closure_ce<3>(r, m & (~m + 1u), m);
        if (comp == m) c.w[m >> 5] |= 1u << (m & 31);
    }
    return c;
}

#if defined(__HIPCC__)
// Row adjacency in constant memory, one table per dimension, for the kernels
// that test link connectivity by a bit-parallel search (the 2D/3D tiles use
// precomputed connectivity bits instead).  Internal linkage: every source file
// that uses a table holds its own copy.
template <int NDIM>
struct AdjTable {
    Mask<NDIM> adj[Rows<NDIM>::K];
};
template <int NDIM>
constexpr AdjTable<NDIM> make_adj()
{
    constexpr Rows<NDIM> r = make_rows_ce<NDIM>();
    AdjTable<NDIM> t{};
    for (int j = 0; j < Rows<NDIM>::K; ++j) t.adj[j] = r.adj[j];
    return t;
}
namespace {
__constant__ AdjTable<1> c_adj1 = make_adj<1>();
__constant__ AdjTable<2> c_adj2 = make_adj<2>();
__constant__ AdjTable<3> c_adj3 = make_adj<3>();
__constant__ AdjTable<4> c_adj4 = make_adj<4>();
__constant__ AdjTable<5> c_adj5 = make_adj<5>();
__constant__ AdjTable<6> c_adj6 = make_adj<6>();
}  // namespace

template <int NDIM>
__device__ __forceinline__ const Mask<NDIM>* adj_table()
{
    if constexpr (NDIM == 1) return c_adj1.adj;
    else if constexpr (NDIM == 2) return c_adj2.adj;
    else if constexpr (NDIM == 3) return c_adj3.adj;
    else if constexpr (NDIM == 4) return c_adj4.adj;
    else if constexpr (NDIM == 5) return c_adj5.adj;
    else return c_adj6.adj;
}

// Index of the lowest set bit of a non-empty mask.
__device__ __forceinline__ int lowest_bit(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
__device__ __forceinline__ int lowest_bit(unsigned __int128 m)
{
    const uint64_t lo = (uint64_t)m;
    return lo ? __ffsll((unsigned long long)lo) - 1 : 64 + __ffsll((unsigned long long)(uint64_t)(m >> 64)) - 1;
}

// Index of the highest set bit of a non-empty mask.
__device__ __forceinline__ int highest_bit(uint64_t m) { return 63 - __clzll((long long)m); }
__device__ __forceinline__ int highest_bit(unsigned __int128 m)
{
    const uint64_t hi = (uint64_t)(m >> 64);
    return hi ? 127 - __clzll((long long)hi) : 63 - __clzll((long long)(uint64_t)m);
}

// Component of `seed` inside `mask` (BFS over link edges, bit-parallel).
template <class M>
__device__ __forceinline__ M closure(M seed, M mask, const M* adj)
{
    M comp = seed, frontier = seed;
    while (frontier != 0) {
        const int j = lowest_bit(frontier);
        frontier &= frontier - 1;
        const M nb = adj[j] & mask & ~comp;
        comp |= nb;
        frontier |= nb;
    }
    return comp;
}
#endif

// Offsets of each row packed two bits per row ((d + 1) in {0,1,2}) for axis i.
template <int NDIM>
constexpr uint64_t pack_axis(const Rows<NDIM>& r, int axis)
{
    uint64_t p = 0;
    for (int j = 0; j < Rows<NDIM>::K; ++j) p |= uint64_t(r.d[j][axis] + 1) << (2 * j);
    return p;
}

}  // namespace eg
