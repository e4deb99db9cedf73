// eg_rows.h -- compile-time neighbour rows of the Freudenthal tessellation.
//
// Rows are the offsets d != 0 with every component in {0,1} or every
// component in {0,-1} (GridAdjacency, Sec. 3.2 Alg. 1), sorted
// lexicographically with axis 0 (the slowest) most significant: the {0,-1}
// half first, then the {0,1} half.  Two rows j, l are joined by a link edge
// iff d_j - d_l is itself such an offset (Sec. 3.3).  The same constexpr code
// feeds the host tables and the device kernels.
#pragma once

#include <stdint.h>

namespace eg {

template <int NDIM>
struct Rows {
    static constexpr int K = 2 * ((1 << NDIM) - 1);
    int8_t d[K][NDIM];
    uint64_t adj[K];
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
        uint64_t m = 0;
        for (int l = 0; l < Rows<NDIM>::K; ++l) {
            int diff[NDIM] = {};
            for (int i = 0; i < NDIM; ++i) diff[i] = r.d[j][i] - r.d[l][i];
            if (alg1_offset(diff, NDIM)) m |= uint64_t(1) << l;
        }
        r.adj[j] = m;
    }
    return r;
}

// Component of `seed` in `mask` using the row adjacency (compile time).
template <int NDIM>
constexpr uint64_t closure_ce(const Rows<NDIM>& r, uint64_t seed, uint64_t mask)
{
    uint64_t comp = seed, frontier = seed;
    while (frontier) {
        int j = 0;
        while (!((frontier >> j) & 1)) ++j;
        frontier &= frontier - 1;
        const uint64_t nb = r.adj[j] & mask & ~comp;
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

constexpr Conn3 make_conn3()
{
    constexpr Rows<3> r = make_rows_ce<3>();
    Conn3 c{};
    for (uint32_t m = 1; m < (1u << 14); ++m) {
        const uint64_t comp = closure_ce<3>(r, m & (~m + 1u), m);
        if (comp == m) c.w[m >> 5] |= 1u << (m & 31);
    }
    return c;
}

// Offsets of each row packed two bits per row ((d + 1) in {0,1,2}) for axis i.
template <int NDIM>
constexpr uint64_t pack_axis(const Rows<NDIM>& r, int axis)
{
    uint64_t p = 0;
    for (int j = 0; j < Rows<NDIM>::K; ++j) p |= uint64_t(r.d[j][axis] + 1) << (2 * j);
    return p;
}

}  // namespace eg
