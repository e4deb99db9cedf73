// eg_link.h -- is an upper link connected?  Set algebra on the link's rows.
//
// The link of a vertex in the Freudenthal triangulation (Alg. 1) has two
// halves: the rows with offsets in {0,1}^n, which are the non-empty subsets a
// of the n axes, and the rows with offsets in {0,-1}^n, the negated subsets
// -b.  Two rows are joined by a link edge iff their difference is again a row
// (a non-zero vector of {0,1}^n or {0,-1}^n), that is:
//   a and a'   (same half)   iff one subset contains the other;
//   a and -b   (across)      iff a and b are disjoint (a + b is a subset).
// So a half of an upper-link mask is a 2^n-bit word (bit s for subset s), and
// the neighbours of a set of rows follow from its superset and subset
// closures (n shift-and-mask steps each) and from complementing every subset
// (a reversal of the word).  The component of one row grows in registers,
// one closure after another until it stops; a saddle (Table 1) is an upper
// link that the component of any one of its rows does not cover.
//
// Row order is the one of the row table (eg_rows.h): all offsets of
// {-1,0,1}^n in lexicographic order, axis 0 first, so the first 2^n - 1 rows
// are the negated subsets in decreasing order of the subset (row j is -(2^n -
// 1 - j)) and the last 2^n - 1 rows the subsets in increasing order (row
// 2^n - 2 + s is subset s), with axis 0 the most significant bit of s.
#pragma once
#include <stdint.h>

namespace eg {

template <int NDIM>
struct SubsetWord {
    using type = uint32_t;
};
template <>
struct SubsetWord<6> {
    using type = uint64_t;
};

// bit s set iff subset s holds axis bit i
template <class W>
__host__ __device__ constexpr W axis_bits(int i)
{
    return (W)(i == 0   ? 0xAAAAAAAAAAAAAAAAull
               : i == 1 ? 0xCCCCCCCCCCCCCCCCull
               : i == 2 ? 0xF0F0F0F0F0F0F0F0ull
               : i == 3 ? 0xFF00FF00FF00FF00ull
               : i == 4 ? 0xFFFF0000FFFF0000ull
                        : 0xFFFFFFFF00000000ull);
}

// every superset (within the n axes) of a subset in a
template <int NDIM, class W>
__host__ __device__ inline W supersets(W a)
{
#pragma unroll
    for (int i = 0; i < NDIM; ++i) a |= (a & ~axis_bits<W>(i)) << (1 << i);
    return a;
}

// every subset of a subset in a (the empty one included)
template <int NDIM, class W>
__host__ __device__ inline W subsets(W a)
{
#pragma unroll
    for (int i = 0; i < NDIM; ++i) a |= (a & axis_bits<W>(i)) >> (1 << i);
    return a;
}

// the complements of the subsets in a: bit s -> bit 2^n - 1 - s
template <int NDIM>
__host__ __device__ inline typename SubsetWord<NDIM>::type complements(typename SubsetWord<NDIM>::type a)
{
    if constexpr (NDIM == 6)
        return __builtin_bitreverse64(a);
    else
        return __builtin_bitreverse32(a) >> (32 - (1 << NDIM));
}

// the highest set bit of a non-empty word
__host__ __device__ inline uint32_t top_bit(uint32_t a) { return 1u << (31 - __builtin_clz(a)); }
__host__ __device__ inline uint64_t top_bit(uint64_t a) { return 1ull << (63 - __builtin_clzll(a)); }

// Rows of the link as the two subset words: ml holds the b of the rows -b,
// mu the a of the rows a.
template <int NDIM, class M>
__host__ __device__ inline void to_subsets(M rows, typename SubsetWord<NDIM>::type& ml,
                                           typename SubsetWord<NDIM>::type& mu)
{
    using W = typename SubsetWord<NDIM>::type;
    constexpr int H = (1 << NDIM) - 1;  // rows per half
    ml = complements<NDIM>((W)(rows & ((M(1) << H) - 1)));
    mu = (W)(rows >> H) << 1;
}

// The component, within the rows ml/mu, of the lowest row among them: in
// place of the seed (cl, cu), grown one edge per round until it stops.
template <int NDIM, class W>
__host__ __device__ inline void grow(W ml, W mu, W& cl, W& cu)
{
    cl = ml ? top_bit(ml) : W(0);  // the lowest row of the -b half has the largest b
    cu = ml ? W(0) : mu & (~mu + 1);
    while (true) {
        // each closure starts from the rows the previous one reached, so a
        // round follows several edges (superset, then subset or across, ...)
        W nu = supersets<NDIM>(cu) & mu;
        nu = subsets<NDIM>(nu | complements<NDIM>(cl)) & mu;
        W nl = supersets<NDIM>(cl) & ml;
        nl = subsets<NDIM>(nl | complements<NDIM>(nu)) & ml;
        // stop when nothing grows, or at once when every row is reached (the
        // usual case: most upper links are connected)
        const bool done = (nu == cu && nl == cl) || (nu == mu && nl == ml);
        cu = nu;
        cl = nl;
        if (done) break;
    }
}

// Whether the rows in `up` (a non-empty mask over the 2(2^n - 1) rows) form
// one connected piece of the link.
template <int NDIM, class M>
__host__ __device__ inline bool link_connected(M up)
{
    typename SubsetWord<NDIM>::type ml, mu, cl, cu;
    to_subsets<NDIM>(up, ml, mu);
    grow<NDIM>(ml, mu, cl, cu);
    return cu == mu && cl == ml;
}

// The component of the lowest row of `rows` (a non-empty mask) within
// `rows`, as a row mask.
template <int NDIM, class M>
__host__ __device__ inline M link_component(M rows)
{
    using W = typename SubsetWord<NDIM>::type;
    constexpr int H = (1 << NDIM) - 1;
    W ml, mu, cl, cu;
    to_subsets<NDIM>(rows, ml, mu);
    grow<NDIM>(ml, mu, cl, cu);
    return M(complements<NDIM>(cl)) | (M(cu >> 1) << H);
}

}  // namespace eg
