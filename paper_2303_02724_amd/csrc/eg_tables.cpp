// eg_tables.cpp -- host-side neighbour tables and workspace layout.
//
// The neighbour rows come from the GridAdjacency test (Sec. 3.2, Alg. 1):
// offset d (nonzero) is a neighbour offset iff every component of d lies in
// {0,1} or every component lies in {0,-1}; two neighbours of the same vertex
// are joined by a link edge iff their offsets differ by such a vector.
#include <algorithm>
#include <array>
#include <cstring>
#include <vector>

#include "eg_internal.h"

namespace eg {

static bool alg1_adjacent(const int* d, int n)
{
    bool in01 = true, in0m1 = true, zero = true;
    for (int i = 0; i < n; ++i) {
        if (d[i] != 0) zero = false;
        if (!(d[i] == 0 || d[i] == 1)) in01 = false;
        if (!(d[i] == 0 || d[i] == -1)) in0m1 = false;
    }
    return !zero && (in01 || in0m1);
}

int make_rows(int ndim, int8_t (*off)[EG_MAX_NDIM], uint64_t* adj)
{
    if (ndim < 1 || ndim > EG_MAX_NDIM) return -1;
    std::vector<std::array<int, EG_MAX_NDIM>> rows;
    int total = 1;
    for (int i = 0; i < ndim; ++i) total *= 3;
    for (int t = 0; t < total; ++t) {
        std::array<int, EG_MAX_NDIM> d{};
        int r = t;
        for (int i = ndim - 1; i >= 0; --i) {
            d[i] = r % 3 - 1;
            r /= 3;
        }
        if (alg1_adjacent(d.data(), ndim)) rows.push_back(d);
    }
    // lexicographic, axis 0 most significant: equals linear-index order
    std::sort(rows.begin(), rows.end(), [ndim](const auto& a, const auto& b) {
        for (int i = 0; i < ndim; ++i)
            if (a[i] != b[i]) return a[i] < b[i];
        return false;
    });
    const int k = (int)rows.size();
    for (int j = 0; j < k; ++j) {
        if (off)
            for (int i = 0; i < EG_MAX_NDIM; ++i) off[j][i] = (int8_t)(i < ndim ? rows[j][i] : 0);
        if (adj) {
            uint64_t m = 0;
            for (int l = 0; l < k; ++l) {
                int diff[EG_MAX_NDIM];
                for (int i = 0; i < ndim; ++i) diff[i] = rows[j][i] - rows[l][i];
                if (alg1_adjacent(diff, ndim)) m |= uint64_t(1) << l;
            }
            adj[j] = m;
        }
    }
    return k;
}

void make_table(const Grid& g, LinkTable* t)
{
    int8_t off[kMaxNb][EG_MAX_NDIM];
    uint64_t adj[kMaxNb];
    std::memset(t, 0, sizeof(*t));
    const int k = make_rows(g.ndim, off, adj);
    int64_t stride[EG_MAX_NDIM];
    int64_t s = 1;
    for (int i = g.ndim - 1; i >= 0; --i) {
        stride[i] = s;
        s *= g.dims[i];
    }
    t->k = k;
    for (int j = 0; j < k; ++j) {
        int64_t lin = 0;
        uint32_t forb = 0;
        for (int i = 0; i < g.ndim; ++i) {
            lin += off[j][i] * stride[i];
            if (off[j][i] < 0) forb |= 1u << (2 * i);
            if (off[j][i] > 0) forb |= 1u << (2 * i + 1);
        }
        t->lin[j] = (int32_t)lin;
        t->forb[j] = forb;
        t->adj[j] = adj[j];
    }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Work carve(void* base, int64_t cap_max, int64_t cap_sad, int64_t cap_pairs)
{
    Work w{};
    w.cap_keys = std::max<int64_t>(cap_pairs + cap_sad, cap_max);
    w.cap_keys = std::max<int64_t>(w.cap_keys, 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    size_t o_ctr = take(sizeof(uint32_t) * C_SLOTS);
    size_t o_umax = take(sizeof(uint32_t) * (size_t)std::max<int64_t>(cap_max, 1));
    size_t o_usad = take(sizeof(uint32_t) * (size_t)std::max<int64_t>(cap_sad, 1));
    size_t o_ka = take(sizeof(uint64_t) * (size_t)w.cap_keys);
    size_t o_kb = take(sizeof(uint64_t) * (size_t)w.cap_keys);
    size_t o_h = take(sizeof(uint32_t) * (256 * kSortBlocks + 2 * kSortBlocks + 64));
    w.bytes = off;
    if (base) {
        char* p = (char*)base;
        w.ctr = (uint32_t*)(p + o_ctr);
        w.umax = (uint32_t*)(p + o_umax);
        w.usad = (uint32_t*)(p + o_usad);
        w.keysA = (uint64_t*)(p + o_ka);
        w.keysB = (uint64_t*)(p + o_kb);
        w.hist = (uint32_t*)(p + o_h);
    }
    return w;
}

}  // namespace eg
