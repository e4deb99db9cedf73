// eg_tables.cpp -- host-side neighbour tables and workspace layout.
//
// The neighbour rows come from the compile-time tables of eg_rows.h
// (GridAdjacency, Sec. 3.2 Alg. 1); here they get the grid's linear offsets
// and boundary bits.
#include <algorithm>
#include <cstring>

#include "eg_internal.h"
#include "eg_rows.h"

namespace eg {

template <int NDIM>
static int copy_rows(int8_t (*off)[EG_MAX_NDIM], uint64_t* adj)
{
    constexpr Rows<NDIM> r = make_rows_ce<NDIM>();
    constexpr int K = Rows<NDIM>::K, W = (K + 63) / 64;
    for (int j = 0; j < K; ++j) {
        if (off)
            for (int i = 0; i < EG_MAX_NDIM; ++i) off[j][i] = (int8_t)(i < NDIM ? r.d[j][i] : 0);
        if (adj)
            for (int w = 0; w < W; ++w) adj[j * W + w] = (uint64_t)(r.adj[j] >> (64 * w));
    }
    return K;
}

int make_rows(int ndim, int8_t (*off)[EG_MAX_NDIM], uint64_t* adj)
{
    switch (ndim) {
        case 1: return copy_rows<1>(off, adj);
        case 2: return copy_rows<2>(off, adj);
        case 3: return copy_rows<3>(off, adj);
        case 4: return copy_rows<4>(off, adj);
        case 5: return copy_rows<5>(off, adj);
        case 6: return copy_rows<6>(off, adj);
        default: return -1;
    }
}

int passes_for(const Tuning& t, int64_t n)
{
    int p = 1;
    for (int64_t reach = t.hops; reach < n && p < t.passes; reach *= t.hops) ++p;
    return p;
}

void make_table(const Grid& g, LinkTable* t)
{
    int8_t off[kMaxNb][EG_MAX_NDIM];
    std::memset(t, 0, sizeof(*t));
    const int k = make_rows(g.ndim, off, nullptr);
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
    }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool decode_tuning(uint32_t t, Tuning* out)
{
    Tuning u{};
    u.tile3 = (int)(t & 0xFu);
    u.tile2 = (int)((t >> 4) & 0xFu);
    const int h = (int)((t >> 8) & 0xFFu);
    const int e = (int)((t >> 16) & 0x1Fu);
    if ((t >> 21) != 0 || u.tile3 > 2 || u.tile2 > 1 || e > 30) return false;
    u.exit_cap = e == 0 ? 0 : int64_t(1) << e;
    u.hops = h == 0 ? kJumpHops : h;
    if (u.hops != 16 && u.hops != 32 && u.hops != 64 && u.hops != 128) return false;
    int bits = 0;
    while ((1 << bits) < u.hops) ++bits;
    u.passes = (31 + bits - 1) / bits;  // hops^passes >= 2^31
    if (u.passes > kMaxPasses) return false;
    *out = u;
    return true;
}

int64_t exit_capacity(int64_t N)
{
    // one entry per vertex whose steepest step leaves its tile: about half
    // of a tile's boundary layer (a quarter of all vertices for 64x8x8 tiles)
    // on smooth fields.  An overflowing tile falls back to vertex codes, so
    // this bounds memory, not correctness.
    int64_t cap = std::max<int64_t>(N / 2, 4096);
    const int64_t room = (int64_t(1) << 31) - 1 - N;
    return std::max<int64_t>(0, std::min(cap, room));
}

Work carve(void* base, int ndim, int64_t N, int64_t X, int64_t cap_sad, int64_t exit_cap)
{
    Work w{};
    w.cap_exit = exit_capacity(N);
    if (exit_cap > 0) w.cap_exit = std::min(w.cap_exit, exit_cap);
    w.words = mask_words(N, X);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    const size_t o_ctr = take(sizeof(uint32_t) * C_SLOTS);
    const size_t o_mm = take(sizeof(uint64_t) * (size_t)w.words);
    const size_t o_sm = take(sizeof(uint64_t) * (size_t)w.words);
    const size_t o_bs = take(sizeof(uint32_t) * 4 * kArcBlocks);
    // the first four arcs of every saddle; 4D and up keep eight (a second
    // block of cap_sad entries)
    const size_t at_rows = ndim >= 4 ? 2 : 1;
    const size_t o_at = take(sizeof(uint4) * at_rows * (size_t)std::max<int64_t>(cap_sad, 1));
    const size_t o_ex = take(sizeof(uint32_t) * (size_t)std::max<int64_t>(w.cap_exit, 1));
    const size_t o_er = take(sizeof(int32_t) * (size_t)std::max<int64_t>(w.cap_exit, 1));
    // grids without LDS tiles read every neighbour from memory: their order
    // keys are computed once, before classification
    const bool untiled = ndim != 2 && ndim != 3;
    const size_t o_k = untiled ? take(sizeof(uint32_t) * (size_t)N) : 0;
    w.bytes = off;
    if (base) {
        char* p = (char*)base;
        w.ctr = (uint32_t*)(p + o_ctr);
        w.mmask = (uint64_t*)(p + o_mm);
        w.smask = (uint64_t*)(p + o_sm);
        w.bsum = (uint32_t*)(p + o_bs);
        w.atmp = (uint4*)(p + o_at);
        w.exits = (uint32_t*)(p + o_ex);
        w.exres = (int32_t*)(p + o_er);
        w.keys = untiled ? (uint32_t*)(p + o_k) : nullptr;
    }
    return w;
}

}  // namespace eg
