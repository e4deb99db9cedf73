// eg_classify_tiled.hip -- LDS-tiled classification for 2D and 3D grids.
//
// One workgroup (4 waves) owns a tile of 64 (x, the fastest axis) x TY (x TZ)
// vertices.  It stages the tile plus a one-vertex halo of order keys in LDS
// (coalesced rows; positions outside the grid get the sentinel key 0, which
// is below every vertex, so boundary vertices need no special case: a missing
// neighbour is never upper and never the steepest one).  Then, per vertex:
//
//   (a) steepest-ascent pointer: highest vertex of the closed neighbourhood
//       (Sec. 3.3; the vertex itself iff its upper link is empty);
//   (c) the upper-link mask over the 2(2^n - 1) Freudenthal rows (Alg. 1) and
//       its connectivity from a compile-time table: empty = maximum,
//       disconnected = saddle (beta+ >= 2, Table 1);
//   (b, first part) tile-local pointer jumping in LDS: every pointer is
//       followed while it stays inside the tile, so the kernel writes, for
//       each vertex, either its maximum or the first vertex of its
//       steepest-ascent path outside the tile.  The global pass then needs
//       only a few hops per vertex.
//
// Workgroups are mapped to tiles so that the tiles of one XCD are
// consecutive in memory (their halos then meet in the same L2).
#include <utility>

#include "eg_internal.h"
#include "eg_rows.h"

namespace eg {

__constant__ Conn3 c_conn3 = make_conn3();

constexpr uint64_t make_conn2()
{
    constexpr Rows<2> r = make_rows_ce<2>();
    uint64_t c = 0;
    for (uint32_t m = 1; m < 64u; ++m)
        if (closure_ce<2>(r, m & (~m + 1u), m) == m) c |= uint64_t(1) << m;
    return c;
}

template <int NDIM, int J>
struct Row {
    static constexpr Rows<NDIM> R = make_rows_ce<NDIM>();
    static constexpr int dz = NDIM == 3 ? R.d[J][0] : 0;
    static constexpr int dy = R.d[J][NDIM - 2];
    static constexpr int dx = R.d[J][NDIM - 1];
};

template <int NDIM>
struct Pack {
    static_assert(NDIM <= 3, "two bits per row must fit 32 bits");
    static constexpr Rows<NDIM> R = make_rows_ce<NDIM>();
    static constexpr uint32_t z = NDIM == 3 ? (uint32_t)pack_axis<NDIM>(R, 0) : 0x55555555u;
    static constexpr uint32_t y = (uint32_t)pack_axis<NDIM>(R, NDIM - 2);
    static constexpr uint32_t x = (uint32_t)pack_axis<NDIM>(R, NDIM - 1);
};

// Label encoding written by the classification kernels: a value m >= 0 is
// final (the maximum m); a value -(e + 1) < 0 says "same label as vertex e",
// a later vertex of the steepest-ascent path.  The jump kernel resolves the
// negative entries.

// Resolve the tile's successor array by pointer jumping.  cur[k] holds the
// successor of this thread's k-th vertex (s_idx(k) is its tile index), scaled
// by UNIT (1: tile indices; 4: byte offsets into s_nxt, which spares the
// address shift in every round): below UNIT TILE a vertex of the tile, at or
// above it a tile-local maximum (UNIT (TILE + its own index)), < 0 the
// tile-local code of the exit by which the path leaves the tile; the last two
// end a chain.  Each round replaces every successor inside the tile by that
// vertex's successor, in place.  Only the owning wave writes an entry, and
// every value written is a vertex further along the same path (or its end),
// so any value a wave reads, old or new, is a valid successor that moves its
// chain forward.  Hence every wave runs its own rounds until its own chains
// have ended, with no barrier (a wave that finishes early leaves final
// entries behind); log2 of the longest in-tile path bounds the rounds.  Call
// after a barrier that follows the last store to s_nxt.
template <int VPT, int TILE, int UNIT, class Idx>
__device__ __forceinline__ void double_tile_chains(int (&cur)[VPT], int32_t* s_nxt, Idx s_idx)
{
    static_assert(UNIT == 1 || UNIT == 4, "tile indices or byte offsets");
    constexpr unsigned END = (unsigned)TILE * UNIT;
    bool pending = false;
#pragma unroll
    for (int k = 0; k < VPT; ++k) pending |= (unsigned)cur[k] < END;
    if (__ballot(pending) == 0) return;
    if constexpr (UNIT == 4) {
        // every round issues all its reads before it writes, with no branch:
        // an entry that has ended reads its own slot, which holds its current
        // value
        do {
            int m[VPT];
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                const int n = cur[k];
                const int at = (unsigned)n < END ? n : 4 * s_idx(k);
                m[k] = *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(s_nxt) + at);
            }
            uint32_t lo = ~0u;
#pragma unroll
            for (int k = 0; k < VPT; ++k) {
                cur[k] = m[k];
                s_nxt[s_idx(k)] = m[k];
                lo = min(lo, (uint32_t)m[k]);
            }
            pending = lo < END;
        } while (__ballot(pending) != 0);
        return;
    }
    // the test at the bottom keeps every cur[k] in one register across rounds
    do {
        pending = false;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int n = cur[k];
            if ((unsigned)n < END) {
                const int m = s_nxt[n];
                cur[k] = m;
                s_nxt[s_idx(k)] = m;
                pending |= (unsigned)m < END;
            }
        }
    } while (__ballot(pending) != 0);
}

// Every vertex whose steepest step leaves the tile gets its own entry of the
// exit list, which records the step's target; before the tile's chains are
// resolved, cur[k] < 0 holds -(target + 1) for such a vertex.  rank_exits
// numbers the tile's exits without a scan: per k, a wave ballot of its
// exiting lanes, the lane's rank among them (mbcnt) and the running count of
// the wave (scalar).  The targets go to s_exv in rank order and cur[k] becomes
// the tile-local code -(rank + 1), which the pointer doubling hands to every
// vertex whose path leaves the tile there.  One atomic per tile claims the
// tile's block of the list: thread 0 issues it here and first needs its value
// in place_exits, after the doubling, so the round trip of a device-wide
// atomic overlaps the doubling instead of stalling the workgroup.  Writes
// s_exv after a barrier, so the caller may alias it with the halo.
template <int VPT>
__device__ __forceinline__ uint32_t rank_exits(int (&cur)[VPT], uint32_t* s_tmp, uint32_t* s_exv,
                                               uint32_t* __restrict__ ctr, uint32_t& claim)
{
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    uint32_t wave_total = 0;
#pragma unroll
    for (int k = 0; k < VPT; ++k) wave_total += (uint32_t)__popcll(__ballot(cur[k] < 0));
    if ((tid & 63) == 0) s_tmp[w] = wave_total;
    __syncthreads();
    uint32_t r0 = 0;  // first rank of this wave's k-th group (uniform)
    for (int k = 0; k < w; ++k) r0 += s_tmp[k];
    const uint32_t total = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    claim = 0;
    if (tid == 0 && total) claim = atomicAdd(&ctr[C_NEXIT], total);
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const uint64_t bal = __ballot(cur[k] < 0);
        if (cur[k] < 0) {
            const uint32_t r =
                r0 + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            s_exv[r] = (uint32_t)(-cur[k] - 1);
            cur[k] = -(int)r - 1;
        }
        r0 += (uint32_t)__popcll(bal);
    }
    return total;
}

// After the doubling: the tile's block of the exit list starts at the claimed
// base; the block is written with coalesced stores.  Entries below the
// capacity are always written, so the list never holds garbage even when the
// tile's block does not fit; such a tile gives its vertices the vertex codes
// of their exits' targets instead of list codes.  Returns whether it fit.
__device__ __forceinline__ bool place_exits(uint32_t total, uint32_t claim, const uint32_t* s_exv, uint32_t* s_tmp,
                                            uint32_t* __restrict__ exits, uint32_t cap_exit, uint32_t& base)
{
    const int tid = threadIdx.x;
    if (tid == 0) s_tmp[4] = claim;
    __syncthreads();
    base = s_tmp[4];
    for (uint32_t i = tid; i < total; i += 256)
        if (base + i < cap_exit) exits[base + i] = s_exv[i];
    return (uint64_t)base + total <= cap_exit;
}

// The offset that turns a tile-local exit code n < 0 into the label code of
// its list entry: exit_list_code(N, base - n - 1) = n - (N + base).  A tile
// whose block did not fit turns its codes into the vertex codes of the exits'
// targets here instead (offset 0).
template <int VPT>
__device__ __forceinline__ int exit_offset(int (&cur)[VPT], bool fit, uint32_t base, const uint32_t* s_exv, int N)
{
    if (fit) return N + (int)base;
#pragma unroll
    for (int k = 0; k < VPT; ++k)
        if (cur[k] < 0) cur[k] = -(int)s_exv[-cur[k] - 1] - 1;
    return 0;
}

// Critical-vertex bitmasks: each wave handles one 64-vertex row segment of
// the tile per step, which is exactly one mask word (tiles start at
// multiples of 64 along x).  Step k parks its maxima word in lane k and its
// saddle word in lane 32 + k; at the end every lane stores at most one word,
// so the masks cost one store instruction per wave and no atomics.
// v_writelane_b32 (lane `lane` of a vector register takes a scalar value) and
// v_bfe_u32 (which reads only the low five bits of the offset), as the
// compiler's own intrinsics
extern "C" __device__ int eg_writelane(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");
extern "C" __device__ uint32_t eg_ubfe(uint32_t src, uint32_t offset, uint32_t width) __asm("llvm.amdgcn.ubfe.i32");

__device__ __forceinline__ void park_word(uint64_t& mine, bool pred, int lane)
{
    const uint64_t b = __ballot(pred);
    uint32_t lo = (uint32_t)eg_writelane((int)(uint32_t)b, lane, (int)(uint32_t)mine);
    uint32_t hi = (uint32_t)eg_writelane((int)(uint32_t)(b >> 32), lane, (int)(uint32_t)(mine >> 32));
    // pin the word here: otherwise the selects sink to the final store and
    // every step's two ballots stay alive in scalar registers until then
    asm volatile("" : "+v"(lo), "+v"(hi));
    mine = ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ void store_words(const TileArgs& a, uint64_t word, int vpt, int row, bool row_in, int tx)
{
    // row: the grid row (gz * Y + gy) of this lane's step; row_in: it exists
    const int lane = __lane_id();
    if ((lane & 31) < vpt && row_in) {
        const int64_t at = (int64_t)row * a.tiles_x + tx;
        (lane < 32 ? a.mmask : a.smask)[at] = word;
    }
}

template <int NDIM, bool MINMODE, int TY, int TZ>
__device__ __forceinline__ void tile_nd(const TileArgs& a, int b, uint32_t* s_u, int32_t* s_nxt, uint32_t* s_conn,
                                        uint32_t* s_tmp)
{
    static_assert(NDIM == 2 || NDIM == 3, "tiled path is for 2D and 3D");
    static_assert(TY % 4 == 0, "four waves split the y rows");
    constexpr int K = 2 * ((1 << NDIM) - 1);
    constexpr int TX = 64;
    constexpr int HX = TX + 2, HY = TY + 2, HZ = NDIM == 3 ? TZ + 2 : 1;
    constexpr int HALO = HX * HY * HZ;
    constexpr int TILE = TX * TY * TZ;
    constexpr int YPT = TY / 4;
    constexpr int VPT = YPT * TZ;
    constexpr int ZH = NDIM == 3 ? 1 : 0;  // halo depth along z
    const float* __restrict__ f = a.f;
    const int X = a.X, Y = a.Y, Z = a.Z;
    int32_t* __restrict__ lab = a.lab;
    int32_t* __restrict__ ptr = a.ptr;
    uint32_t* __restrict__ ctr = a.ctr;

    // the wave index is uniform: keep it (and every row quantity) scalar
    const int tid = threadIdx.x, lx = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tx = b % a.tiles_x;
    const int rr = b / a.tiles_x;
    const int ty = rr % a.tiles_y;
    const int tz = rr / a.tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int SY = X;
    const int SZ = X * Y;

    if constexpr (NDIM == 3)
        for (int i = tid; i < 512; i += 256) s_conn[i] = c_conn3.w[i];
    bool nan = false;
    if constexpr (NDIM == 2) {
        // rows of 64 aligned values, one per lane, from a uniform row address
        // (rows outside the grid read a clamped row and are replaced), then
        // the two edge columns of every row (one value per thread); all loads
        // are issued before the first is used
        constexpr int RPW = (HY + 3) / 4;
        constexpr int EDGES = 2 * HY;
        static_assert(EDGES <= 256, "one edge value per thread");
        const int gx = x0 + lx;
        const bool xin = gx < X;
        const int gxc = xin ? gx : X - 1;
        float vals[RPW];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int gy = y0 + wv + 4 * i - 1;
            const int gyc = min(max(gy, 0), Y - 1);
            vals[i] = f[(int64_t)gyc * SY + gxc];
        }
        const int erow = tid >> 1;
        const int egx = (tid & 1) ? x0 + TX : x0 - 1;
        const int egy = y0 + erow - 1;
        const bool ein = tid < EDGES && (unsigned)egx < (unsigned)X && (unsigned)egy < (unsigned)Y;
        const float eval = f[ein ? (int64_t)egy * SY + egx : 0];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int hy = wv + 4 * i;  // uniform
            if (hy < HY) {
                const int gy = y0 + hy - 1;
                const bool ok = xin && (unsigned)gy < (unsigned)Y;
                nan |= ok && hy >= 1 && hy <= TY && vals[i] != vals[i];
                s_u[hy * HX + lx + 1] = ok ? mode_key<MINMODE>(vals[i]) : 0u;
            }
        }
        if (tid < EDGES) s_u[erow * HX + ((tid & 1) ? HX - 1 : 0)] = ein ? mode_key<MINMODE>(eval) : 0u;
    } else {
        constexpr int PER = (HALO + 255) / 256;
        float vals[PER];
        bool vin[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            const int hx = e % HX;
            const int q = e / HX;
            const int hy = q % HY;
            const int hz = q / HY;
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - ZH;
            vin[i] = e < HALO && (unsigned)gx < (unsigned)X && (unsigned)gy < (unsigned)Y && (unsigned)gz < (unsigned)Z;
            vals[i] = vin[i] ? f[gz * SZ + gy * SY + gx] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int e = tid + 256 * i;
            if (e < HALO) {
                const int hx = e % HX;
                const int q = e / HX;
                const int hy = q % HY;
                const int hz = q / HY;
                const bool own = hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && hz >= ZH && hz < ZH + TZ;
                nan |= vin[i] && own && (vals[i] != vals[i]);
                s_u[e] = vin[i] ? mode_key<MINMODE>(vals[i]) : 0u;
            }
        }
    }
    __syncthreads();

    constexpr uint64_t CONN2 = make_conn2();
    static_assert(VPT <= 32, "one mask word per lane");
    int nxt[VPT];
    uint64_t word = 0;  // this lane's parked mask word
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int ly = wv + 4 * (k % YPT);
        const int lz = k / YPT;
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        const bool in = gx < X && gy < Y && gz < Z;
        const int li = (lz * TY + ly) * TX + lx;
        int n = TILE + li;  // vertices outside the grid end their own chain and are never written
        bool is_max = false, is_sad = false;
        int v = 0;
        if (in) {
            const int c = ((lz + ZH) * HY + (ly + 1)) * HX + (lx + 1);
            const uint32_t uv = s_u[c];
            uint32_t up = 0, best_u = 0;
            int best_j = K;  // K stands for the vertex itself
            // closed neighbourhood in index order (reversed for the minimum
            // graph), so that the later of two equal keys wins with >=
            static_for<0, K + 1>([&](auto step) {
                constexpr int s = decltype(step)::value;
                constexpr int pos = MINMODE ? K - s : s;
                if constexpr (pos == K / 2) {
                    if (uv >= best_u) {
                        best_u = uv;
                        best_j = K;
                    }
                } else {
                    constexpr int j = pos < K / 2 ? pos : pos - 1;
                    using RJ = Row<NDIM, j>;
                    constexpr int off = (RJ::dz * HY + RJ::dy) * HX + RJ::dx;
                    constexpr bool wins_tie = (j >= K / 2) != MINMODE;
                    const uint32_t u = s_u[c + off];
                    const bool above = wins_tie ? (u >= uv) : (u > uv);
                    up |= uint32_t(above) << j;
                    if (u >= best_u) {
                        best_u = u;
                        best_j = j;
                    }
                }
            });
            is_max = up == 0;
            bool connected;
            if constexpr (NDIM == 3)
                connected = (s_conn[up >> 5] >> (up & 31)) & 1u;
            else
                connected = (CONN2 >> up) & 1ull;
            is_sad = !is_max && !connected;
            v = gz * SZ + gy * SY + gx;
            int pv = v;
            if (best_j == K) {
                n = TILE + li;  // a maximum ends its chain
            } else {
                const int dz = NDIM == 3 ? (int)((Pack<NDIM>::z >> (2 * best_j)) & 3u) - 1 : 0;
                const int dy = (int)((Pack<NDIM>::y >> (2 * best_j)) & 3u) - 1;
                const int dx = (int)((Pack<NDIM>::x >> (2 * best_j)) & 3u) - 1;
                pv = v + dz * SZ + dy * SY + dx;
                const int lz2 = lz + dz, ly2 = ly + dy, lx2 = lx + dx;
                const bool inside = (unsigned)lz2 < (unsigned)TZ && (unsigned)ly2 < (unsigned)TY &&
                                    (unsigned)lx2 < (unsigned)TX;
                n = inside ? (lz2 * TY + ly2) * TX + lx2 : -(pv + 1);
            }
            if (ptr) ptr[v] = pv;
        }
        nxt[k] = n;
        park_word(word, is_max, k);
        park_word(word, is_sad, 32 + k);
    }
    {
        const int k = __lane_id() & 31;
        const int ly = wv + 4 * (k % YPT), lz = k / YPT;
        store_words(a, word, VPT, (z0 + lz) * Y + y0 + ly, y0 + ly < Y && z0 + lz < Z, tx);
    }
    if (__ballot(nan) != 0 && __lane_id() == 0) atomicOr(&ctr[C_NAN], 1u);
    const int N = X * Y * Z;
    uint32_t claim;
    const uint32_t nexit = rank_exits<VPT>(nxt, s_tmp, s_u, ctr, claim);  // the halo is no longer read
    auto s_idx = [&](int k) { return ((k / YPT) * TY + wv + 4 * (k % YPT)) * TX + lx; };
#pragma unroll
    for (int k = 0; k < VPT; ++k) s_nxt[s_idx(k)] = nxt[k];
    __syncthreads();
    // global offset of every tile row from the tile's first vertex (one LDS
    // read per vertex instead of quarter-rate multiplies)
    __shared__ int s_rowoff[TY * TZ];
    if (tid < TY * TZ) s_rowoff[tid] = (tid / TY) * SZ + (tid % TY) * SY;
    double_tile_chains<VPT, TILE, 1>(nxt, s_nxt, s_idx);
    uint32_t base;
    const bool fit = place_exits(nexit, claim, s_u, s_tmp, a.exits, a.cap_exit, base);
    const int xoff = exit_offset<VPT>(nxt, fit, base, s_u, N);
    const int tile0 = z0 * SZ + y0 * SY + x0;
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int ly = wv + 4 * (k % YPT);
        const int lz = k / YPT;
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        const int n = nxt[k];
        if (gx < X && gy < Y && gz < Z)
            lab[tile0 + s_rowoff[lz * TY + ly] + lx] =
                n >= 0 ? tile0 + s_rowoff[(n - TILE) >> 6] + (n & 63) : n - xoff;
    }
}

// 3D variant tuned for large grids.  Rows of the halo are loaded aligned
// (one 256-byte wave load per row plus the two edge columns); each thread
// walks YPT columns of the tile along z with a sliding window of three planes
// of the seven in-plane positions a vertex's neighbourhood touches, so a
// vertex costs 7 LDS reads instead of 15; pointer targets stay in registers
// until the halo is no longer needed, then reuse its LDS for the tile-local
// chains, which are resolved by pointer doubling.
// Successor of a vertex as one 32-bit literal per neighbour row, chosen with
// the steepest candidate:
//   bits 0..5   faces of the tile the step crosses if the vertex lies on them
//               (x-, x+, y-, y+, z-, z+)
//   bits 6..31  tile-local offset in bytes of the chain array (signed)
// The vertex itself (a maximum) has no faces and the offset 4 TILE, which
// turns its own byte offset into the chain end 4 (TILE + index).  The 3D
// chains hold byte offsets, so a doubling round reads its successor's entry
// without an address shift.

// Store to lane lx of a row whose first element sits at the uniform address
// `row`: the address stays scalar and only the lane's byte offset lives in a
// vector register.
__device__ __forceinline__ void store_row(int32_t* row, uint32_t lane_b, int32_t v)
{
    *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(row) + lane_b) = v;
}

__device__ __forceinline__ uint32_t max3u(uint32_t a, uint32_t b, uint32_t c) { return max(max(a, b), c); }

// An order-preserving key of the bit pattern, in four instructions: negative
// values map to -b, the others to b | 2^31, so -0 and +0 meet at 2^31 and the
// order of the numbers is kept (keys of the same value are equal, the index
// decides); the top is clamped, so every vertex key lies in [1, 0xFFFFFFFE]
// and the key 0 of positions outside the grid stays below all of them, NaN
// included: no pointer can leave the grid.  The minimum graph takes the
// complement.
template <bool MINMODE>
__device__ __forceinline__ uint32_t bits_key(uint32_t b)
{
    const uint32_t m = (uint32_t)((int32_t)b >> 31);
    const uint32_t k = min((b ^ (m | 0x80000000u)) - m, 0xFFFFFFFEu);
    return MINMODE ? ~k : k;
}

// Keys of numbers lie in [0x00800000, 0xFF800000] (-inf and +inf at the
// ends), complemented in the minimum graph; keys outside come from NaN
// patterns.
template <bool MINMODE>
__device__ __forceinline__ bool nan_key(uint32_t k)
{
    return MINMODE ? (k < 0x007FFFFFu || k >= 0xFF800000u) : (k < 0x00800000u || k > 0xFF800000u);
}

// The key with its last four bits replaced by st (one instruction).
template <int ST>
__device__ __forceinline__ uint32_t bucket_step(uint32_t u)
{
    uint32_t r;
    asm("v_and_or_b32 %0, %1, -16, %2" : "=v"(r) : "v"(u), "n"(ST));
    return r;
}

template <int TY, int HY, int HX>
__device__ __forceinline__ constexpr uint32_t succ_pack(int dz, int dy, int dx)
{
    const int loff = (dz * TY + dy) * 64 + dx;
    const uint32_t em = (dx < 0 ? 1u : 0u) | (dx > 0 ? 2u : 0u) | (dy < 0 ? 4u : 0u) | (dy > 0 ? 8u : 0u) |
                        (dz < 0 ? 16u : 0u) | (dz > 0 ? 32u : 0u);
    return em | (uint32_t(4 * loff) << 6);
}

template <int NDIM_, int J>
struct Win {
    // index of row J's (dy, dx) among the seven window positions
    // (-1,-1) (-1,0) (0,-1) (0,0) (0,1) (1,0) (1,1), and its plane dz + 1
    static constexpr int dy = Row<3, J>::dy, dx = Row<3, J>::dx, dz = Row<3, J>::dz;
    static constexpr int pos = dy < 0 ? (dx < 0 ? 0 : 1) : dy == 0 ? (dx < 0 ? 2 : dx == 0 ? 3 : 4) : (dx == 0 ? 5 : 6);
    static constexpr int plane = dz + 1;
};

template <bool MINMODE, int TY, int TZ, bool FULL, bool PTR>
__device__ __forceinline__ void tile3d_body(const TileArgs& a, int b, uint32_t* s_u, uint32_t* s_conn, uint32_t* s_tmp)
{
    constexpr int K = 14;
    constexpr int TX = 64;
    constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    constexpr int HALO = HX * HY * HZ;
    constexpr int TILE = TX * TY * TZ;
    constexpr int YPT = TY / 4;
    constexpr int VPT = YPT * TZ;
    // only vertices on the tile's faces can step out of it
    constexpr int SURF = TILE - (TX - 2) * (TY - 2) * (TZ - 2);
    static_assert(TILE + SURF <= HALO, "the chains and the exit targets reuse the halo's LDS");
    static_assert(TY % 4 == 0, "four waves split the y rows");
    static_assert(((TY * TZ) & (TY * TZ - 1)) == 0, "row count is a power of two");
    const float* __restrict__ f = a.f;
    const int X = a.X, Y = a.Y, Z = a.Z;
    int32_t* __restrict__ lab = a.lab;
    int32_t* __restrict__ ptr = a.ptr;
    uint32_t* __restrict__ ctr = a.ctr;
    int32_t* s_nxt = reinterpret_cast<int32_t*>(s_u);
    // per row (and K = the vertex itself): packed successor and global offset
    uint32_t* s_pack = s_tmp + 8;
    int32_t* s_gdel = reinterpret_cast<int32_t*>(s_tmp + 8 + 16);
    int32_t* s_hoff = reinterpret_cast<int32_t*>(s_tmp + 8 + 32);  // halo index offset

    // the wave index is uniform: keep it (and every row quantity) scalar
    const int tid = threadIdx.x, lx = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tx = b % a.tiles_x;
    const int rr = b / a.tiles_x;
    const int ty = rr % a.tiles_y;
    const int tz = rr / a.tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int SY = X;
    const int SZ = X * Y;
    if (tid <= K) {
        // entry st: the candidate visited at step st (the vertex itself at K / 2)
        const int pos = MINMODE ? K - tid : tid;
        uint32_t pk = (uint32_t)(4 * TILE) << 6;
        int gd = 0, ho = 0;
        if (pos != K / 2) {
            const int j = pos < K / 2 ? pos : pos - 1;
            const int dz = (int)((Pack<3>::z >> (2 * j)) & 3u) - 1;
            const int dy = (int)((Pack<3>::y >> (2 * j)) & 3u) - 1;
            const int dx = (int)((Pack<3>::x >> (2 * j)) & 3u) - 1;
            pk = succ_pack<TY, HY, HX>(dz, dy, dx);
            gd = dz * SZ + dy * SY + dx;
            ho = (dz * HY + dy) * HX + dx;
        }
        s_pack[tid] = pk;
        s_gdel[tid] = gd;
        s_hoff[tid] = ho;
    }

    bool nan = false;
    {
        // every load of this thread is issued before the first one is used:
        // rows of 64 aligned values (one per lane) from a uniform row address,
        // then the two edge columns of every row (one value per thread);
        // positions outside the grid get the sentinel key 0
        constexpr int ROWS = HY * HZ;
        constexpr int RPW = (ROWS + 3) / 4;
        // every row index a wave takes exists when the rows split evenly
        // (all the tile shapes here): the test then folds away instead of
        // leaving a lane mask per row alive until the stores
        constexpr bool EVEN = ROWS % 4 == 0;
        constexpr int EDGES = 2 * ROWS;
        static_assert(EDGES <= 256, "one edge value per thread");
        static_assert(RPW <= 32, "row flags fit a word");
        const uint32_t* __restrict__ fb = reinterpret_cast<const uint32_t*>(f);
        const int gx = x0 + lx;
        const bool xin = gx < X;
        const int gxc = FULL ? gx : (xin ? gx : X - 1);  // lanes past the grid read a safe address
        const uint32_t lane_boff = 4u * (uint32_t)gxc;
        uint32_t vals[RPW];
        uint32_t rin_bits = 0;  // rows of this wave inside the grid (bit i)
        // a tile whose halo rows all lie in the grid (most of them) steps
        // through its rows by byte offsets from the halo's first row, four
        // rows at a time, on the scalar unit: no per-row division, clamp,
        // test or 64-bit address
        const bool interior = EVEN && y0 >= 1 && z0 >= 1 && y0 + TY < Y && z0 + TZ < Z &&
                              (int64_t)(TZ + 1) * SZ + (int64_t)(TY + 1) * SY + X < (int64_t(1) << 29);
        if (interior) {
            // a raw buffer at the halo's first row: the lane's byte offset in
            // a vector register, the row's in a scalar one (offsets stay
            // below 2^31 bytes, checked above, so the record limit 2^31 - 1
            // never clips a load); the last descriptor word selects 32-bit
            // data, as for any raw dword access on this architecture
            const uint32_t* org = fb + ((int64_t)(z0 - 1) * SZ + (int64_t)(y0 - 1) * SY);
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(org), (short)0, 0x7fffffff, 0x00020000);
            int hy = wv;
            uint32_t off = 4u * (uint32_t)(wv * SY);
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                vals[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, lane_boff, off, 0);
                const bool wrap = hy + 4 >= HY;
                off += wrap ? 4u * (uint32_t)(SZ + (4 - HY) * SY) : 4u * (uint32_t)(4 * SY);
                hy += wrap ? 4 - HY : 4;
            }
            rin_bits = RPW == 32 ? ~0u : (1u << RPW) - 1u;
        } else {
#pragma unroll
            for (int i = 0; i < RPW; ++i) {
                const int row = wv + 4 * i;
                const int hy = row % HY, hz = row / HY;
                const int gy = y0 + hy - 1, gz = z0 + hz - 1;
                rin_bits |= ((EVEN || row < ROWS) && (unsigned)gy < (unsigned)Y && (unsigned)gz < (unsigned)Z ? 1u : 0u)
                            << i;
                // rows outside the grid read a clamped row (their keys are
                // replaced below): the address needs no per-row condition
                const int gyc = min(max(gy, 0), Y - 1), gzc = min(max(gz, 0), Z - 1);
                const char* rowp = reinterpret_cast<const char*>(fb + ((int64_t)gzc * SZ + (int64_t)gyc * SY));
                vals[i] = *reinterpret_cast<const uint32_t*>(rowp + lane_boff);
            }
        }
        rin_bits = __builtin_amdgcn_readfirstlane(rin_bits);
        // edge value of this thread: row tid >> 1, left (x0 - 1) or right (x0 + 64)
        const int erow = tid >> 1;
        const int ehy = erow % HY, ehz = erow / HY;
        const int egx = (tid & 1) ? x0 + TX : x0 - 1;
        const int egy = y0 + ehy - 1, egz = z0 + ehz - 1;
        const bool ein = tid < EDGES && (unsigned)egx < (unsigned)X && (unsigned)egy < (unsigned)Y &&
                         (unsigned)egz < (unsigned)Z;
        const uint32_t eval = fb[ein ? egz * SZ + egy * SY + egx : 0];
        const uint32_t conn_a = c_conn3.w[tid], conn_b = c_conn3.w[tid + 256];
        s_conn[tid] = conn_a;
        s_conn[tid + 256] = conn_b;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int row = wv + 4 * i;
            const bool ok = ((rin_bits >> i) & 1u) && (FULL || xin);
            // one base address, the rows at immediate offsets from it
            if (EVEN || row < ROWS) (s_u + wv * HX + lx + 1)[4 * i * HX] = ok ? bits_key<MINMODE>(vals[i]) : 0u;
        }
        if (tid < EDGES) s_u[erow * HX + ((tid & 1) ? HX - 1 : 0)] = ein ? bits_key<MINMODE>(eval) : 0u;
    }
    __syncthreads();

    static_assert(VPT <= 32, "one mask word per lane");
    int nxt[VPT];
    uint64_t word = 0;  // this lane's parked mask word
    // x faces of the tile this lane's columns lie on (bit 0: lx = 0, bit 1:
    // lx = 63), by shifts rather than compares, so that no lane mask has to
    // stay alive across the unrolled loop
    const uint32_t bx = ((uint32_t)(lx - 1) >> 31) | (((uint32_t)(lx + 1) >> 6) << 1);
    const uint32_t lane_b = 4u * (uint32_t)lx;
#pragma unroll
    for (int c = 0; c < YPT; ++c) {
        const int ly = wv + 4 * c;
        const int gy = y0 + ly;
        const int gx = x0 + lx;
        // tile faces this column lies on (see succ_pack)
        const uint32_t bb_xy = bx | (ly == 0 ? 4u : 0u) | (ly == TY - 1 ? 8u : 0u);
        // window[p][q]: plane hz = lz + p, position q
        uint32_t win[3][7];
        auto load_plane = [&](uint32_t* w, int hz) {
            // one opaque address per plane, at position (-1, -1): the seven
            // reads lie within 2 HX + 2 words of it and pair into ds_read2
            // without an address of their own
            uint32_t boff = 4u * (uint32_t)((hz * HY + ly) * HX) + lane_b;
            asm("" : "+v"(boff));
            const uint32_t* p = reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(s_u) + boff);
            w[0] = p[0];
            w[1] = p[1];
            w[2] = p[HX];
            w[3] = p[HX + 1];
            w[4] = p[HX + 2];
            w[5] = p[2 * HX + 1];
            w[6] = p[2 * HX + 2];
        };
        load_plane(win[0], 0);
        load_plane(win[1], 1);
#pragma unroll
        for (int lz = 0; lz < TZ; ++lz) {
            load_plane(win[(lz + 2) % 3], lz + 2);
            const int gz = z0 + lz;
            const bool in = FULL || (gx < X && gy < Y && gz < Z);
            const uint32_t uv = win[(lz + 1) % 3][3];
            nan |= in && nan_key<MINMODE>(uv);
            // upper-link mask: row 13 first, so that row j ends in bit j; each
            // row's comparison is the carry of an add that doubles the mask
            uint32_t up = 0;
            static_for<0, K>([&](auto step) {
                constexpr int j = K - 1 - decltype(step)::value;
                using WJ = Win<3, j>;
                constexpr bool wins_tie = (j >= K / 2) != MINMODE;
                if constexpr (j == K - 1)
                    up = first_above<wins_tie>(win[(lz + WJ::plane) % 3][WJ::pos], uv);
                else
                    up = push_above<wins_tie>(up, win[(lz + WJ::plane) % 3][WJ::pos], uv);
            });
            // steepest candidate: the maximum of (key with its last four bits
            // replaced by the visiting step), so that equal keys go to the
            // later step; exact unless a key 1..15 units below the maximum
            // sits at a later step than it, which the check below catches
            uint32_t us[K + 1];  // the candidates by visiting step
            static_for<0, K + 1>([&](auto step) {
                constexpr int st = decltype(step)::value;
                constexpr int pos = MINMODE ? K - st : st;
                if constexpr (pos == K / 2) {
                    us[st] = uv;
                } else {
                    constexpr int j = pos < K / 2 ? pos : pos - 1;
                    using WJ = Win<3, j>;
                    us[st] = win[(lz + WJ::plane) % 3][WJ::pos];
                }
            });
            uint32_t pbest = 0;
            static_for<0, K + 1>([&](auto step) {
                constexpr int st = decltype(step)::value;
                pbest = max(pbest, bucket_step<st>(us[st]));
            });
            // the exact maximum as a balanced tree of three-way maxima
            const uint32_t kbest = max3u(max3u(max3u(us[0], us[1], us[2]), max3u(us[3], us[4], us[5]),
                                               max3u(us[6], us[7], us[8])),
                                         max3u(us[9], us[10], us[11]), max3u(us[12], us[13], us[14]));
            int best_st = (int)(pbest & 15u);
            const int cidx = ((lz + 1) * HY + ly + 1) * HX + lx + 1;
            if (s_u[cidx + s_hoff[best_st]] != kbest) {
                // a near tie decided by the dropped bits: the last step that
                // holds the maximum
                static_for<0, K + 1>([&](auto step) {
                    constexpr int st = decltype(step)::value;
                    if (us[st] == kbest) best_st = st;
                });
            }
            // every quantity below without a branch (the successor tables are
            // indexed by visiting step; the table marks the empty link as no
            // saddle, so a maximum needs no test of its own)
            const bool is_max = in && up == 0;
            const bool is_sad = in && eg_ubfe(s_conn[up >> 5], up, 1u) == 0u;
            const uint32_t best_p = s_pack[best_st];
            const int row0 = gz * SZ + gy * SY + x0;  // uniform
            const int pv = row0 + lx + s_gdel[best_st];
            const int li4 = 4 * ((lz * TY + ly) * TX) + (int)lane_b;  // byte offset in the chain array
            // leaves the tile iff it steps across a face the vertex lies on
            const uint32_t faces = bb_xy | (lz == 0 ? 16u : 0u) | (lz == TZ - 1 ? 32u : 0u);
            int n = (faces & best_p & 63u) ? -(pv + 1) : li4 + ((int)best_p >> 6);
            if constexpr (!FULL) n = in ? n : 4 * TILE + li4;  // a vertex outside the grid ends its own chain
            if constexpr (PTR)
                if (in) store_row(ptr + row0, lane_b, pv);
            nxt[c * TZ + lz] = n;
            park_word(word, is_max, c * TZ + lz);
            park_word(word, is_sad, 32 + c * TZ + lz);
        }
    }
    {
        const int k = __lane_id() & 31;
        const int ly = wv + 4 * (k / TZ), lz = k % TZ;
        store_words(a, word, VPT, (z0 + lz) * Y + y0 + ly, y0 + ly < Y && z0 + lz < Z, tx);
    }
    if (__ballot(nan) != 0 && __lane_id() == 0) atomicOr(&ctr[C_NAN], 1u);
    // exit targets go behind the chains, in LDS the halo no longer needs
    uint32_t claim;
    const uint32_t nexit = rank_exits<VPT>(nxt, s_tmp, s_u + TILE, ctr, claim);
#pragma unroll
    for (int c = 0; c < YPT; ++c)
#pragma unroll
        for (int lz = 0; lz < TZ; ++lz) s_nxt[(lz * TY + wv + 4 * c) * TX + lx] = nxt[c * TZ + lz];
    __syncthreads();
    // global offset of every tile row (lz, ly) from the tile's first vertex,
    // so that a tile index becomes a vertex id with one LDS read instead of
    // two quarter-rate multiplies; then every chain inside the tile is
    // followed to its end (double_tile_chains names the three kinds of entry)
    __shared__ int s_rowoff[TY * TZ];
    if (tid < TY * TZ) s_rowoff[tid] = (tid / TY) * SZ + (tid % TY) * SY;
    double_tile_chains<VPT, TILE, 4>(nxt, s_nxt,
                                     [&](int k) { return ((k % TZ) * TY + wv + 4 * (k / TZ)) * TX + lx; });
    uint32_t base;
    const bool fit = place_exits(nexit, claim, s_u + TILE, s_tmp, a.exits, a.cap_exit, base);
    const int xoff = exit_offset<VPT>(nxt, fit, base, s_u + TILE, X * Y * Z);
    const int tile0 = z0 * SZ + y0 * SY + x0;
#pragma unroll
    for (int c = 0; c < YPT; ++c) {
        const int ly = wv + 4 * c;
        const int gx = x0 + lx, gy = y0 + ly;
#pragma unroll
        for (int lz = 0; lz < TZ; ++lz) {
            const int gz = z0 + lz;
            const int n = nxt[c * TZ + lz];
            // the row offset is read for every vertex (masked into range), so
            // that the label is a select rather than a branch
            const int ro = s_rowoff[((uint32_t)(n - 4 * TILE) >> 8) & (TY * TZ - 1)];
            if (FULL || (gx < X && gy < Y && gz < Z))
                store_row(lab + (gz * SZ + gy * SY + x0), lane_b, n >= 0 ? tile0 + ro + ((n >> 2) & 63) : n - xoff);
        }
    }
}

// Full tiles (every vertex in the grid, the common case) run a variant without
// per-vertex bounds tests; whether pointers are written is a compile-time
// choice too, which keeps the output address out of the unrolled loop.
template <bool MINMODE, int TY, int TZ>
__device__ __forceinline__ void tile3d(const TileArgs& a, int b, uint32_t* s_u, uint32_t* s_conn, uint32_t* s_tmp)
{
    const int tx = b % a.tiles_x;
    const int rr = b / a.tiles_x;
    const int ty = rr % a.tiles_y;
    const int tz = rr / a.tiles_y;
    const bool full = (tx + 1) * 64 <= a.X && (ty + 1) * TY <= a.Y && (tz + 1) * TZ <= a.Z;
    if (a.ptr) {
        if (full)
            tile3d_body<MINMODE, TY, TZ, true, true>(a, b, s_u, s_conn, s_tmp);
        else
            tile3d_body<MINMODE, TY, TZ, false, true>(a, b, s_u, s_conn, s_tmp);
    } else {
        if (full)
            tile3d_body<MINMODE, TY, TZ, true, false>(a, b, s_u, s_conn, s_tmp);
        else
            tile3d_body<MINMODE, TY, TZ, false, false>(a, b, s_u, s_conn, s_tmp);
    }
}

// Tiles of one XCD are consecutive in memory: workgroups are dispatched to
// the eight XCDs round-robin, so block b takes tile (b % 8) * (T / 8) + b / 8.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    return (ntiles & 7) == 0 ? (b & 7) * (ntiles >> 3) + (b >> 3) : b;
}

// Label pass over a tiled grid, one workgroup per tile: the exit codes of a
// tile's vertices point into that tile's own block of the exit list, which
// stays in cache while the tile's rows stream through.  Entries with vertex
// codes (a tile whose exits did not fit the list) follow their path for up to
// `hops` links and raise the pass flag if they stop short; the linear passes
// after this one finish them.
template <int TY, int TZ>
__device__ __forceinline__ void final_tile(const TileArgs& a, int b, const int32_t* __restrict__ res, int hops,
                                           uint32_t* flag)
{
    constexpr int YPT = TY / 4;
    const int X = a.X, Y = a.Y, Z = a.Z;
    const int N = X * Y * Z;
    const int SY = X, SZ = X * Y;
    int32_t* lab = a.lab;
    // the wave index is uniform: keep it (and every row quantity) scalar
    const int tid = threadIdx.x, lx = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tx = b % a.tiles_x;
    const int rr = b / a.tiles_x;
    const int ty = rr % a.tiles_y;
    const int tz = rr / a.tiles_y;
    const int gx = tx * 64 + lx;
    constexpr int VPT = YPT * TZ;
    bool notdone = false;
    int vid[VPT], x[VPT];
    // every load of the thread first, then the exit-list look-ups, then the
    // stores: loads and stores of the same array would otherwise serialise;
    // the codes and labels stream through once, so both bypass the caches'
    // normal retention (the exit list stays cached for the look-ups)
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int gy = ty * TY + wv + 4 * (k / TZ), gz = tz * TZ + (k % TZ);
        const bool in = gx < X && gy < Y && gz < Z;
        vid[k] = in ? gz * SZ + gy * SY + gx : -1;
        x[k] = in ? __builtin_nontemporal_load(&lab[vid[k]]) : 0;
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k)
        if (x[k] < -N) x[k] = res[-x[k] - 1 - N];
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        if (x[k] < 0) {
            int y = x[k];
            for (int h = 0; y < 0 && h < hops; ++h) y = y >= -N ? lab[-y - 1] : res[-y - 1 - N];
            x[k] = y;
            notdone |= y < 0;
        }
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k)
        if (vid[k] >= 0) __builtin_nontemporal_store(x[k], &lab[vid[k]]);
    if (__ballot(notdone) != 0 && __lane_id() == 0) atomicOr(flag, 1u);
}

template <int TY, int TZ>
__global__ __launch_bounds__(256) void k_final_tiled(TileArgs a, const int32_t* __restrict__ res, int hops,
                                                     int flag_slot)
{
    final_tile<TY, TZ>(a, xcd_tile(blockIdx.x, a.ntiles), res, hops, &a.ctr[flag_slot]);
}

// The same pass over the tiles of every 2D (or every 3D) field of a batch:
// classes 2 * (NDIM - 2) and the one after it (maximum and minimum graphs)
// own consecutive tiles.
template <int NDIM, int TY, int TZ>
__global__ __launch_bounds__(256) void k_final_tiled_batched(const BatchPlan* __restrict__ plan)
{
    constexpr int c0 = 2 * (NDIM - 2);
    const EG_GPTR(BatchField) fs = plan->fields;
    const int64_t item = plan->class_tile[c0] + blockIdx.x;
    int lo = plan->class_field[c0], hi = plan->class_field[c0 + 2] - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fs[mid].tile_base <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int f = __builtin_amdgcn_readfirstlane(lo);
    const TileArgs a = fs[f].ta;
    final_tile<TY, TZ>(a, (int)(item - fs[f].tile_base), fs[f].exres, plan->tuning.hops, &plan->bctr[C_FINAL]);
}

hipError_t launch_final_tiled_batched(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    const Tuning& tu = hplan.tuning;
    const int64_t t2 = hplan.class_tile[2] - hplan.class_tile[0];
    const int64_t t3 = hplan.class_tile[4] - hplan.class_tile[2];
    if (t2 > 0) {
        if (tu.tile2 == 1)
            hipLaunchKernelGGL((k_final_tiled_batched<2, 16, 1>), dim3((unsigned)t2), dim3(256), 0, s, dplan);
        else
            hipLaunchKernelGGL((k_final_tiled_batched<2, 32, 1>), dim3((unsigned)t2), dim3(256), 0, s, dplan);
    }
    if (t3 > 0) {
        if (tu.tile3 == 1)
            hipLaunchKernelGGL((k_final_tiled_batched<3, 4, 16>), dim3((unsigned)t3), dim3(256), 0, s, dplan);
        else if (tu.tile3 == 2)
            hipLaunchKernelGGL((k_final_tiled_batched<3, 8, 4>), dim3((unsigned)t3), dim3(256), 0, s, dplan);
        else
            hipLaunchKernelGGL((k_final_tiled_batched<3, 8, 8>), dim3((unsigned)t3), dim3(256), 0, s, dplan);
    }
    return hipGetLastError();
}

// The tiles [first, first + count): every tile of the grid, or the tile rows
// of one slab of a streamed build.
template <bool MINMODE, int TY, int TZ>
__global__ __launch_bounds__(256) void k_classify3d(TileArgs a, int first, int count)
{
    constexpr int HALO = 66 * (TY + 2) * (TZ + 2);
    __shared__ uint32_t s_u[HALO];
    __shared__ uint32_t s_conn[512];
    __shared__ uint32_t s_tmp[64];
    tile3d<MINMODE, TY, TZ>(a, first + xcd_tile(blockIdx.x, count), s_u, s_conn, s_tmp);
}

template <bool MINMODE, int TY>
__global__ __launch_bounds__(256) void k_classify2d(TileArgs a, int first, int count)
{
    __shared__ uint32_t s_u[66 * (TY + 2)];
    __shared__ int32_t s_nxt[64 * TY];
    __shared__ uint32_t s_tmp[8];
    tile_nd<2, MINMODE, TY, 1>(a, first + xcd_tile(blockIdx.x, count), s_u, s_nxt, nullptr, s_tmp);
}

TileArgs tile_args(const float* f, const Grid& g, int32_t* lab, int32_t* ptr, const Work& w, int ty, int tz)
{
    TileArgs a{};
    a.f = gptr(f);
    a.lab = gptr(lab);
    a.ptr = gptr(ptr);
    a.ctr = gptr(w.ctr);
    a.mmask = gptr(w.mmask);
    a.smask = gptr(w.smask);
    a.exits = gptr(w.exits);
    a.X = g.dims[g.ndim - 1];
    a.Y = g.dims[g.ndim - 2];
    a.Z = g.ndim == 3 ? g.dims[0] : 1;
    a.tiles_x = (a.X + 63) / 64;
    a.tiles_y = (a.Y + ty - 1) / ty;
    const int tiles_z = (a.Z + tz - 1) / tz;
    a.ntiles = a.tiles_x * a.tiles_y * tiles_z;
    a.cap_exit = (uint32_t)w.cap_exit;
    return a;
}

// Classification of a batch: for each class of fields (2D/3D x maximum/
// minimum graph) one launch covers the work list of (field, tile) items of
// that class, one workgroup per item, which runs the tile code of its field.
template <int NDIM, bool MINMODE, int TY, int TZ>
__global__ __launch_bounds__(256) void k_classify_batched(const BatchPlan* __restrict__ plan, int cls)
{
    constexpr int HALO3 = 66 * (TY + 2) * (TZ + 2);
    constexpr int HALO2 = 66 * (TY + 2);
    constexpr int WORDS = NDIM == 3 ? HALO3 : HALO2 + 64 * TY;
    __shared__ uint32_t s_u[WORDS];
    __shared__ uint32_t s_conn[NDIM == 3 ? 512 : 1];
    __shared__ uint32_t s_tmp[64];
    const EG_GPTR(BatchField) fs = plan->fields;
    const int f0 = plan->class_field[cls], f1 = plan->class_field[cls + 1];
    const int64_t item = plan->class_tile[cls] + blockIdx.x;
    // the field of this item: binary search over the class's tile bases
    int lo = f0, hi = f1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fs[mid].tile_base <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int f = __builtin_amdgcn_readfirstlane(lo);
    const int tile = (int)(item - fs[f].tile_base);
    const TileArgs a = fs[f].ta;
    if constexpr (NDIM == 3)
        tile3d<MINMODE, TY, TZ>(a, tile, s_u, s_conn, s_tmp);
    else
        tile_nd<2, MINMODE, TY, 1>(a, tile, s_u, reinterpret_cast<int32_t*>(s_u + HALO2), nullptr, s_tmp);
}

template <int NDIM, int TY, int TZ>
static void launch_class(int c, unsigned grid, const BatchPlan* dplan, hipStream_t s)
{
    if (c & 1)
        hipLaunchKernelGGL((k_classify_batched<NDIM, true, TY, TZ>), dim3(grid), dim3(256), 0, s, dplan, c);
    else
        hipLaunchKernelGGL((k_classify_batched<NDIM, false, TY, TZ>), dim3(grid), dim3(256), 0, s, dplan, c);
}

hipError_t launch_classify_batched(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    for (int c = 0; c < 4; ++c) {
        const int64_t tiles = hplan.class_tile[c + 1] - hplan.class_tile[c];
        if (tiles <= 0) continue;
        const unsigned grid = (unsigned)tiles;
        const Tuning& tu = hplan.tuning;
        if (c < 2) {
            if (tu.tile2 == 1)
                launch_class<2, 16, 1>(c, grid, dplan, s);
            else
                launch_class<2, 32, 1>(c, grid, dplan, s);
        } else {
            if (tu.tile3 == 1)
                launch_class<3, 4, 16>(c, grid, dplan, s);
            else if (tu.tile3 == 2)
                launch_class<3, 8, 4>(c, grid, dplan, s);
            else
                launch_class<3, 8, 8>(c, grid, dplan, s);
        }
    }
    return hipGetLastError();
}

template <int TY, int TZ>
static void launch_3d(const TileArgs& a, bool minima, int first, int count, hipStream_t s)
{
    if (minima)
        hipLaunchKernelGGL((k_classify3d<true, TY, TZ>), dim3(count), dim3(256), 0, s, a, first, count);
    else
        hipLaunchKernelGGL((k_classify3d<false, TY, TZ>), dim3(count), dim3(256), 0, s, a, first, count);
}

template <int TY>
static void launch_2d(const TileArgs& a, bool minima, int first, int count, hipStream_t s)
{
    if (minima)
        hipLaunchKernelGGL((k_classify2d<true, TY>), dim3(count), dim3(256), 0, s, a, first, count);
    else
        hipLaunchKernelGGL((k_classify2d<false, TY>), dim3(count), dim3(256), 0, s, a, first, count);
}

hipError_t launch_final_tiled(const Grid& g, int32_t* lab, const Work& w, const Tuning& tu, int flag_slot,
                              hipStream_t s)
{
    int ty, tz;
    tile_shape(tu, g.ndim, &ty, &tz);
    const TileArgs a = tile_args(nullptr, g, lab, nullptr, w, ty, tz);
    if (g.ndim == 3) {
        if (tu.tile3 == 1)
            hipLaunchKernelGGL((k_final_tiled<4, 16>), dim3(a.ntiles), dim3(256), 0, s, a, w.exres, tu.hops, flag_slot);
        else if (tu.tile3 == 2)
            hipLaunchKernelGGL((k_final_tiled<8, 4>), dim3(a.ntiles), dim3(256), 0, s, a, w.exres, tu.hops, flag_slot);
        else
            hipLaunchKernelGGL((k_final_tiled<8, 8>), dim3(a.ntiles), dim3(256), 0, s, a, w.exres, tu.hops, flag_slot);
    } else if (g.ndim == 2) {
        if (tu.tile2 == 1)
            hipLaunchKernelGGL((k_final_tiled<16, 1>), dim3(a.ntiles), dim3(256), 0, s, a, w.exres, tu.hops, flag_slot);
        else
            hipLaunchKernelGGL((k_final_tiled<32, 1>), dim3(a.ntiles), dim3(256), 0, s, a, w.exres, tu.hops, flag_slot);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_classify_tiled(const float* f, const Grid& g, bool minima, int32_t* lab, int32_t* ptr,
                                 const Work& w, const Tuning& tu, hipStream_t s, int64_t first, int64_t count)
{
    int ty, tz;
    tile_shape(tu, g.ndim, &ty, &tz);
    const TileArgs a = tile_args(f, g, lab, ptr, w, ty, tz);
    if (count < 0) {
        first = 0;
        count = a.ntiles;
    }
    if (first < 0 || first + count > a.ntiles) return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    const int f0 = (int)first, n = (int)count;
    if (g.ndim == 3) {
        if (tu.tile3 == 1)
            launch_3d<4, 16>(a, minima, f0, n, s);
        else if (tu.tile3 == 2)
            launch_3d<8, 4>(a, minima, f0, n, s);
        else
            launch_3d<8, 8>(a, minima, f0, n, s);
    } else if (g.ndim == 2) {
        if (tu.tile2 == 1)
            launch_2d<16>(a, minima, f0, n, s);
        else
            launch_2d<32>(a, minima, f0, n, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace eg
