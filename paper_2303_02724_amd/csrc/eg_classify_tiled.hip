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

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

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

// Tile-local successor index -> global id (TX = 64).
template <int TY>
__device__ __forceinline__ int tile_to_global(int n, int x0, int y0, int z0, int SY, int SZ)
{
    const int lx = n & 63, ly = (n >> 6) % TY, lz = (n >> 6) / TY;
    return (z0 + lz) * SZ + (y0 + ly) * SY + x0 + lx;
}

// Resolve the tile's successor array by pointer doubling.  cur[k] holds the
// successor of this thread's k-th vertex (s_idx(k) is its tile index): >= 0 a
// tile index (a maximum is its own successor), < 0 the exit code of the first
// vertex outside the tile.  Each round replaces every successor by the
// successor's successor, so log2 of the longest in-tile path bounds the
// rounds.  On return cur[k] is a tile-local maximum (>= 0) or an exit code.
// Must be called by the whole workgroup, after s_nxt holds every successor.
template <int VPT, class Idx>
__device__ __forceinline__ void double_tile_chains(int (&cur)[VPT], int32_t* s_nxt, Idx s_idx)
{
    for (;;) {
        int changed = 0;
#pragma unroll
        for (int k = 0; k < VPT; ++k) {
            const int n = cur[k];
            if (n >= 0) {
                const int m = s_nxt[n];
                changed |= m != n;
                cur[k] = m;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < VPT; ++k) s_nxt[s_idx(k)] = cur[k];
        if (!__syncthreads_or(changed)) break;
    }
}

// After the tile's chains are resolved, cur[k] is a tile-local maximum (>= 0)
// or -(h + 1) for the exit at halo position h.  The tile flags the halo
// positions used as exits, numbers them with a block scan, appends their
// vertex ids to the exit list (one atomic per tile) and turns every exit into
// an exit-list code, so the label pass resolves each exit once.  A tile that
// does not fit in the list keeps vertex-id codes.  s_words must hold
// (HALO + 1) / 2 words of LDS that nobody else uses any more.
template <int VPT, int HALO, class H2G>
__device__ __forceinline__ void publish_exits(int (&cur)[VPT], uint32_t* s_words, uint32_t* s_tmp,
                                              uint32_t* __restrict__ ctr, uint32_t* __restrict__ exits,
                                              uint32_t cap_exit, int N, H2G h2g)
{
    constexpr int WORDS = (HALO + 1) / 2;
    constexpr int SEG = (HALO + 255) / 256;
    uint16_t* s_map = reinterpret_cast<uint16_t*>(s_words);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i < WORDS; i += 256) s_words[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VPT; ++k)
        if (cur[k] < 0) s_map[-cur[k] - 1] = 1;
    __syncthreads();
    const int lo = tid * SEG;
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < SEG; ++i)
        if (lo + i < HALO) cnt += s_map[lo + i];
    // block-wide exclusive scan of the counts
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_tmp[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int k = 0; k < w; ++k) pre += s_tmp[k];
    const uint32_t total = s_tmp[0] + s_tmp[1] + s_tmp[2] + s_tmp[3];
    if (tid == 0) s_tmp[4] = total ? atomicAdd(&ctr[C_NEXIT], total) : 0u;
    __syncthreads();
    const uint32_t base = s_tmp[4];
    const bool ok = (uint64_t)base + total <= cap_exit;
    uint32_t r = pre + inc - cnt;
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
        const int h = lo + i;
        if (h < HALO && s_map[h]) {
            // entries below the capacity are always written, so the list
            // never holds garbage even when this tile does not use it
            if (base + r < cap_exit) exits[base + r] = (uint32_t)h2g(h);
            s_map[h] = (uint16_t)r;
            ++r;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        if (cur[k] < 0) {
            const int h = -cur[k] - 1;
            cur[k] = ok ? exit_list_code(N, base + s_map[h]) : -(h2g(h) + 1);
        }
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
    constexpr int YPT = TY / 4;
    constexpr int VPT = YPT * TZ;
    constexpr int ZH = NDIM == 3 ? 1 : 0;  // halo depth along z
    const float* __restrict__ f = a.f;
    const int X = a.X, Y = a.Y, Z = a.Z;
    int32_t* __restrict__ lab = a.lab;
    int32_t* __restrict__ ptr = a.ptr;
    uint32_t* __restrict__ ctr = a.ctr;

    const int tid = threadIdx.x, lx = tid & 63, wv = tid >> 6;
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
    {
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
    int nxt[VPT];
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int ly = wv + 4 * (k % YPT);
        const int lz = k / YPT;
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        const bool in = gx < X && gy < Y && gz < Z;
        const int li = (lz * TY + ly) * TX + lx;
        int n = li;  // vertices outside the grid stay put and are never written
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
                n = li;  // a maximum points to itself
            } else {
                const int dz = NDIM == 3 ? (int)((Pack<NDIM>::z >> (2 * best_j)) & 3u) - 1 : 0;
                const int dy = (int)((Pack<NDIM>::y >> (2 * best_j)) & 3u) - 1;
                const int dx = (int)((Pack<NDIM>::x >> (2 * best_j)) & 3u) - 1;
                pv = v + dz * SZ + dy * SY + dx;
                const int lz2 = lz + dz, ly2 = ly + dy, lx2 = lx + dx;
                const bool inside = (unsigned)lz2 < (unsigned)TZ && (unsigned)ly2 < (unsigned)TY &&
                                    (unsigned)lx2 < (unsigned)TX;
                n = inside ? (lz2 * TY + ly2) * TX + lx2 : -(c + (dz * HY + dy) * HX + dx + 1);
            }
            if (ptr) ptr[v] = pv;
        }
        nxt[k] = n;
        s_nxt[li] = n;
        wave_append(is_max, (uint32_t)v, &ctr[C_NMAX], a.umax, a.cap_max);
        wave_append(is_sad, (uint32_t)v, &ctr[C_NSAD], a.usad, a.cap_sad);
    }
    if (__ballot(nan) != 0 && __lane_id() == 0) atomicOr(&ctr[C_NAN], 1u);
    __syncthreads();

    double_tile_chains<VPT>(nxt, s_nxt, [&](int k) { return ((k / YPT) * TY + wv + 4 * (k % YPT)) * TX + lx; });
    const int N = X * Y * Z;
    publish_exits<VPT, HALO>(nxt, s_u, s_tmp, ctr, a.exits, a.cap_exit, N, [&](int h) {
        const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
        return (z0 + hz - ZH) * SZ + (y0 + hy - 1) * SY + x0 + hx - 1;
    });
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
        const int ly = wv + 4 * (k % YPT);
        const int lz = k / YPT;
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        const int n = nxt[k];
        if (gx < X && gy < Y && gz < Z) lab[gz * SZ + gy * SY + gx] = n >= 0 ? tile_to_global<TY>(n, x0, y0, z0, SY, SZ) : n;
    }
}

// 3D variant tuned for large grids.  Rows of the halo are loaded aligned
// (one 256-byte wave load per row plus the two edge columns); each thread
// walks YPT columns of the tile along z with a sliding window of three planes
// of the seven in-plane positions a vertex's neighbourhood touches, so a
// vertex costs 7 LDS reads instead of 15; pointer targets stay in registers
// until the halo is no longer needed, then reuse its LDS for the tile-local
// chains, which are resolved by pointer doubling.
template <int NDIM_, int J>
struct Win {
    // index of row J's (dy, dx) among the seven window positions
    // (-1,-1) (-1,0) (0,-1) (0,0) (0,1) (1,0) (1,1), and its plane dz + 1
    static constexpr int dy = Row<3, J>::dy, dx = Row<3, J>::dx, dz = Row<3, J>::dz;
    static constexpr int pos = dy < 0 ? (dx < 0 ? 0 : 1) : dy == 0 ? (dx < 0 ? 2 : dx == 0 ? 3 : 4) : (dx == 0 ? 5 : 6);
    static constexpr int plane = dz + 1;
};

template <bool MINMODE, int TY, int TZ>
__device__ __forceinline__ void tile3d(const TileArgs& a, int b, uint32_t* s_u, uint32_t* s_conn, uint32_t* s_tmp)
{
    constexpr int K = 14;
    constexpr int TX = 64;
    constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    constexpr int HALO = HX * HY * HZ;
    constexpr int TILE = TX * TY * TZ;
    constexpr int YPT = TY / 4;
    constexpr int VPT = YPT * TZ;
    static_assert(TILE <= HALO, "the chains reuse the halo's LDS");
    static_assert(TY % 4 == 0, "four waves split the y rows");
    const float* __restrict__ f = a.f;
    const int X = a.X, Y = a.Y, Z = a.Z;
    int32_t* __restrict__ lab = a.lab;
    int32_t* __restrict__ ptr = a.ptr;
    uint32_t* __restrict__ ctr = a.ctr;
    int32_t* s_nxt = reinterpret_cast<int32_t*>(s_u);

    const int tid = threadIdx.x, lx = tid & 63, wv = tid >> 6;
    const int tx = b % a.tiles_x;
    const int rr = b / a.tiles_x;
    const int ty = rr % a.tiles_y;
    const int tz = rr / a.tiles_y;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int SY = X;
    const int SZ = X * Y;

    bool nan = false;
    {
        // every row load of this wave is issued before the first one is used
        constexpr int ROWS = HY * HZ;
        constexpr int RPW = (ROWS + 3) / 4;
        const int gx = x0 + lx;
        const bool xin = gx < X;
        // edge columns: lane 0 -> x0 - 1, lane 1 -> x0 + 64
        const int ex = lx == 0 ? x0 - 1 : x0 + TX;
        const bool ein = lx < 2 && (unsigned)ex < (unsigned)X;
        const int ehx = lx == 0 ? 0 : HX - 1;
        float vals[RPW], evals[RPW];
        bool vin[RPW], vein[RPW];
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int row = wv + 4 * i;
            const int hy = row % HY, hz = row / HY;
            const int gy = y0 + hy - 1, gz = z0 + hz - 1;
            const bool rin = row < ROWS && (unsigned)gy < (unsigned)Y && (unsigned)gz < (unsigned)Z;
            const int rbase = gz * SZ + gy * SY;
            vin[i] = rin && xin;
            vein[i] = rin && ein;
            vals[i] = vin[i] ? f[rbase + gx] : 0.0f;
            evals[i] = vein[i] ? f[rbase + ex] : 0.0f;
        }
        const uint32_t conn_a = c_conn3.w[tid], conn_b = c_conn3.w[tid + 256];
        s_conn[tid] = conn_a;
        s_conn[tid + 256] = conn_b;
#pragma unroll
        for (int i = 0; i < RPW; ++i) {
            const int row = wv + 4 * i;
            if (row < ROWS) {
                const int hy = row % HY, hz = row / HY;
                const float val = vals[i];
                s_u[row * HX + lx + 1] = vin[i] ? mode_key<MINMODE>(val) : 0u;
                nan |= vin[i] && (hy >= 1 && hy <= TY && hz >= 1 && hz <= TZ) && (val != val);
                if (lx < 2) s_u[row * HX + ehx] = vein[i] ? mode_key<MINMODE>(evals[i]) : 0u;
            }
        }
    }
    __syncthreads();

    int nxt[VPT];
#pragma unroll
    for (int c = 0; c < YPT; ++c) {
        const int ly = wv + 4 * c;
        const int gy = y0 + ly;
        const int gx = x0 + lx;
        // window[p][q]: plane hz = lz + p, position q
        uint32_t win[3][7];
        auto load_plane = [&](uint32_t* w, int hz) {
            const int base = (hz * HY + ly + 1) * HX + lx + 1;
            w[0] = s_u[base - HX - 1];
            w[1] = s_u[base - HX];
            w[2] = s_u[base - 1];
            w[3] = s_u[base];
            w[4] = s_u[base + 1];
            w[5] = s_u[base + HX];
            w[6] = s_u[base + HX + 1];
        };
        load_plane(win[0], 0);
        load_plane(win[1], 1);
#pragma unroll
        for (int lz = 0; lz < TZ; ++lz) {
            load_plane(win[(lz + 2) % 3], lz + 2);
            const int gz = z0 + lz;
            const bool in = gx < X && gy < Y && gz < Z;
            const uint32_t uv = win[(lz + 1) % 3][3];
            uint32_t up = 0, best_u = 0;
            int best_j = K;
            static_for<0, K + 1>([&](auto step) {
                constexpr int st = decltype(step)::value;
                constexpr int pos = MINMODE ? K - st : st;
                if constexpr (pos == K / 2) {
                    if (uv >= best_u) {
                        best_u = uv;
                        best_j = K;
                    }
                } else {
                    constexpr int j = pos < K / 2 ? pos : pos - 1;
                    using WJ = Win<3, j>;
                    constexpr bool wins_tie = (j >= K / 2) != MINMODE;
                    const uint32_t u = win[(lz + WJ::plane) % 3][WJ::pos];
                    const bool above = wins_tie ? (u >= uv) : (u > uv);
                    up |= uint32_t(above) << j;
                    if (u >= best_u) {
                        best_u = u;
                        best_j = j;
                    }
                }
            });
            const bool is_max = in && up == 0;
            const bool is_sad = in && up != 0 && !((s_conn[up >> 5] >> (up & 31)) & 1u);
            const int v = gz * SZ + gy * SY + gx;
            int n = (lz * TY + ly) * TX + lx;  // vertices outside the grid stay put
            if (in) {
                int pv = v;
                if (best_j == K) {
                    n = (lz * TY + ly) * TX + lx;  // a maximum points to itself
                } else {
                    const int dz = (int)((Pack<3>::z >> (2 * best_j)) & 3u) - 1;
                    const int dy = (int)((Pack<3>::y >> (2 * best_j)) & 3u) - 1;
                    const int dx = (int)((Pack<3>::x >> (2 * best_j)) & 3u) - 1;
                    pv = v + dz * SZ + dy * SY + dx;
                    const int lz2 = lz + dz, ly2 = ly + dy, lx2 = lx + dx;
                    const bool inside = (unsigned)lz2 < (unsigned)TZ && (unsigned)ly2 < (unsigned)TY &&
                                        (unsigned)lx2 < (unsigned)TX;
                    const int hpos = ((lz + 1 + dz) * HY + ly + 1 + dy) * HX + lx + 1 + dx;
                    n = inside ? (lz2 * TY + ly2) * TX + lx2 : -(hpos + 1);
                }
                if (ptr) ptr[v] = pv;
            }
            nxt[c * TZ + lz] = n;
            wave_append(is_max, (uint32_t)v, &ctr[C_NMAX], a.umax, a.cap_max);
            wave_append(is_sad, (uint32_t)v, &ctr[C_NSAD], a.usad, a.cap_sad);
        }
    }
    if (__ballot(nan) != 0 && __lane_id() == 0) atomicOr(&ctr[C_NAN], 1u);
    __syncthreads();  // halo no longer read: its LDS now holds the chains
#pragma unroll
    for (int c = 0; c < YPT; ++c)
#pragma unroll
        for (int lz = 0; lz < TZ; ++lz) s_nxt[(lz * TY + wv + 4 * c) * TX + lx] = nxt[c * TZ + lz];
    __syncthreads();
    // follow every chain inside the tile: entries >= 0 are tile-local
    // successors (a maximum is its own successor), entries < 0 are
    // -(id + 1) of the first vertex outside the tile
    double_tile_chains<VPT>(nxt, s_nxt, [&](int k) { return ((k % TZ) * TY + wv + 4 * (k / TZ)) * TX + lx; });
    publish_exits<VPT, HALO>(nxt, s_u, s_tmp, ctr, a.exits, a.cap_exit, X * Y * Z, [&](int h) {
        const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
        return (z0 + hz - 1) * SZ + (y0 + hy - 1) * SY + x0 + hx - 1;
    });
#pragma unroll
    for (int c = 0; c < YPT; ++c) {
        const int ly = wv + 4 * c;
        const int gx = x0 + lx, gy = y0 + ly;
#pragma unroll
        for (int lz = 0; lz < TZ; ++lz) {
            const int gz = z0 + lz;
            const int n = nxt[c * TZ + lz];
            if (gx < X && gy < Y && gz < Z) lab[gz * SZ + gy * SY + gx] = n >= 0 ? tile_to_global<TY>(n, x0, y0, z0, SY, SZ) : n;
        }
    }
}

// Tiles of one XCD are consecutive in memory: workgroups are dispatched to
// the eight XCDs round-robin, so block b takes tile (b % 8) * (T / 8) + b / 8.
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    return (ntiles & 7) == 0 ? (b & 7) * (ntiles >> 3) + (b >> 3) : b;
}

template <bool MINMODE, int TY, int TZ>
__global__ __launch_bounds__(256) void k_classify3d(TileArgs a)
{
    constexpr int HALO = 66 * (TY + 2) * (TZ + 2);
    __shared__ uint32_t s_u[HALO];
    __shared__ uint32_t s_conn[512];
    __shared__ uint32_t s_tmp[8];
    tile3d<MINMODE, TY, TZ>(a, xcd_tile(blockIdx.x, a.ntiles), s_u, s_conn, s_tmp);
}

template <bool MINMODE, int TY>
__global__ __launch_bounds__(256) void k_classify2d(TileArgs a)
{
    __shared__ uint32_t s_u[66 * (TY + 2)];
    __shared__ int32_t s_nxt[64 * TY];
    __shared__ uint32_t s_tmp[8];
    tile_nd<2, MINMODE, TY, 1>(a, xcd_tile(blockIdx.x, a.ntiles), s_u, s_nxt, nullptr, s_tmp);
}

TileArgs tile_args(const float* f, const Grid& g, int32_t* lab, int32_t* ptr, const Work& w, int64_t cap_max,
                   int64_t cap_sad, int ty, int tz)
{
    TileArgs a{};
    a.f = f;
    a.lab = lab;
    a.ptr = ptr;
    a.ctr = w.ctr;
    a.umax = w.umax;
    a.usad = w.usad;
    a.exits = w.exits;
    a.X = g.dims[g.ndim - 1];
    a.Y = g.dims[g.ndim - 2];
    a.Z = g.ndim == 3 ? g.dims[0] : 1;
    a.tiles_x = (a.X + 63) / 64;
    a.tiles_y = (a.Y + ty - 1) / ty;
    const int tiles_z = (a.Z + tz - 1) / tz;
    a.ntiles = a.tiles_x * a.tiles_y * tiles_z;
    a.cap_max = (uint32_t)cap_max;
    a.cap_sad = (uint32_t)cap_sad;
    a.cap_exit = (uint32_t)w.cap_exit;
    return a;
}

// Persistent classification of a batch: a fixed grid walks the work list of
// (field, tile) items of all fields; each item runs the 2D or 3D tile code of
// its field.  The LDS of the largest tile type is shared by both.
__device__ __forceinline__ int find_field(const BatchField* fs, int count, int64_t item, int64_t BatchField::*base)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fs[mid].*base <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_classify_batched(const BatchPlan* __restrict__ plan)
{
    constexpr int HALO3 = 66 * (kTile3Y + 2) * (kTile3Z + 2);
    constexpr int HALO2 = 66 * (kTile2Y + 2);
    static_assert(HALO2 + 64 * kTile2Y <= HALO3, "2D tile fits in the 3D tile's LDS");
    __shared__ uint32_t s_u[HALO3];
    __shared__ uint32_t s_conn[512];
    __shared__ uint32_t s_tmp[8];
    const int count = plan->count;
    const int64_t total = plan->total_tiles;
    const BatchField* fs = plan->fields;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int f = __builtin_amdgcn_readfirstlane(find_field(fs, count, item, &BatchField::tile_base));
        const int tile = (int)(item - fs[f].tile_base);
        const TileArgs a = fs[f].ta;
        const int ndim = fs[f].ndim, minima = fs[f].minima;
        __syncthreads();  // the previous item's LDS reads are done
        if (ndim == 3) {
            if (minima)
                tile3d<true, kTile3Y, kTile3Z>(a, tile, s_u, s_conn, s_tmp);
            else
                tile3d<false, kTile3Y, kTile3Z>(a, tile, s_u, s_conn, s_tmp);
        } else {
            int32_t* s_nxt = reinterpret_cast<int32_t*>(s_u + HALO2);
            if (minima)
                tile_nd<2, true, kTile2Y, 1>(a, tile, s_u, s_nxt, nullptr, s_tmp);
            else
                tile_nd<2, false, kTile2Y, 1>(a, tile, s_u, s_nxt, nullptr, s_tmp);
        }
    }
}

hipError_t launch_classify_batched(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    // five 28 KB workgroups fit a CU; 256 CUs
    const int64_t grid = hplan.total_tiles < 1280 ? hplan.total_tiles : 1280;
    hipLaunchKernelGGL(k_classify_batched, dim3((unsigned)(grid > 0 ? grid : 1)), dim3(256), 0, s, dplan);
    return hipGetLastError();
}

hipError_t launch_classify_tiled(const float* f, const Grid& g, bool minima, int32_t* lab, int32_t* ptr,
                                 const Work& w, int64_t cap_max, int64_t cap_sad, hipStream_t s)
{
    if (g.ndim == 3) {
        const TileArgs a = tile_args(f, g, lab, ptr, w, cap_max, cap_sad, kTile3Y, kTile3Z);
        if (minima)
            hipLaunchKernelGGL((k_classify3d<true, kTile3Y, kTile3Z>), dim3(a.ntiles), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_classify3d<false, kTile3Y, kTile3Z>), dim3(a.ntiles), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    if (g.ndim == 2) {
        const TileArgs a = tile_args(f, g, lab, ptr, w, cap_max, cap_sad, kTile2Y, 1);
        if (minima)
            hipLaunchKernelGGL((k_classify2d<true, kTile2Y>), dim3(a.ntiles), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_classify2d<false, kTile2Y>), dim3(a.ntiles), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

}  // namespace eg
