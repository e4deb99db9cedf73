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

template <int NDIM, bool MINMODE, int TY, int TZ>
__global__ __launch_bounds__(256) void k_classify_tiled(const float* __restrict__ f, int X, int Y, int Z, int tiles_x,
                                                        int tiles_y, int ntiles, int32_t* __restrict__ lab,
                                                        int32_t* __restrict__ ptr, uint32_t* __restrict__ ctr,
                                                        uint32_t* __restrict__ umax, uint32_t cap_max,
                                                        uint32_t* __restrict__ usad, uint32_t cap_sad)
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

    __shared__ uint32_t s_u[HALO];
    __shared__ int32_t s_nxt[TILE];
    __shared__ uint32_t s_conn[NDIM == 3 ? 512 : 1];

    const int tid = threadIdx.x, lx = tid & 63, wv = tid >> 6;
    int b = blockIdx.x;
    if ((ntiles & 7) == 0) b = (b & 7) * (ntiles >> 3) + (b >> 3);
    const int tx = b % tiles_x;
    const int rr = b / tiles_x;
    const int ty = rr % tiles_y;
    const int tz = rr / tiles_y;
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
        int n = -1;
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
                n = inside ? (lz2 * TY + ly2) * TX + lx2 : -(pv + 1);
            }
            if (ptr) ptr[v] = pv;
        }
        nxt[k] = n;
        s_nxt[li] = n;
        wave_append(is_max, (uint32_t)v, &ctr[C_NMAX], umax, cap_max);
        wave_append(is_sad, (uint32_t)v, &ctr[C_NSAD], usad, cap_sad);
    }
    if (__ballot(nan) != 0 && __lane_id() == 0) atomicOr(&ctr[C_NAN], 1u);
    __syncthreads();

    double_tile_chains<VPT>(nxt, s_nxt, [&](int k) { return ((k / YPT) * TY + wv + 4 * (k % YPT)) * TX + lx; });
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
__global__ __launch_bounds__(256) void k_classify3d(const float* __restrict__ f, int X, int Y, int Z, int tiles_x,
                                                    int tiles_y, int ntiles, int32_t* __restrict__ lab,
                                                    int32_t* __restrict__ ptr, uint32_t* __restrict__ ctr,
                                                    uint32_t* __restrict__ umax, uint32_t cap_max,
                                                    uint32_t* __restrict__ usad, uint32_t cap_sad)
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

    __shared__ uint32_t s_u[HALO];
    __shared__ uint32_t s_conn[512];
    int32_t* s_nxt = reinterpret_cast<int32_t*>(s_u);

    const int tid = threadIdx.x, lx = tid & 63, wv = tid >> 6;
    int b = blockIdx.x;
    if ((ntiles & 7) == 0) b = (b & 7) * (ntiles >> 3) + (b >> 3);
    const int tx = b % tiles_x;
    const int rr = b / tiles_x;
    const int ty = rr % tiles_y;
    const int tz = rr / tiles_y;
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
            int n = -1;
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
                    n = inside ? (lz2 * TY + ly2) * TX + lx2 : -(pv + 1);
                }
                if (ptr) ptr[v] = pv;
            }
            nxt[c * TZ + lz] = n;
            wave_append(is_max, (uint32_t)v, &ctr[C_NMAX], umax, cap_max);
            wave_append(is_sad, (uint32_t)v, &ctr[C_NSAD], usad, cap_sad);
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

template <bool MINMODE, int TY, int TZ>
static hipError_t launch_3d_t(const float* f, const Grid& g, int32_t* lab, int32_t* ptr, const Work& w,
                              int64_t cap_max, int64_t cap_sad, hipStream_t s)
{
    const int X = g.dims[2], Y = g.dims[1], Z = g.dims[0];
    const int tiles_x = (X + 63) / 64, tiles_y = (Y + TY - 1) / TY, tiles_z = (Z + TZ - 1) / TZ;
    const int64_t ntiles = (int64_t)tiles_x * tiles_y * tiles_z;
    hipLaunchKernelGGL((k_classify3d<MINMODE, TY, TZ>), dim3((unsigned)ntiles), dim3(256), 0, s, f, X, Y, Z,
                       tiles_x, tiles_y, (int)ntiles, lab, ptr, w.ctr, w.umax, (uint32_t)cap_max, w.usad,
                       (uint32_t)cap_sad);
    return hipGetLastError();
}

template <int NDIM, bool MINMODE, int TY, int TZ>
static hipError_t launch_tiled_t(const float* f, const Grid& g, int32_t* lab, int32_t* ptr, const Work& w,
                                 int64_t cap_max, int64_t cap_sad, hipStream_t s)
{
    const int X = g.dims[NDIM - 1], Y = g.dims[NDIM - 2], Z = NDIM == 3 ? g.dims[0] : 1;
    const int tiles_x = (X + 63) / 64, tiles_y = (Y + TY - 1) / TY, tiles_z = (Z + TZ - 1) / TZ;
    const int64_t ntiles = (int64_t)tiles_x * tiles_y * tiles_z;
    hipLaunchKernelGGL((k_classify_tiled<NDIM, MINMODE, TY, TZ>), dim3((unsigned)ntiles), dim3(256), 0, s, f, X, Y,
                       Z, tiles_x, tiles_y, (int)ntiles, lab, ptr, w.ctr, w.umax, (uint32_t)cap_max, w.usad,
                       (uint32_t)cap_sad);
    return hipGetLastError();
}

hipError_t launch_classify_tiled(const float* f, const Grid& g, bool minima, int32_t* lab, int32_t* ptr,
                                 const Work& w, int64_t cap_max, int64_t cap_sad, hipStream_t s)
{
    if (g.ndim == 3)
        return minima ? launch_3d_t<true, 8, 8>(f, g, lab, ptr, w, cap_max, cap_sad, s)
                      : launch_3d_t<false, 8, 8>(f, g, lab, ptr, w, cap_max, cap_sad, s);
    if (g.ndim == 2)
        return minima ? launch_tiled_t<2, true, 32, 1>(f, g, lab, ptr, w, cap_max, cap_sad, s)
                      : launch_tiled_t<2, false, 32, 1>(f, g, lab, ptr, w, cap_max, cap_sad, s);
    return hipErrorInvalidValue;
}

}  // namespace eg
