// eg_classify.hip -- per-vertex classification, labels and saddle reps.
//
// k_classify_generic  stages (a) and (c) of the method for n = 1: one
//   thread per vertex reads its closed neighbourhood, forms the upper-link
//   mask (Sec. 3.3), the steepest-ascent pointer (highest upper-link vertex,
//   Sec. 3.3) and decides maximum (empty upper link) / saddle (>= 2
//   components, Table 1) by set algebra on the link's rows (eg_link.h).
// k_classify_slab  the same for n = 4, 5 and 6, reading the neighbourhood
//   from planes of keys staged in LDS.
// k_exit_*, k_final  stage (b): pointer jumping until every vertex names its
//   maximum (the end of the walk of Alg. 2).
#include "eg_internal.h"
#include "eg_rows.h"
#include "eg_link.h"

namespace eg {

__global__ void k_init(uint32_t* __restrict__ ctr, int32_t* __restrict__ header)
{
    const int i = threadIdx.x;
    if (i < C_SLOTS) ctr[i] = 0;
    if (header && i < EG_H_SLOTS) header[i] = 0;
}

hipError_t launch_init(uint32_t* ctr, int32_t* header, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, s, ctr, header);
    return hipGetLastError();
}

// Visit the closed neighbourhood of v in the order in which later vertices
// win ties; fills the upper-link mask and the steepest-ascent target.  The
// rows are unrolled, one load per row under the row's own branch; a row's
// linear offset and the boundary bits that rule it out follow from the
// compile-time rows and the grid strides st[] (uniform, scalar work).
template <int NDIM, bool MINMODE>
__device__ __forceinline__ void scan_unrolled(const uint32_t* __restrict__ keys, const int* st, int v,
                                              uint32_t bits, uint32_t uv, Mask<NDIM>& up, int& best)
{
    constexpr Rows<NDIM> R = make_rows_ce<NDIM>();
    constexpr int K = Rows<NDIM>::K;
    uint32_t best_u = 0;
    best = v;
    auto visit = [&](int j) {
        int lin = 0;
        uint32_t forb = 0;
#pragma unroll
        for (int i = 0; i < NDIM; ++i) {
            lin += R.d[j][i] * st[i];
            forb |= R.d[j][i] < 0 ? 1u << (2 * i) : R.d[j][i] > 0 ? 1u << (2 * i + 1) : 0u;
        }
        if ((bits & forb) == 0) {
            const int u_id = v + lin;
            const uint32_t u = keys[u_id];
            const bool above = row_wins_tie<MINMODE>(j, K) ? (u >= uv) : (u > uv);
            up |= Mask<NDIM>(above) << j;
            if (u >= best_u) {
                best_u = u;
                best = u_id;
            }
        }
    };
    auto self = [&]() {
        if (uv >= best_u) {
            best_u = uv;
            best = v;
        }
    };
    if (!MINMODE) {
#pragma unroll
        for (int j = 0; j < K / 2; ++j) visit(j);
        self();
#pragma unroll
        for (int j = K / 2; j < K; ++j) visit(j);
    } else {
#pragma unroll
        for (int j = K - 1; j >= K / 2; --j) visit(j);
        self();
#pragma unroll
        for (int j = K / 2 - 1; j >= 0; --j) visit(j);
    }
}

template <int NDIM>
__device__ __forceinline__ uint32_t boundary_bits(const Grid& g, int v)
{
    uint32_t bits = 0;
    int rem = v;
#pragma unroll
    for (int i = NDIM - 1; i >= 0; --i) {
        const int d = g.dims[i];
        const int c = rem % d;
        rem /= d;
        bits |= boundary_bit(c, d, i);
    }
    return bits;
}

__global__ __launch_bounds__(256) void k_zero_words(uint64_t* __restrict__ a, uint64_t* __restrict__ b, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = 0;
        b[i] = 0;
    }
}

// OR the bits of the lanes with `pred` into the row-padded mask: lanes that
// share a word form a run of consecutive lanes (consecutive x), and the first
// lane of each run writes the run's bits with one atomic.  Words are shared
// only by the runs at either end of a wave, so atomics rarely meet.
__device__ __forceinline__ void mask_or(bool pred, int64_t word, int bit, uint64_t* __restrict__ mask)
{
    const uint64_t b = __ballot(pred);
    if (b == 0) return;
    const int lane = __lane_id();
    const int64_t prev = __shfl_up(word, 1);
    const bool lead = lane == 0 || prev != word;
    const uint64_t leads = __ballot(lead);
    const uint64_t later = lane == 63 ? 0ull : (leads >> (lane + 1)) << (lane + 1);
    const int next = later ? __ffsll((unsigned long long)later) - 1 : 64;
    const int len = next - lane;
    const uint64_t run = len >= 64 ? ~0ull : ((1ull << len) - 1ull);
    const uint64_t bits = ((b >> lane) & run) << bit;
    if (lead && word >= 0 && bits) atomicOr((unsigned long long*)&mask[word], (unsigned long long)bits);
}

// Order keys of every vertex (reversed for the minimum graph), once, for the
// grids whose classification reads neighbours from memory; NaN is flagged.
template <bool MINMODE>
__global__ __launch_bounds__(256) void k_keys(const float* __restrict__ f, int N, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ ctr)
{
    bool nan = false;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const float x = f[i];
        nan |= x != x;
        keys[i] = mode_key<MINMODE>(x);
    }
    if (__ballot(nan) != 0 && __lane_id() == 0) atomicOr(&ctr[C_NAN], 1u);
}

template <int NDIM, bool MINMODE>
__global__ __launch_bounds__(256) void k_classify_generic(const uint32_t* __restrict__ keys, Grid g, LinkTable t,
                                                          int32_t* __restrict__ lab, int32_t* __restrict__ ptr,
                                                          uint64_t* __restrict__ mmask, uint64_t* __restrict__ smask)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    bool is_max = false, is_sad = false;
    if (v < g.N) {
        const uint32_t bits = boundary_bits<NDIM>(g, v);
        const uint32_t uv = keys[v];
        Mask<NDIM> up = 0;
        int best;
        int st[NDIM];
        st[NDIM - 1] = 1;
#pragma unroll
        for (int i = NDIM - 2; i >= 0; --i) st[i] = st[i + 1] * g.dims[i + 1];
        scan_unrolled<NDIM, MINMODE>(keys, st, v, bits, uv, up, best);
        is_max = up == 0;
        if (!is_max) is_sad = !link_connected<NDIM>(up);
        lab[v] = is_max ? v : -(best + 1);  // final label, or "same as best"
        if (ptr) ptr[v] = best;
    }
    // this vertex's bit in the row-padded masks (rows run along the last axis)
    const int X = g.dims[NDIM - 1];
    const int row = v / X, x = v - row * X;
    const int64_t word = v < g.N ? (int64_t)row * ((X + 63) >> 6) + (x >> 6) : -1;
    mask_or(is_max, word, x & 63, mmask);
    mask_or(is_sad, word, x & 63, smask);
}

// -------------------------------------------------------- 4D-6D slab tiles
//
// k_classify_slab  the same outputs as k_classify_generic for n = 4, 5 and 6,
//   with the neighbourhood read from LDS instead of through the caches (62
//   gathers per vertex in 5D, 126 in 6D, leave a kernel that reads them from
//   memory bound by the memory pipeline, not by arithmetic).  A block owns a
//   tile of the hyperplanes orthogonal to axis 0 (2x4x32 vertices in 4D,
//   2x2x2x32 in 5D, 2x2x2x2x16 in 6D, one per thread) and a run of zc
//   consecutive planes along axis 0.  It keeps three
//   consecutive planes of the tile plus a one-vertex halo in a ring in LDS
//   (positions outside the grid hold key 0, below every vertex, so every row
//   of the table may be read), and slides it along axis 0: while one plane is
//   classified, the loads of the plane after next are in flight.
template <int NDIM>
__host__ __device__ constexpr int slab_e(int i)  // interior extent along axis i (1..n-1)
{
    return i == NDIM - 1 ? (NDIM == 6 ? 16 : 32) : (NDIM == 4 && i == 2) ? 4 : 2;
}
template <int NDIM>
__host__ __device__ constexpr int slab_hs(int i)  // LDS stride of axis i in a halo plane
{
    int s = 1;
    for (int k = NDIM - 1; k > i; --k) s *= slab_e<NDIM>(k) + 2;
    return s;
}
template <int NDIM>
__host__ __device__ constexpr int slab_size()  // keys per halo plane
{
    return slab_hs<NDIM>(0);
}
template <int NDIM>
__host__ __device__ constexpr int slab_inner()  // vertices per tile plane
{
    int s = 1;
    for (int k = 1; k < NDIM; ++k) s *= slab_e<NDIM>(k);
    return s;
}

struct SlabArgs {
    int32_t zc;                  // planes along axis 0 per block
    int32_t zblocks;             // blocks along axis 0: ceil(dims[0] / zc)
    int32_t nt[EG_MAX_NDIM];     // tiles along axes 1..n-1
    int32_t st[EG_MAX_NDIM];     // grid strides (st[n-1] = 1)
    int32_t rows_per_plane;      // rows of X vertices in one plane (st[0] / X)
};

template <int NDIM, bool MINMODE>
__global__ __launch_bounds__(256) void k_classify_slab(const uint32_t* __restrict__ keys, Grid g, LinkTable t,
                                                       SlabArgs a, int32_t* __restrict__ lab,
                                                       int32_t* __restrict__ ptr, uint64_t* __restrict__ mmask,
                                                       uint64_t* __restrict__ smask)
{
    constexpr int K = Rows<NDIM>::K;
    constexpr Rows<NDIM> R = make_rows_ce<NDIM>();
    constexpr int S = slab_size<NDIM>();
    constexpr int PER = (S + 255) / 256;
    constexpr int EX = slab_e<NDIM>(NDIM - 1);
    static_assert(slab_inner<NDIM>() == 256, "one interior vertex per thread");
    static_assert(64 % EX == 0, "a wave holds whole rows of the tile");
    // halo index of interior position (0,..,0), the smallest a row may reach
    constexpr int B = [] {
        int b = 0;
        for (int i = 1; i < NDIM; ++i) b += slab_hs<NDIM>(i);
        return b;
    }();
    __shared__ uint32_t s_ring[3 * S];
    __shared__ int32_t s_glin[K];
    const int tid = threadIdx.x;
    for (int i = tid; i < K; i += blockDim.x) s_glin[i] = t.lin[i];

    int rest = blockIdx.x;
    const int zb = rest % a.zblocks;
    rest /= a.zblocks;
    int t0[NDIM];  // first coordinate of the tile along axes 1..n-1
#pragma unroll
    for (int i = NDIM - 1; i >= 1; --i) {
        const int q = rest % a.nt[i];
        rest /= a.nt[i];
        t0[i] = q * slab_e<NDIM>(i);
    }
    const int z0 = zb * a.zc;
    const int z1 = min(z0 + a.zc, g.dims[0]);

    // the halo positions this thread loads: offset inside a plane of the
    // grid, or -1 outside the grid
    int goff[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        int h = tid + 256 * k;
        bool in = h < S;
        int off = 0;
#pragma unroll
        for (int i = NDIM - 1; i >= 1; --i) {
            const int he = slab_e<NDIM>(i) + 2;
            const int c = t0[i] + h % he - 1;
            h /= he;
            in &= (c >= 0) & (c < g.dims[i]);
            off += c * a.st[i];
        }
        goff[k] = in ? off : -1;
    }
    // this thread's interior vertex: its halo index minus B, and its offset
    // inside a plane of the grid
    int center = 0, vin = 0;
    bool mine = true;
    {
        int r = tid;
#pragma unroll
        for (int i = NDIM - 1; i >= 1; --i) {
            const int e = r % slab_e<NDIM>(i);
            r /= slab_e<NDIM>(i);
            const int c = t0[i] + e;
            mine &= c < g.dims[i];
            center += e * slab_hs<NDIM>(i);
            vin += c * a.st[i];
        }
    }
    const int X = g.dims[NDIM - 1];
    const int x = t0[NDIM - 1] + tid % EX;
    const int rin = mine ? (vin - x) / X : 0;  // row of the vertex inside its plane
    const int XW = (X + 63) >> 6;

    uint32_t r[PER];
    auto fetch = [&](int z) {
        const bool zok = z >= 0 && z < g.dims[0];
        const int zoff = zok ? z * a.st[0] : 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const bool ok = zok && goff[k] >= 0;
            const uint32_t u = keys[ok ? zoff + goff[k] : 0];
            r[k] = ok ? u : 0u;
        }
    };
    auto put = [&](int slot) {
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (tid + 256 * k < S) s_ring[slot * S + tid + 256 * k] = r[k];
    };
    fetch(z0 - 1);
    put(0);
    fetch(z0);
    put(1);
    fetch(z0 + 1);
    int sp = 0;  // slot of plane z-1; plane z is in the next slot, z+1 in the one after
    for (int z = z0; z < z1; ++z) {
        const int s1 = sp == 2 ? 0 : sp + 1;
        const int s2 = s1 == 2 ? 0 : s1 + 1;
        __syncthreads();  // slot s2 (plane z-2) is no longer read
        put(s2);
        __syncthreads();
        if (z + 1 < z1) fetch(z + 2);  // in flight during this plane

        const int v = z * a.st[0] + vin;
        bool is_max = false, is_sad = false;
        if (mine) {
            const uint32_t* p0 = s_ring + sp * S + center;
            const uint32_t* p1 = s_ring + s1 * S + center;
            const uint32_t* p2 = s_ring + s2 * S + center;
            const uint32_t uv = p1[B];
            auto key = [&](int j) {
                int d = B;
#pragma unroll
                for (int i = 1; i < NDIM; ++i) d += R.d[j][i] * slab_hs<NDIM>(i);
                const uint32_t* p = R.d[j][0] < 0 ? p0 : R.d[j][0] > 0 ? p2 : p1;
                return p[d];
            };
            // the upper-link mask, and the highest key of the closed
            // neighbourhood (rows outside the grid hold key 0 < uv)
            // 32 rows per word, pushed from the highest row down so that row
            // j ends in bit j % 32 of word j / 32 (two instructions a row)
            constexpr int NW = (K + 31) / 32;
            uint32_t wd[NW];
            uint32_t top = uv;
            static_for<0, K>([&](auto step) {
                constexpr int j = K - 1 - decltype(step)::value;
                constexpr bool wins = (j >= K / 2) != MINMODE;
                const uint32_t u = key(j);
                if constexpr (j == K - 1 || j % 32 == 31)
                    wd[j / 32] = first_above<wins>(u, uv);
                else
                    wd[j / 32] = push_above<wins>(wd[j / 32], u, uv);
                top = max(top, u);
            });
            Mask<NDIM> up = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) up |= Mask<NDIM>(wd[w]) << (32 * w);
            // the steepest target: the last vertex holding `top` in the order
            // in which later vertices win ties (v itself between the halves)
            int best_j = -1;
            auto visit = [&](int j) {
                if (key(j) == top) best_j = j;
            };
            auto self = [&]() {
                if (uv == top) best_j = -1;
            };
            if (!MINMODE) {
#pragma unroll
                for (int j = 0; j < K / 2; ++j) visit(j);
                self();
#pragma unroll
                for (int j = K / 2; j < K; ++j) visit(j);
            } else {
#pragma unroll
                for (int j = K - 1; j >= K / 2; --j) visit(j);
                self();
#pragma unroll
                for (int j = K / 2 - 1; j >= 0; --j) visit(j);
            }
            is_max = up == 0;
            if (!is_max) is_sad = !link_connected<NDIM>(up);
            const int best = best_j < 0 ? v : v + s_glin[best_j];
            lab[v] = is_max ? v : -(best + 1);
            if (ptr) ptr[v] = best;
        }
        const int64_t word = mine ? (int64_t)(z * a.rows_per_plane + rin) * XW + (x >> 6) : -1;
        mask_or(is_max, word, x & 63, mmask);
        mask_or(is_sad, word, x & 63, smask);
        sp = s1;
    }
}

template <int NDIM, bool MINMODE>
static void launch_classify_t(const float* f, const Grid& g, const LinkTable& t, int32_t* lab, int32_t* ptr,
                              const Work& w, hipStream_t s)
{
    const int64_t zwant = (w.words + 255) / 256;
    const int zblocks = (int)(zwant < 4096 ? (zwant > 0 ? zwant : 1) : 4096);
    hipLaunchKernelGGL(k_zero_words, dim3(zblocks), dim3(256), 0, s, w.mmask, w.smask, w.words);
    const int64_t kwant = ((int64_t)g.N + 255) / 256;
    const int kblocks = (int)(kwant < 8192 ? kwant : 8192);
    hipLaunchKernelGGL(k_keys<MINMODE>, dim3(kblocks), dim3(256), 0, s, f, g.N, w.keys, w.ctr);
    if constexpr (NDIM >= 4) {
        SlabArgs a{};
        a.st[NDIM - 1] = 1;
        for (int i = NDIM - 2; i >= 0; --i) a.st[i] = a.st[i + 1] * g.dims[i + 1];
        int64_t tiles = 1;
        for (int i = 1; i < NDIM; ++i) {
            a.nt[i] = (g.dims[i] + slab_e<NDIM>(i) - 1) / slab_e<NDIM>(i);
            tiles *= a.nt[i];
        }
        // about 8192 blocks, each over as many planes as that allows
        const int64_t D0 = g.dims[0];
        const int64_t zc = std::min<int64_t>(D0, std::max<int64_t>(1, (D0 * tiles + 8191) / 8192));
        a.zc = (int)zc;
        a.zblocks = (int)((D0 + zc - 1) / zc);
        a.rows_per_plane = a.st[0] / g.dims[NDIM - 1];
        const int64_t blocks = tiles * a.zblocks;
        hipLaunchKernelGGL((k_classify_slab<NDIM, MINMODE>), dim3((unsigned)blocks), dim3(256), 0, s, w.keys, g, t,
                           a, lab, ptr, w.mmask, w.smask);
    } else {
        const int blocks = (int)((g.N + 255) / 256);
        hipLaunchKernelGGL((k_classify_generic<NDIM, MINMODE>), dim3(blocks), dim3(256), 0, s, w.keys, g, t, lab,
                           ptr, w.mmask, w.smask);
    }
}

hipError_t launch_classify(const float* f, const Grid& g, const LinkTable& t, bool minima, int32_t* lab,
                           int32_t* ptr, const Work& w, const Tuning& tu, hipStream_t s)
{
    if (g.ndim == 2 || g.ndim == 3) return launch_classify_tiled(f, g, minima, lab, ptr, w, tu, s);
#define EG_CASE(N)                                                \
    case N:                                                       \
        if (minima)                                               \
            launch_classify_t<N, true>(f, g, t, lab, ptr, w, s);  \
        else                                                      \
            launch_classify_t<N, false>(f, g, t, lab, ptr, w, s); \
        break;
    switch (g.ndim) {
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
    return hipGetLastError();
}

// ------------------------------------------------------------------ labels

// Stage (b): labels.  After classification every vertex holds a final label
// (its maximum) or a code for a later vertex of its steepest-ascent path: a
// vertex id, or an entry of the exit list (the distinct vertices where paths
// leave a tile, published once per tile).  The pass resolves the short exit
// list first, by pointer jumping, and then every vertex with one look-up;
// vertex-id codes (grids without tiling, or a full exit list) are resolved by
// pointer jumping over the label array itself.
//
// Entries are updated in place while other threads read them.  Every value
// ever stored says something true about the same path, so any value read is
// usable.  A pass follows at most `hops` links per entry; a pass that stops
// short raises its flag and the next pass runs.  After pass p every entry has
// advanced hops^p links or become final, so the launcher's pass count
// (hops^passes >= 2^31) covers any path in a grid of fewer than 2^31 vertices.

__device__ __forceinline__ int next_link(const int32_t* lab, const int32_t* res, int N, int x)
{
    return x >= -N ? lab[-x - 1] : res[-x - 1 - N];
}

__device__ __forceinline__ bool gate(const uint32_t* ctr, int flag_base, int pass)
{
    return pass == 0 ||
           __hip_atomic_load(&ctr[flag_base + pass - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Both exit-list kernels take four consecutive entries per thread (one
// 16-byte access, four independent gathers or chains in flight): the links
// are latency-bound gathers, so more of them per thread hide more latency.
// The list base is 16-byte aligned (the workspace is carved in 256-byte
// steps).
__global__ __launch_bounds__(256) void k_exit_init(const uint32_t* __restrict__ exits, int32_t* __restrict__ res,
                                                   const int32_t* __restrict__ lab, const uint32_t* __restrict__ ctr,
                                                   uint32_t cap)
{
    const uint32_t req = __hip_atomic_load(&ctr[C_NEXIT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t n = req < cap ? req : cap;
    const uint32_t nq = n >> 2;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint4* e4 = reinterpret_cast<const uint4*>(exits);
    int4* r4 = reinterpret_cast<int4*>(res);
    for (uint32_t q = t; q < nq; q += stride) {
        const uint4 e = e4[q];
        r4[q] = make_int4(lab[e.x], lab[e.y], lab[e.z], lab[e.w]);
    }
    if (t < (n & 3u)) res[(nq << 2) + t] = lab[exits[(nq << 2) + t]];
}

__global__ __launch_bounds__(256) void k_exit_jump(int32_t* res, const int32_t* __restrict__ lab, int N,
                                                   uint32_t* __restrict__ ctr, uint32_t cap, int pass, int hops)
{
    if (!gate(ctr, C_JUMP, pass)) return;
    const uint32_t req = __hip_atomic_load(&ctr[C_NEXIT], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t n = req < cap ? req : cap;
    const uint32_t nq = n >> 2;
    const uint32_t stride = gridDim.x * blockDim.x;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    int4* r4 = reinterpret_cast<int4*>(res);
    bool notdone = false;
    for (uint32_t q = t; q < nq; q += stride) {
        const int4 x = r4[q];
        if ((x.x | x.y | x.z | x.w) >= 0) continue;  // all four final
        int y0 = x.x, y1 = x.y, y2 = x.z, y3 = x.w;
        for (int h = 0; (y0 < 0 || y1 < 0 || y2 < 0 || y3 < 0) && h < hops; ++h) {
            if (y0 < 0) y0 = next_link(lab, res, N, y0);
            if (y1 < 0) y1 = next_link(lab, res, N, y1);
            if (y2 < 0) y2 = next_link(lab, res, N, y2);
            if (y3 < 0) y3 = next_link(lab, res, N, y3);
        }
        r4[q] = make_int4(y0, y1, y2, y3);
        notdone |= (y0 < 0) | (y1 < 0) | (y2 < 0) | (y3 < 0);
    }
    if (t < (n & 3u)) {
        const uint32_t i = (nq << 2) + t;
        int x = res[i];
        for (int h = 0; x < 0 && h < hops; ++h) x = next_link(lab, res, N, x);
        res[i] = x;
        notdone |= x < 0;
    }
    if (__ballot(notdone) != 0 && __lane_id() == 0) atomicOr(&ctr[C_JUMP + pass], 1u);
}

// Per-vertex pass: four consecutive vertices per thread (one 16-byte load,
// four independent chains).
__global__ __launch_bounds__(256) void k_final(int32_t* lab, const int32_t* __restrict__ res, int32_t N,
                                               uint32_t* __restrict__ ctr, int pass, int hops)
{
    if (!gate(ctr, C_FINAL, pass)) return;
    bool notdone = false;
    const int nq = N >> 2;
    const int stride = gridDim.x * blockDim.x;
    int4* lab4 = reinterpret_cast<int4*>(lab);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
        const int4 x = lab4[q];
        if ((x.x | x.y | x.z | x.w) >= 0) continue;  // all four final
        int y0 = x.x < 0 ? next_link(lab, res, N, x.x) : x.x;
        int y1 = x.y < 0 ? next_link(lab, res, N, x.y) : x.y;
        int y2 = x.z < 0 ? next_link(lab, res, N, x.z) : x.z;
        int y3 = x.w < 0 ? next_link(lab, res, N, x.w) : x.w;
        int h = 1;
        while ((y0 < 0 || y1 < 0 || y2 < 0 || y3 < 0) && h < hops) {
            if (y0 < 0) y0 = next_link(lab, res, N, y0);
            if (y1 < 0) y1 = next_link(lab, res, N, y1);
            if (y2 < 0) y2 = next_link(lab, res, N, y2);
            if (y3 < 0) y3 = next_link(lab, res, N, y3);
            ++h;
        }
        lab4[q] = make_int4(y0, y1, y2, y3);
        notdone |= (y0 < 0) | (y1 < 0) | (y2 < 0) | (y3 < 0);
    }
    // the last N % 4 vertices
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (N & 3)) {
        const int v = (nq << 2) + t;
        int y = lab[v];
        for (int h = 0; y < 0 && h < hops; ++h) y = next_link(lab, res, N, y);
        lab[v] = y;
        notdone |= y < 0;
    }
    if (__ballot(notdone) != 0 && __lane_id() == 0) atomicOr(&ctr[C_FINAL + pass], 1u);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctr[C_PASSES], 1u);
}

hipError_t launch_labels(const Grid& g, int32_t* lab, const Work& w, const Tuning& tu, hipStream_t s)
{
    const int32_t N = g.N;
    if (reinterpret_cast<uintptr_t>(lab) & 15u) return hipErrorInvalidValue;
    const uint32_t cap = (uint32_t)w.cap_exit;
    if ((reinterpret_cast<uintptr_t>(w.exits) | reinterpret_cast<uintptr_t>(w.exres)) & 15u)
        return hipErrorInvalidValue;
    const int64_t ewant = (w.cap_exit / 4 + 255) / 256;
    const int eblocks = (int)(ewant < 2048 ? (ewant > 0 ? ewant : 1) : 2048);
    // a later pass runs only when the pass before it stopped short, which
    // the tiled grids' passes practically never do: most of these launches
    // return at once, and small grids keep them cheap (a pass that does run
    // then takes longer)
    const int eblocks_late = eblocks < 128 ? eblocks : 128;
    // the first pass reads entries that other threads of the same pass have
    // already advanced, which shortens long chains: it needs every entry
    // initialised first
    hipLaunchKernelGGL(k_exit_init, dim3(eblocks), dim3(256), 0, s, w.exits, w.exres, lab, w.ctr, cap);
    for (int p = 0; p < tu.passes; ++p)
        hipLaunchKernelGGL(k_exit_jump, dim3(p == 0 ? eblocks : eblocks_late), dim3(256), 0, s, w.exres, lab, N,
                           w.ctr, cap, p, tu.hops);
    const int64_t want = ((int64_t)N / 4 + 255) / 256;
    const int blocks = (int)(want < 2048 ? (want > 0 ? want : 1) : 2048);
    const bool tiled = g.ndim == 2 || g.ndim == 3;
    int p = 0;
    if (tiled) {
        // pass 0 in tile order (the classification wrote exit-list codes)
        const hipError_t e = launch_final_tiled(g, lab, w, tu, C_FINAL, s);
        if (e != hipSuccess) return e;
        p = 1;
    }
    // untiled grids resolve their vertex codes in these passes: full grids
    const int blocks_late = tiled && blocks > 128 ? 128 : blocks;
    for (; p < tu.passes; ++p)
        hipLaunchKernelGGL(k_final, dim3(p == 0 ? blocks : blocks_late), dim3(256), 0, s, lab, w.exres, N, w.ctr, p,
                           tu.hops);
    return hipGetLastError();
}

}  // namespace eg
