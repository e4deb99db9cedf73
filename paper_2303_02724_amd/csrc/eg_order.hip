// eg_order.hip -- order surrogates of fields of other sample types.
//
// Only the simulated-perturbation order of the samples enters the graph
// (Sec. 3.3), so a field of any of the input types of Sec. 4 is replaced by a
// float32 field with the same order and the float32 path runs unchanged.
//
//   8- and 16-bit integers   converted to float32: exact, ties stay ties.
//   32/64-bit, float64       ranked: each sample gets an order-preserving
//                            unsigned key (sign flip for signed integers; for
//                            floats the usual sign-magnitude flip after -0 is
//                            folded into +0), the keys are sorted stably by a
//                            least-significant-digit radix sort that starts
//                            from index order, and the vertex at sorted
//                            position p receives the p-th float of a strictly
//                            increasing sequence of normal floats.  Equal
//                            values keep index order, so the ranks realise the
//                            tie-break as well.
//
// Radix sort.  8-bit digits of (key - min key); passes above the highest bit
// in which the keys differ are skipped on the device (the range is reduced
// first, the host never waits).  Each pass: per-block digit histograms, a
// scan of each digit's row over the blocks, and a stable scatter in which a
// block ranks a tile of 2048 keys by wave ballots (each wave its own quarter),
// sorts the tile by digit in LDS and writes each digit's run contiguously.
// The last pass that runs writes no keys: each element's final position is
// its rank, stored straight into the surrogate (one 4-byte store per vertex,
// at no particular place).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "eg.h"

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // keys per scatter round
constexpr int kMaxBlocks = 1024;          // histogram columns: every block resident at once
constexpr int kDigits = 256;
static_assert(kThreads == kDigits, "one thread per digit");

struct Ctl {
    uint64_t kmin;
    uint32_t nbits;  // bits of (max key - min key)
    uint32_t nnan;
};

// ---------------------------------------------------------------- keys

template <typename T>
struct Key;
template <>
struct Key<double> {
    using K = uint64_t;
    static __device__ bool nan(double x) { return x != x; }
    static __device__ K of(double x)
    {
        const uint64_t b = (uint64_t)__double_as_longlong(x + 0.0);  // -0 + 0 = +0
        return (b >> 63) ? ~b : (b | (uint64_t(1) << 63));
    }
};
template <>
struct Key<int64_t> {
    using K = uint64_t;
    static __device__ bool nan(int64_t) { return false; }
    static __device__ K of(int64_t x) { return (uint64_t)x ^ (uint64_t(1) << 63); }
};
template <>
struct Key<uint64_t> {
    using K = uint64_t;
    static __device__ bool nan(uint64_t) { return false; }
    static __device__ K of(uint64_t x) { return x; }
};
template <>
struct Key<int32_t> {
    using K = uint32_t;
    static __device__ bool nan(int32_t) { return false; }
    static __device__ K of(int32_t x) { return (uint32_t)x ^ 0x80000000u; }
};
template <>
struct Key<uint32_t> {
    using K = uint32_t;
    static __device__ bool nan(uint32_t) { return false; }
    static __device__ K of(uint32_t x) { return x; }
};

// Contiguous chunk of block b: [lo, hi).
__device__ __forceinline__ void chunk(uint32_t n, uint32_t per, uint32_t b, uint32_t& lo, uint32_t& hi)
{
    const uint64_t l = uint64_t(b) * per;
    lo = (uint32_t)(l < n ? l : n);
    const uint64_t h = uint64_t(lo) + per;
    hi = (uint32_t)(h < n ? h : n);
}

template <typename K>
__device__ __forceinline__ K wave_min(K x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const K y = __shfl_xor(x, o);
        x = y < x ? y : x;
    }
    return x;
}
template <typename K>
__device__ __forceinline__ K wave_max(K x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const K y = __shfl_xor(x, o);
        x = y > x ? y : x;
    }
    return x;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Keys of block b's chunk, and the chunk's min / max key and NaN count.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_keys(const T* __restrict__ f, uint32_t n, uint32_t per,
                                                   typename Key<T>::K* __restrict__ keys, uint64_t* __restrict__ pmin,
                                                   uint64_t* __restrict__ pmax, uint32_t* __restrict__ pnan)
{
    using K = typename Key<T>::K;
    __shared__ uint64_t smin[kThreads / 64], smax[kThreads / 64];
    __shared__ uint32_t snan[kThreads / 64];
    uint32_t lo, hi;
    chunk(n, per, blockIdx.x, lo, hi);
    K mn = ~K(0), mx = 0;
    uint32_t nn = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kThreads) {
        const T x = f[i];
        K k;
        if (Key<T>::nan(x)) {
            ++nn;
            k = ~K(0);  // kept out of the range; the surrogate is NaN anyway
        } else {
            k = Key<T>::of(x);
            mn = k < mn ? k : mn;
            mx = k > mx ? k : mx;
        }
        keys[i] = k;
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    nn = wave_sum(nn);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin[w] = mn;
        smax[w] = mx;
        snan[w] = nn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = smin[0], b = smax[0];
        uint32_t c = snan[0];
        for (int k = 1; k < kThreads / 64; ++k) {
            a = smin[k] < a ? smin[k] : a;
            b = smax[k] > b ? smax[k] : b;
            c += snan[k];
        }
        pmin[blockIdx.x] = a;
        pmax[blockIdx.x] = b;
        pnan[blockIdx.x] = c;
    }
}

// Min key, bit width of the key range and NaN count over the G partials.
__global__ __launch_bounds__(kThreads) void k_range(const uint64_t* __restrict__ pmin,
                                                    const uint64_t* __restrict__ pmax,
                                                    const uint32_t* __restrict__ pnan, uint32_t G,
                                                    Ctl* __restrict__ ctl)
{
    __shared__ uint64_t smin[kThreads / 64], smax[kThreads / 64];
    __shared__ uint32_t snan[kThreads / 64];
    uint64_t mn = ~uint64_t(0), mx = 0;
    uint32_t nn = 0;
    for (uint32_t b = threadIdx.x; b < G; b += kThreads) {
        mn = pmin[b] < mn ? pmin[b] : mn;
        mx = pmax[b] > mx ? pmax[b] : mx;
        nn += pnan[b];
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    nn = wave_sum(nn);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin[w] = mn;
        smax[w] = mx;
        snan[w] = nn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mn = smin[0];
        mx = smax[0];
        nn = snan[0];
        for (int k = 1; k < kThreads / 64; ++k) {
            mn = smin[k] < mn ? smin[k] : mn;
            mx = smax[k] > mx ? smax[k] : mx;
            nn += snan[k];
        }
        // every sample NaN: an empty range
        const uint64_t span = mx >= mn ? mx - mn : 0;
        ctl->kmin = mx >= mn ? mn : 0;
        ctl->nbits = span == 0 ? 0u : (uint32_t)(64 - __clzll((long long)span));
        ctl->nnan = nn;
    }
}

// The p-th float of a strictly increasing sequence of normal floats, p < 2^31:
// negative normals for p < 2^30, positive ones above.
__device__ __forceinline__ float rank_float(uint32_t p)
{
    const int64_t t = int64_t(p) - (int64_t(1) << 30);
    const uint32_t bits = t >= 0 ? 0x00800000u + (uint32_t)t : 0x80800000u + (uint32_t)(-t - 1);
    return __uint_as_float(bits);
}

template <typename K>
__device__ __forceinline__ uint32_t digit(K k, K kmin, int shift)
{
    return (uint32_t)((k - kmin) >> shift) & (kDigits - 1);
}

// Digit histogram of block b's chunk: hist[d * G + b].
template <typename K>
__global__ __launch_bounds__(kThreads) void k_hist(const K* __restrict__ keys, uint32_t n, uint32_t per, int shift,
                                                   const Ctl* __restrict__ ctl, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[kThreads / 64][kDigits];
    if ((uint32_t)shift >= ctl->nbits) return;
    const K kmin = (K)ctl->kmin;
    const int tid = threadIdx.x, w = tid >> 6;
    for (int k = 0; k < kThreads / 64; ++k) h[k][tid] = 0;
    __syncthreads();
    uint32_t lo, hi;
    chunk(n, per, blockIdx.x, lo, hi);
    for (uint32_t i = lo + tid; i < hi; i += kThreads) atomicAdd(&h[w][digit(keys[i], kmin, shift)], 1u);
    __syncthreads();
    hist[tid * gridDim.x + blockIdx.x] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// Row d (one block per digit): exclusive scan of hist[d * G .. d * G + G) in
// place and the row total into rows[d].  G <= 2 * 1024.
__global__ __launch_bounds__(1024) void k_scan_row(uint32_t* __restrict__ hist, uint32_t G, int shift,
                                                   const Ctl* __restrict__ ctl, uint32_t* __restrict__ rows)
{
    __shared__ uint32_t ws[16];
    if ((uint32_t)shift >= ctl->nbits) return;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    uint32_t* row = hist + (size_t)blockIdx.x * G;
    const uint32_t i0 = 2 * tid, i1 = 2 * tid + 1;
    const uint32_t a = i0 < G ? row[i0] : 0u, b = i1 < G ? row[i1] : 0u;
    const uint32_t s = a + b;
    const uint32_t inc = wave_incl_scan(s);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    if (w == 0) {
        uint32_t y = lane < 16 ? ws[lane] : 0u;
        y = wave_incl_scan(y);
        if (lane < 16) ws[lane] = y;
    }
    __syncthreads();
    const uint32_t ex = (w > 0 ? ws[w - 1] : 0u) + inc - s;
    if (i0 < G) row[i0] = ex;
    if (i1 < G) row[i1] = ex + a;
    if (tid == 0) rows[blockIdx.x] = ws[15];
}

// Stable scatter of block b's chunk.  first: the input indices are the
// positions themselves (the pass that reads the keys in index order).
// A tile of 2048 keys is split into four contiguous quarters, one per wave;
// a wave ranks its keys by digit with ballots against its own running digit
// counts (wave-private, so no barrier is needed), then one block-wide step
// turns the four waves' counts into tile offsets.  Tile order is index order,
// so the ranks are stable.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ iin,
                                                      K* __restrict__ kout, uint32_t* __restrict__ iout, uint32_t n,
                                                      uint32_t per, int shift, const Ctl* __restrict__ ctl,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ rows, bool first,
                                                      float* __restrict__ out)
{
    constexpr int W = kThreads / 64;
    __shared__ uint32_t run[kDigits];      // next output position of each digit
    __shared__ uint32_t toff[kDigits];     // tile offset of each digit
    __shared__ uint32_t wcnt[W][kDigits];  // each wave's digit counts in the tile
    __shared__ uint32_t wpre[W][kDigits];  // digit counts of the waves before it
    __shared__ uint32_t wsum[W];
    __shared__ K skey[kTile];
    __shared__ uint32_t sidx[kTile];
    if ((uint32_t)shift >= ctl->nbits) return;
    uint32_t lo, hi;
    chunk(n, per, blockIdx.x, lo, hi);
    if (lo >= hi) return;
    const K kmin = (K)ctl->kmin;
    const bool last = (uint32_t)shift + 8u >= ctl->nbits;
    const bool nan = ctl->nnan != 0;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;

    // digit bases: exclusive scan of the row totals, plus this block's column
    {
        const uint32_t x = rows[tid];
        const uint32_t inc = wave_incl_scan(x);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
        for (int k = 0; k < w; ++k) pre += wsum[k];
        run[tid] = pre + inc - x + hist[tid * gridDim.x + blockIdx.x];
    }
    for (int k = 0; k < W; ++k) wcnt[k][tid] = 0;
    __syncthreads();
    const uint64_t lt = (uint64_t(1) << lane) - 1;

    for (uint32_t base = lo; base < hi; base += kTile) {
        K key[kItems];
        uint32_t id[kItems], dg[kItems], rk[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t i = base + (w * kItems + j) * 64 + lane;
            const bool valid = i < hi;
            key[j] = valid ? kin[i] : K(0);
            id[j] = valid ? (first ? i : iin[i]) : 0u;
            dg[j] = valid ? digit(key[j], kmin, shift) : (uint32_t)kDigits;
        }
        // ranks within the wave: lanes read the running count, then the first
        // lane of each digit group adds the group (in program order)
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const bool valid = dg[j] < (uint32_t)kDigits;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const bool on = (dg[j] >> bit) & 1u;
                const uint64_t bm = __ballot(on);
                peers &= on ? bm : ~bm;
            }
            const uint32_t r = (uint32_t)__popcll(peers & lt);
            const uint32_t before = valid ? wcnt[w][dg[j]] : 0u;
            rk[j] = before + r;
            if (valid && r == 0) wcnt[w][dg[j]] = before + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        // per digit (thread = digit): the waves' prefixes and the tile offsets
        uint32_t tcnt = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            wpre[k][tid] = tcnt;
            tcnt += wcnt[k][tid];
            wcnt[k][tid] = 0;
        }
        {
            const uint32_t inc = wave_incl_scan(tcnt);
            if (lane == 63) wsum[w] = inc;
            __syncthreads();
            uint32_t pre = 0;
            for (int k = 0; k < w; ++k) pre += wsum[k];
            toff[tid] = pre + inc - tcnt;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            if (dg[j] < (uint32_t)kDigits) {
                const uint32_t p = toff[dg[j]] + wpre[w][dg[j]] + rk[j];
                skey[p] = key[j];
                sidx[p] = id[j];
            }
        }
        __syncthreads();
        const uint32_t tn = hi - base < (uint32_t)kTile ? hi - base : (uint32_t)kTile;
        for (uint32_t p = tid; p < tn; p += kThreads) {
            const K k = skey[p];
            const uint32_t d = digit(k, kmin, shift);
            const uint32_t g = run[d] + (p - toff[d]);
            if (last) {
                out[sidx[p]] = nan ? __uint_as_float(0x7FC00000u) : rank_float(g);
            } else {
                kout[g] = k;
                iout[g] = sidx[p];
            }
        }
        __syncthreads();
        run[tid] += tcnt;
    }
}

// Keys that are all equal (no pass runs): index order is the sorted order.
// A NaN anywhere makes every entry NaN.
__global__ __launch_bounds__(kThreads) void k_fill(uint32_t n, const Ctl* __restrict__ ctl, float* __restrict__ out)
{
    if (ctl->nbits != 0) return;
    const bool nan = ctl->nnan != 0;
    for (uint32_t p = blockIdx.x * kThreads + threadIdx.x; p < n; p += gridDim.x * kThreads)
        out[p] = nan ? __uint_as_float(0x7FC00000u) : rank_float(p);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_convert(const T* __restrict__ f, uint32_t n, float* __restrict__ out)
{
    for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) out[i] = (float)f[i];
}

// ---------------------------------------------------------------- host

struct Layout {
    size_t keysA, keysB, idxA, idxB, hist, rows, pmin, pmax, pnan, ctl, total;
    uint32_t G, per;
};

size_t key_bytes(int dtype)
{
    switch (dtype) {
        case EG_I32:
        case EG_U32: return 4;
        case EG_I64:
        case EG_U64:
        case EG_F64: return 8;
        default: return 0;
    }
}

size_t sample_bytes(int dtype)
{
    switch (dtype) {
        case EG_I8:
        case EG_U8: return 1;
        case EG_I16:
        case EG_U16: return 2;
        case EG_F32:
        case EG_I32:
        case EG_U32: return 4;
        default: return 8;
    }
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout(int dtype, int64_t n)
{
    Layout L{};
    const size_t kb = key_bytes(dtype);
    int64_t g = (n + 16383) / 16384;
    g = g < 1 ? 1 : (g > kMaxBlocks ? kMaxBlocks : g);
    const int64_t per0 = (n + g - 1) / g;
    const int64_t per = (per0 + kTile - 1) / kTile * kTile;
    L.G = (uint32_t)((n + per - 1) / per);
    L.per = (uint32_t)per;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t o = at;
        at += up256(bytes);
        return o;
    };
    L.keysA = take(kb * (size_t)n);
    L.keysB = take(kb * (size_t)n);
    L.idxA = take(4 * (size_t)n);
    L.idxB = take(4 * (size_t)n);
    L.hist = take(4 * (size_t)kDigits * kMaxBlocks);
    L.rows = take(4 * (size_t)kDigits);
    L.pmin = take(8 * (size_t)kMaxBlocks);
    L.pmax = take(8 * (size_t)kMaxBlocks);
    L.pnan = take(4 * (size_t)kMaxBlocks);
    L.ctl = take(sizeof(Ctl));
    L.total = at;
    return L;
}

template <typename T>
hipError_t rank_field(const T* f, uint32_t n, float* out, char* ws, const Layout& L, hipStream_t s)
{
    using K = typename Key<T>::K;
    K* kA = reinterpret_cast<K*>(ws + L.keysA);
    K* kB = reinterpret_cast<K*>(ws + L.keysB);
    uint32_t* iA = reinterpret_cast<uint32_t*>(ws + L.idxA);
    uint32_t* iB = reinterpret_cast<uint32_t*>(ws + L.idxB);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + L.hist);
    uint32_t* rows = reinterpret_cast<uint32_t*>(ws + L.rows);
    uint64_t* pmin = reinterpret_cast<uint64_t*>(ws + L.pmin);
    uint64_t* pmax = reinterpret_cast<uint64_t*>(ws + L.pmax);
    uint32_t* pnan = reinterpret_cast<uint32_t*>(ws + L.pnan);
    Ctl* ctl = reinterpret_cast<Ctl*>(ws + L.ctl);
    const dim3 G(L.G), B(kThreads);
    hipLaunchKernelGGL(k_keys<T>, G, B, 0, s, f, n, L.per, kA, pmin, pmax, pnan);
    hipLaunchKernelGGL(k_range, dim3(1), B, 0, s, pmin, pmax, pnan, L.G, ctl);
    const int passes = (int)(8 * sizeof(K) / 8);
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        const K* ki = (p & 1) ? kB : kA;
        K* ko = (p & 1) ? kA : kB;
        const uint32_t* ii = (p & 1) ? iB : iA;
        uint32_t* io = (p & 1) ? iA : iB;
        hipLaunchKernelGGL(k_hist<K>, G, B, 0, s, ki, n, L.per, shift, ctl, hist);
        hipLaunchKernelGGL(k_scan_row, dim3(kDigits), dim3(1024), 0, s, hist, L.G, shift, ctl, rows);
        hipLaunchKernelGGL(k_scatter<K>, G, B, 0, s, ki, ii, ko, io, n, L.per, shift, ctl, hist, rows, p == 0,
                           out);
    }
    const uint32_t eb = (uint32_t)std::min<uint64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_fill, dim3(eb), B, 0, s, n, ctl, out);
    return hipGetLastError();
}

template <typename T>
hipError_t convert_field(const T* f, uint32_t n, float* out, hipStream_t s)
{
    const uint32_t eb = (uint32_t)std::min<uint64_t>((n + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(k_convert<T>, dim3(eb), dim3(kThreads), 0, s, f, n, out);
    return hipGetLastError();
}

}  // namespace

extern "C" size_t eg_order_workspace_bytes(int dtype, int64_t n)
{
    if (dtype < EG_F32 || dtype > EG_U64 || n < 1 || n >= (int64_t(1) << 31)) return 0;
    if (key_bytes(dtype) == 0) return 0;
    return layout(dtype, n).total;
}

extern "C" eg_status eg_order_field(int dtype, const void* field, int64_t n, float* out, void* workspace,
                                    size_t ws_bytes, void* stream)
{
    if (dtype < EG_F32 || dtype > EG_U64 || !field || !out || n < 1) return EG_ERR_ARG;
    if (n >= (int64_t(1) << 31)) return EG_ERR_TOO_LARGE;
    const uintptr_t fa = (uintptr_t)field, oa = (uintptr_t)out;
    const uintptr_t fe = fa + (uintptr_t)(sample_bytes(dtype) * (size_t)n), oe = oa + 4 * (size_t)n;
    if (fa < oe && oa < fe) return EG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t nn = (uint32_t)n;
    hipError_t e = hipSuccess;
    if (key_bytes(dtype) == 0) {
        switch (dtype) {
            case EG_F32: e = convert_field((const float*)field, nn, out, s); break;
            case EG_I8: e = convert_field((const int8_t*)field, nn, out, s); break;
            case EG_U8: e = convert_field((const uint8_t*)field, nn, out, s); break;
            case EG_I16: e = convert_field((const int16_t*)field, nn, out, s); break;
            default: e = convert_field((const uint16_t*)field, nn, out, s); break;
        }
        return e == hipSuccess ? EG_OK : EG_ERR_HIP;
    }
    const Layout L = layout(dtype, n);
    if (!workspace || ((uintptr_t)workspace & 255) || ws_bytes < L.total) return EG_ERR_WORKSPACE;
    char* ws = (char*)workspace;
    switch (dtype) {
        case EG_I32: e = rank_field((const int32_t*)field, nn, out, ws, L, s); break;
        case EG_U32: e = rank_field((const uint32_t*)field, nn, out, ws, L, s); break;
        case EG_I64: e = rank_field((const int64_t*)field, nn, out, ws, L, s); break;
        case EG_U64: e = rank_field((const uint64_t*)field, nn, out, ws, L, s); break;
        default: e = rank_field((const double*)field, nn, out, ws, L, s); break;
    }
    return e == hipSuccess ? EG_OK : EG_ERR_HIP;
}
