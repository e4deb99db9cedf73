// eg_sort.hip -- device LSD radix sort of 64-bit keys and the CSR build.
//
// Stage (d) of the method ends with a de-duplicated set of (saddle, maximum)
// arcs (arcs form a set, Sec. 2; Alg. 2 returns a set of paths).  The keys
// (saddle << (b+1)) | (marker << b) | low are sorted here; equal arcs become
// neighbours and collapse, and the per-saddle marker (low = component count)
// sorts after its saddle's arcs, closing the CSR row.
//
// Every kernel reads its element count from device memory, so the host never
// waits for the counts: the grid is fixed and each block takes a contiguous
// chunk of whole 256-key tiles.  The scatter is stable (ranks from wave
// ballots, waves in order), as LSD radix sort requires.
#include "eg_internal.h"

namespace eg {

// Blocks take contiguous runs of whole 256-key tiles; only the first
// `active` blocks get work, so small inputs touch few histogram columns.
__device__ __forceinline__ uint32_t chunk_range(uint32_t n, uint32_t nblocks, uint32_t blk, uint32_t& lo,
                                                uint32_t& hi)
{
    const uint32_t tiles = (n + 255u) / 256u;
    // at least kMinTilesPerBlock tiles per block: small inputs use few blocks
    // and a short histogram
    uint32_t per = tiles == 0 ? 1u : (tiles + nblocks - 1u) / nblocks;
    per = per < kMinTilesPerBlock ? kMinTilesPerBlock : per;
    const uint32_t active = (tiles + per - 1u) / per;
    const uint64_t l = uint64_t(blk) * per * 256u;
    lo = (uint32_t)(l < n ? l : n);
    const uint64_t h = uint64_t(lo) + uint64_t(per) * 256u;
    hi = (uint32_t)(h < n ? h : n);
    return active;
}

__device__ __forceinline__ uint32_t load_count(const uint32_t* count, uint32_t cap)
{
    const uint32_t n = __hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return n < cap ? n : cap;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

// The maxima become the first keys; the saddle entries are appended after
// them (the key counter starts at the number of maxima).
__global__ __launch_bounds__(256) void k_load_maxima(const uint32_t* __restrict__ umax, uint32_t* __restrict__ ctr,
                                                     uint32_t cap_max, uint64_t* __restrict__ keys, int b)
{
    const uint32_t n = load_count(&ctr[C_NMAX], cap_max);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        keys[i] = max_key(umax[i], b);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctr[C_NKEYS], n);
}

hipError_t launch_load_maxima(const Work& w, int64_t cap_max, int bits, hipStream_t s)
{
    int64_t want = (cap_max + 255) / 256;
    const int blocks = (int)(want < 1024 ? (want > 0 ? want : 1) : 1024);
    hipLaunchKernelGGL(k_load_maxima, dim3(blocks), dim3(256), 0, s, w.umax, w.ctr, (uint32_t)cap_max, w.keysA,
                       bits);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t* __restrict__ keys, const uint32_t* count,
                                                    uint32_t cap, int shift, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint32_t n = load_count(count, cap);
    uint32_t lo, hi;
    const uint32_t active = chunk_range(n, gridDim.x, blockIdx.x, lo, hi);
    if (blockIdx.x >= active) return;
    for (uint32_t i = lo + tid; i < hi; i += 256) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[tid * active + blockIdx.x] = h[tid];
}

// Exclusive scan, in place, of the 256 x active histogram (digit-major), by
// one block of 1024 threads; chunks of 4096 pass through LDS so that global
// accesses stay coalesced.
__global__ __launch_bounds__(1024) void k_scan_hist(uint32_t* __restrict__ a, const uint32_t* count, uint32_t cap,
                                                    uint32_t nblocks)
{
    __shared__ uint32_t buf[4096];
    __shared__ uint32_t wsum[16];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint32_t n = load_count(count, cap);
    uint32_t lo, hi;
    const uint32_t active = chunk_range(n, nblocks, 0, lo, hi);
    const uint32_t total = 256u * active;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < total; base += 4096) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = base + k * 1024 + tid;
            buf[k * 1024 + tid] = i < total ? a[i] : 0u;
        }
        __syncthreads();
        const uint32_t x0 = buf[4 * tid], x1 = buf[4 * tid + 1], x2 = buf[4 * tid + 2], x3 = buf[4 * tid + 3];
        const uint32_t sum = x0 + x1 + x2 + x3;
        const uint32_t inc = wave_incl_scan(sum);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        if (w == 0) {
            uint32_t y = lane < 16 ? wsum[lane] : 0u;
            y = wave_incl_scan(y);
            if (lane < 16) wsum[lane] = y;
        }
        __syncthreads();
        const uint32_t ex = carry + (w > 0 ? wsum[w - 1] : 0u) + inc - sum;
        buf[4 * tid] = ex;
        buf[4 * tid + 1] = ex + x0;
        buf[4 * tid + 2] = ex + x0 + x1;
        buf[4 * tid + 3] = ex + x0 + x1 + x2;
        carry += wsum[15];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = base + k * 1024 + tid;
            if (i < total) a[i] = buf[k * 1024 + tid];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                       const uint32_t* count, uint32_t cap, int shift,
                                                       const uint32_t* __restrict__ hist)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const uint32_t n = load_count(count, cap);
    uint32_t lo, hi;
    const uint32_t active = chunk_range(n, gridDim.x, blockIdx.x, lo, hi);
    if (blockIdx.x >= active) return;
    run[tid] = hist[tid * active + blockIdx.x];
    const uint64_t lt = (1ull << lane) - 1ull;
    for (uint32_t base = lo; base < hi; base += 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) wcnt[k][tid] = 0;
        __syncthreads();
        const uint32_t i = base + tid;
        const bool valid = i < hi;
        const uint64_t key = valid ? in[i] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bm = __ballot(on);
            peers &= on ? bm : ~bm;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pre = run[d];
            for (int k = 0; k < w; ++k) pre += wcnt[k][d];
            out[pre + rank] = key;
        }
        __syncthreads();
        run[tid] += wcnt[0][tid] + wcnt[1][tid] + wcnt[2][tid] + wcnt[3][tid];
        __syncthreads();
    }
}

hipError_t launch_sort(uint64_t* a, uint64_t* b, const uint32_t* count, int64_t cap, int nbits, uint32_t* hist,
                       uint64_t** sorted, hipStream_t s)
{
    const int passes = (nbits + kRadixBits - 1) / kRadixBits;
    uint64_t* src = a;
    uint64_t* dst = b;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        hipLaunchKernelGGL(k_radix_hist, dim3(kSortBlocks), dim3(kSortThreads), 0, s, src, count, (uint32_t)cap,
                           shift, hist);
        hipLaunchKernelGGL(k_scan_hist, dim3(1), dim3(1024), 0, s, hist, count, (uint32_t)cap,
                           (uint32_t)kSortBlocks);
        hipLaunchKernelGGL(k_radix_scatter, dim3(kSortBlocks), dim3(kSortThreads), 0, s, src, dst, count,
                           (uint32_t)cap, shift, hist);
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    if (sorted) *sorted = src;
    return hipGetLastError();
}

// ------------------------------------------------------------------ CSR

struct KeyFlags {
    bool maximum;  // a maximum entry (they sort first, so their rank is their index)
    bool arc;      // first copy of a (saddle, maximum) key
    bool marker;   // end-of-saddle marker
};

__device__ __forceinline__ KeyFlags key_flags(const uint64_t* keys, uint32_t i, uint32_t n, int b)
{
    KeyFlags r{false, false, false};
    if (i < n) {
        const uint64_t k = keys[i];
        r.maximum = !((k >> (2 * b + 1)) & 1ull);
        r.marker = !r.maximum && ((k >> b) & 1ull);
        r.arc = !r.maximum && !r.marker && (i == 0 || keys[i - 1] != k);
    }
    return r;
}

// Block-wide exclusive rank of a flag over 256 threads; returns the rank and
// writes the block total.  Uses `tmp[4]` of LDS.
__device__ __forceinline__ uint32_t block_rank(bool flag, uint32_t* tmp, uint32_t& total)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t m = __ballot(flag);
    if (lane == 0) tmp[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t pre = 0;
    for (int k = 0; k < w; ++k) pre += tmp[k];
    total = tmp[0] + tmp[1] + tmp[2] + tmp[3];
    __syncthreads();
    return pre + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

__global__ __launch_bounds__(256) void k_csr_count(const uint64_t* __restrict__ keys, const uint32_t* count,
                                                   uint32_t cap, int b, uint32_t* __restrict__ bsum)
{
    __shared__ uint32_t tmp[8];
    const uint32_t n = load_count(count, cap);
    uint32_t lo, hi;
    chunk_range(n, gridDim.x, blockIdx.x, lo, hi);
    uint32_t na = 0, ns = 0;
    for (uint32_t base = lo; base < hi; base += 256) {
        const KeyFlags fl = key_flags(keys, base + threadIdx.x, hi, b);
        na += fl.arc;
        ns += fl.marker;
    }
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint32_t ra = wave_incl_scan(na), rs = wave_incl_scan(ns);
    if (lane == 63) {
        tmp[w] = ra;
        tmp[4 + w] = rs;
    }
    __syncthreads();
    if (tid == 0) {
        bsum[blockIdx.x] = tmp[0] + tmp[1] + tmp[2] + tmp[3];
        bsum[gridDim.x + blockIdx.x] = tmp[4] + tmp[5] + tmp[6] + tmp[7];
    }
}

// Exclusive scan of the two block-sum rows (G <= 256 entries each) and the
// totals into the counters.
__global__ __launch_bounds__(256) void k_csr_scan(uint32_t* __restrict__ bsum, int G, uint32_t* __restrict__ ctr)
{
    __shared__ uint32_t tmp[8];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int row = 0; row < 2; ++row) {
        const uint32_t x = tid < G ? bsum[row * G + tid] : 0u;
        const uint32_t inc = wave_incl_scan(x);
        if (lane == 63) tmp[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
        for (int k = 0; k < w; ++k) pre += tmp[k];
        if (tid < G) bsum[row * G + tid] = pre + inc - x;
        if (tid == 0) ctr[row == 0 ? C_NARC : C_NSADF] = tmp[0] + tmp[1] + tmp[2] + tmp[3];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_csr_write(const uint64_t* __restrict__ keys, const uint32_t* count,
                                                   uint32_t cap, int b, const uint32_t* __restrict__ bsum,
                                                   int32_t* __restrict__ saddles, int32_t* __restrict__ beta,
                                                   int32_t* __restrict__ offsets, uint32_t cap_sad,
                                                   int32_t* __restrict__ arc_maxima, uint32_t cap_arc,
                                                   int32_t* __restrict__ maxima, uint32_t cap_max)
{
    __shared__ uint32_t tmp[4];
    const uint32_t n = load_count(count, cap);
    uint32_t lo, hi;
    chunk_range(n, gridDim.x, blockIdx.x, lo, hi);
    uint32_t abase = bsum[blockIdx.x], sbase = bsum[gridDim.x + blockIdx.x];
    if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
    const uint64_t lowmask = (1ull << b) - 1ull;
    for (uint32_t base = lo; base < hi; base += 256) {
        const uint32_t i = base + threadIdx.x;
        const KeyFlags fl = key_flags(keys, i, hi, b);
        uint32_t ta, ts;
        const uint32_t ra = block_rank(fl.arc, tmp, ta);
        const uint32_t rs = block_rank(fl.marker, tmp, ts);
        if (fl.maximum) {
            if (i < cap_max) maxima[i] = (int32_t)(uint32_t)(keys[i] >> (b + 1));
        } else if (fl.arc || fl.marker) {
            const uint64_t k = keys[i];
            const uint32_t low = (uint32_t)(k & lowmask);
            if (fl.arc) {
                const uint32_t ap = abase + ra;
                if (ap < cap_arc) arc_maxima[ap] = (int32_t)low;
            } else {
                const uint32_t sp = sbase + rs;
                if (sp < cap_sad) {
                    saddles[sp] = (int32_t)((k >> (b + 1)) & lowmask);
                    if (beta) beta[sp] = (int32_t)low;
                    offsets[sp + 1] = (int32_t)(abase + ra);
                }
            }
        }
        abase += ta;
        sbase += ts;
    }
}

hipError_t launch_csr_counts(const uint64_t* keys, const uint32_t* count, int64_t cap, int bits, uint32_t* hist,
                             uint32_t* ctr, hipStream_t s)
{
    uint32_t* bsum = hist + 256 * kSortBlocks;
    hipLaunchKernelGGL(k_csr_count, dim3(kSortBlocks), dim3(256), 0, s, keys, count, (uint32_t)cap, bits, bsum);
    hipLaunchKernelGGL(k_csr_scan, dim3(1), dim3(256), 0, s, bsum, kSortBlocks, ctr);
    return hipGetLastError();
}

hipError_t launch_csr(const uint64_t* keys, const Work& w, int bits, const eg_out& o, hipStream_t s)
{
    uint32_t* bsum = w.hist + 256 * kSortBlocks;
    const uint32_t* count = &w.ctr[C_NKEYS];
    hipError_t e = launch_csr_counts(keys, count, w.cap_keys, bits, w.hist, w.ctr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_write, dim3(kSortBlocks), dim3(256), 0, s, keys, count, (uint32_t)w.cap_keys, bits,
                       bsum, o.saddles, o.saddle_beta, o.arc_offsets, (uint32_t)o.cap_sad, o.arc_maxima,
                       (uint32_t)o.cap_arc, o.maxima, (uint32_t)o.cap_max);
    return hipGetLastError();
}

}  // namespace eg
