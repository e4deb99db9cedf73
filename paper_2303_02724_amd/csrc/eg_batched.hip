// eg_batched.hip -- the stages after classification for a batch of fields.
//
// Every kernel here covers all fields of the batch in one launch: the grid's
// y dimension is the field, x strides over that field's items.  The arcs of
// all fields go through one radix sort: the field index sits above the key
// bits of a single field (bits 2B+2 and up, B = id bits of the largest
// field), so the sorted keys come out grouped by field, and the CSR kernels
// subtract each field's segment start to get field-local positions.
#include "eg_internal.h"
#include "eg_rows.h"

namespace eg {

constexpr int kBatchBlocksPerField = 48;

template <int NDIM>
struct AdjTable {
    uint64_t adj[Rows<NDIM>::K];
};
template <int NDIM>
constexpr AdjTable<NDIM> make_adj()
{
    constexpr Rows<NDIM> r = make_rows_ce<NDIM>();
    AdjTable<NDIM> t{};
    for (int j = 0; j < Rows<NDIM>::K; ++j) t.adj[j] = r.adj[j];
    return t;
}
__constant__ AdjTable<2> c_adj2 = make_adj<2>();
__constant__ AdjTable<3> c_adj3 = make_adj<3>();

__device__ __forceinline__ uint32_t rd(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool bgate(const uint32_t* bctr, int flag_base, int pass)
{
    return pass == 0 || rd(&bctr[flag_base + pass - 1]) != 0;
}

__device__ __forceinline__ int next_link_b(const int32_t* lab, const int32_t* res, int N, int x)
{
    return x >= -N ? lab[-x - 1] : res[-x - 1 - N];
}

__global__ __launch_bounds__(256) void k_binit(const BatchPlan* __restrict__ plan)
{
    const BatchField& F = plan->fields[blockIdx.x];
    const int t = threadIdx.x;
    if (t < C_SLOTS) F.ta.ctr[t] = 0;
    if (t < EG_H_SLOTS) F.header[t] = 0;
    if (blockIdx.x == 0) {
        if (t < C_SLOTS) plan->bctr[t] = 0;
        for (int i = t; i < 3 * (plan->count + 1); i += blockDim.x) plan->seg[i] = 0;
    }
}

// ------------------------------------------------------------------ labels

__global__ __launch_bounds__(256) void k_bexit_init(const BatchPlan* __restrict__ plan)
{
    const BatchField& F = plan->fields[blockIdx.y];
    const uint32_t req = rd(&F.ta.ctr[C_NEXIT]);
    const uint32_t n = req < F.ta.cap_exit ? req : F.ta.cap_exit;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        F.exres[i] = F.ta.lab[F.ta.exits[i]];
}

__global__ __launch_bounds__(256) void k_bexit_jump(const BatchPlan* __restrict__ plan, int pass)
{
    if (!bgate(plan->bctr, C_JUMP, pass)) return;
    const BatchField& F = plan->fields[blockIdx.y];
    const uint32_t req = rd(&F.ta.ctr[C_NEXIT]);
    const uint32_t n = req < F.ta.cap_exit ? req : F.ta.cap_exit;
    const int N = F.N;
    const int32_t* lab = F.ta.lab;
    int32_t* res = F.exres;
    bool notdone = false;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        int x = res[i];
        if (x >= 0) continue;
        int h = 0;
        do {
            x = next_link_b(lab, res, N, x);
            ++h;
        } while (x < 0 && h < plan->tuning.hops);
        res[i] = x;
        notdone |= x < 0;
    }
    if (__ballot(notdone) != 0 && __lane_id() == 0) atomicOr(&plan->bctr[C_JUMP + pass], 1u);
}

__global__ __launch_bounds__(256) void k_bfinal(const BatchPlan* __restrict__ plan, int pass)
{
    if (!bgate(plan->bctr, C_FINAL, pass)) return;
    const BatchField& F = plan->fields[blockIdx.y];
    const int N = F.N;
    int32_t* lab = F.ta.lab;
    const int32_t* res = F.exres;
    bool notdone = false;
    const int nq = N >> 2;
    int4* lab4 = reinterpret_cast<int4*>(lab);
    const int stride = gridDim.x * blockDim.x;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
        const int4 x = lab4[q];
        if ((x.x | x.y | x.z | x.w) >= 0) continue;
        int y0 = x.x < 0 ? next_link_b(lab, res, N, x.x) : x.x;
        int y1 = x.y < 0 ? next_link_b(lab, res, N, x.y) : x.y;
        int y2 = x.z < 0 ? next_link_b(lab, res, N, x.z) : x.z;
        int y3 = x.w < 0 ? next_link_b(lab, res, N, x.w) : x.w;
        int h = 1;
        const int hops = plan->tuning.hops;
        while ((y0 < 0 || y1 < 0 || y2 < 0 || y3 < 0) && h < hops) {
            if (y0 < 0) y0 = next_link_b(lab, res, N, y0);
            if (y1 < 0) y1 = next_link_b(lab, res, N, y1);
            if (y2 < 0) y2 = next_link_b(lab, res, N, y2);
            if (y3 < 0) y3 = next_link_b(lab, res, N, y3);
            ++h;
        }
        lab4[q] = make_int4(y0, y1, y2, y3);
        notdone |= (y0 < 0) | (y1 < 0) | (y2 < 0) | (y3 < 0);
    }
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (N & 3)) {
        const int v = (nq << 2) + t;
        int y = lab[v];
        for (int h = 0; y < 0 && h < plan->tuning.hops; ++h) y = next_link_b(lab, res, N, y);
        lab[v] = y;
        notdone |= y < 0;
    }
    if (__ballot(notdone) != 0 && __lane_id() == 0) atomicOr(&plan->bctr[C_FINAL + pass], 1u);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&F.ta.ctr[C_PASSES], 1u);
}

// ------------------------------------------------------------------ arcs

__device__ __forceinline__ uint64_t field_key(uint32_t f, uint64_t k, int B) { return (uint64_t(f) << (2 * B + 2)) | k; }

__global__ __launch_bounds__(256) void k_bload_maxima(const BatchPlan* __restrict__ plan)
{
    const uint32_t f = blockIdx.y;
    const BatchField& F = plan->fields[f];
    const int B = plan->bits;
    const uint32_t req = rd(&F.ta.ctr[C_NMAX]);
    const uint32_t n = req < F.ta.cap_max ? req : F.ta.cap_max;
    const uint32_t cap = (uint32_t)plan->cap_keys;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&F.ta.ctr[C_NKEYS], n);
    const int lane = __lane_id();
    for (uint32_t base = (blockIdx.x * blockDim.x + threadIdx.x) & ~63u; base < n; base += gridDim.x * blockDim.x) {
        const uint32_t i = base + lane;
        const uint32_t m = (uint32_t)__popcll(__ballot(i < n));
        uint32_t pos = 0;
        if (lane == 0) pos = atomicAdd(&plan->bctr[C_NKEYS], m);
        pos = __shfl(pos, 0) + lane;
        if (i < n && pos < cap) plan->keysA[pos] = field_key(f, max_key(F.ta.umax[i], B), B);
    }
}

// Saddle reps of 2D/3D fields with the compile-time rows; coordinates give
// the boundary test.
template <int NDIM>
__device__ __forceinline__ void breps_one(const BatchField& F, uint32_t f, int v, const BatchPlan* plan, int B)
{
    constexpr Rows<NDIM> R = make_rows_ce<NDIM>();
    constexpr int K = Rows<NDIM>::K;
    const TileArgs& a = F.ta;
    const int X = a.X, Y = a.Y, Z = a.Z;
    const int x = v % X, y = (v / X) % Y, z = NDIM == 3 ? v / (X * Y) : 0;
    const bool minima = F.minima != 0;
    const uint32_t kv = order_key(a.f[v]);
    const uint32_t uv = minima ? ~kv : kv;
    uint32_t up = 0;
    int ids[K];
    uint32_t us[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int dz = NDIM == 3 ? R.d[j][0] : 0, dy = R.d[j][NDIM - 2], dx = R.d[j][NDIM - 1];
        const bool in = (unsigned)(x + dx) < (unsigned)X && (unsigned)(y + dy) < (unsigned)Y &&
                        (unsigned)(z + dz) < (unsigned)Z;
        const int u_id = v + (dz * Y + dy) * X + dx;
        ids[j] = u_id;
        uint32_t u = 0;
        if (in) {
            const uint32_t ku = order_key(a.f[u_id]);
            u = minima ? ~ku : ku;
        }
        us[j] = u;
        const bool wins_tie = (j >= K / 2) != minima;
        const bool above = in && (wins_tie ? (u >= uv) : (u > uv));
        up |= uint32_t(above) << j;
    }
    const uint64_t* adj = NDIM == 3 ? c_adj3.adj : c_adj2.adj;
    int beta = 0;
    for (uint32_t rem = up; rem;) {
        rem &= ~(uint32_t)closure(rem & (~rem + 1u), rem, adj);
        ++beta;
    }
    const uint32_t cap = (uint32_t)plan->cap_keys;
    atomicAdd(&a.ctr[C_NKEYS], (uint32_t)(beta + 1));
    uint32_t q = atomicAdd(&plan->bctr[C_NKEYS], (uint32_t)(beta + 1));
    for (uint32_t rem = up; rem;) {
        const uint32_t c = (uint32_t)closure(rem & (~rem + 1u), rem, adj);
        rem &= ~c;
        uint32_t best_u = 0;
        int rep = v;
        for (uint32_t xm = c; xm;) {
            const int j = minima ? 31 - __clz(xm) : __ffs(xm) - 1;
            xm &= ~(1u << j);
            if (us[j] >= best_u) {
                best_u = us[j];
                rep = ids[j];
            }
        }
        if (q < cap) plan->keysA[q] = field_key(f, saddle_key((uint32_t)v, (uint32_t)a.lab[rep], 0u, B), B);
        ++q;
    }
    if (q < cap) plan->keysA[q] = field_key(f, saddle_key((uint32_t)v, (uint32_t)beta, 1u, B), B);
}

__global__ __launch_bounds__(256) void k_breps(const BatchPlan* __restrict__ plan)
{
    const uint32_t f = blockIdx.y;
    const BatchField& F = plan->fields[f];
    const int B = plan->bits;
    const uint32_t req = rd(&F.ta.ctr[C_NSAD]);
    const uint32_t n = req < F.ta.cap_sad ? req : F.ta.cap_sad;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int v = (int)F.ta.usad[i];
        if (F.ndim == 3)
            breps_one<3>(F, f, v, plan, B);
        else
            breps_one<2>(F, f, v, plan, B);
    }
}

// ------------------------------------------------------------------ CSR

__device__ __forceinline__ uint32_t bchunk(uint32_t n, uint32_t nblocks, uint32_t blk, uint32_t& lo, uint32_t& hi)
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

struct BFlags {
    bool maximum, arc, marker, start;
    uint32_t f;
};

__device__ __forceinline__ BFlags bkey_flags(const uint64_t* keys, uint32_t i, uint32_t n, int B)
{
    BFlags r{false, false, false, false, 0};
    if (i < n) {
        const uint64_t k = keys[i];
        r.f = (uint32_t)(k >> (2 * B + 2));
        r.maximum = !((k >> (2 * B + 1)) & 1ull);
        r.marker = !r.maximum && ((k >> B) & 1ull);
        const uint64_t prev = i > 0 ? keys[i - 1] : ~0ull;
        r.arc = !r.maximum && !r.marker && prev != k;
        r.start = i == 0 || (uint32_t)(prev >> (2 * B + 2)) != r.f;
    }
    return r;
}

__device__ __forceinline__ uint32_t brank(bool flag, uint32_t* tmp, uint32_t& total)
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

// Pass 1 (segment starts) and pass 2 (writes) share the rank computation.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_bcsr(const BatchPlan* __restrict__ plan, const uint64_t* __restrict__ keys)
{
    __shared__ uint32_t tmp[4];
    const int B = plan->bits;
    const uint32_t req = rd(&plan->bctr[C_NKEYS]);
    const uint32_t cap = (uint32_t)plan->cap_keys;
    const uint32_t n = req < cap ? req : cap;
    uint32_t lo, hi;
    bchunk(n, gridDim.x, blockIdx.x, lo, hi);
    const uint32_t* bsum = plan->hist + 256 * kSortBlocks;
    uint32_t abase = bsum[blockIdx.x], sbase = bsum[gridDim.x + blockIdx.x];
    uint32_t* seg = plan->seg;
    const uint64_t lowmask = (1ull << B) - 1ull;
    for (uint32_t base = lo; base < hi; base += 256) {
        const uint32_t i = base + threadIdx.x;
        const BFlags fl = bkey_flags(keys, i, hi, B);
        uint32_t ta, ts;
        const uint32_t ra = abase + brank(fl.arc, tmp, ta);
        const uint32_t rs = sbase + brank(fl.marker, tmp, ts);
        if (!WRITE) {
            if (fl.start) {
                seg[3 * fl.f] = i;
                seg[3 * fl.f + 1] = ra;
                seg[3 * fl.f + 2] = rs;
            }
        } else if (i < hi) {
            const BatchField& F = plan->fields[fl.f];
            const uint64_t k = keys[i];
            const uint32_t low = (uint32_t)(k & lowmask);
            if (fl.maximum) {
                const uint32_t m = i - seg[3 * fl.f];
                if (m < F.ta.cap_max) F.maxima[m] = (int32_t)(uint32_t)((k >> (B + 1)) & lowmask);
            } else if (fl.arc) {
                const uint32_t ap = ra - seg[3 * fl.f + 1];
                if (ap < F.cap_arc) F.arcs[ap] = (int32_t)low;
            } else if (fl.marker) {
                const uint32_t sp = rs - seg[3 * fl.f + 2];
                if (sp < F.ta.cap_sad) {
                    F.saddles[sp] = (int32_t)((k >> (B + 1)) & lowmask);
                    if (F.beta) F.beta[sp] = (int32_t)low;
                    F.offsets[sp + 1] = (int32_t)(ra - seg[3 * fl.f + 1]);
                }
            }
        }
        abase += ta;
        sbase += ts;
    }
    if (!WRITE && blockIdx.x == 0 && threadIdx.x == 0) {
        const int c = plan->count;
        seg[3 * c] = n;
        seg[3 * c + 1] = rd(&plan->bctr[C_NARC]);
        seg[3 * c + 2] = rd(&plan->bctr[C_NSADF]);
    }
}

__global__ void k_bfinalize(const BatchPlan* __restrict__ plan)
{
    if (threadIdx.x != 0) return;
    const int f = blockIdx.x;
    const BatchField& F = plan->fields[f];
    const uint32_t* c = F.ta.ctr;
    const uint32_t* seg = plan->seg;
    const int64_t nmax = c[C_NMAX], nsad = c[C_NSAD], nkeys = c[C_NKEYS];
    const int64_t narc = (int64_t)seg[3 * (f + 1) + 1] - (int64_t)seg[3 * f + 1];
    const bool keys_over = rd(&plan->bctr[C_NKEYS]) > plan->cap_keys;
    const bool sad_over = nsad > F.ta.cap_sad;
    const int64_t nmax_keys = nmax < F.ta.cap_max ? nmax : F.ta.cap_max;
    int status = EG_OK;
    if (c[C_NAN])
        status = EG_ERR_NAN;
    else if (nmax > F.ta.cap_max || sad_over || keys_over || narc > F.cap_arc)
        status = EG_ERR_CAPACITY;
    F.offsets[0] = 0;
    F.header[EG_H_STATUS] = status;
    F.header[EG_H_NMAX] = (int32_t)nmax;
    F.header[EG_H_NSAD] = (int32_t)nsad;
    F.header[EG_H_NARC] = (sad_over || keys_over) ? -1 : (int32_t)narc;
    F.header[EG_H_NPAIRS] = sad_over ? -1 : (int32_t)(nkeys - nsad - nmax_keys);
    F.header[EG_H_PASSES] = (int32_t)c[C_PASSES];
    F.header[EG_H_EXITS] = (int32_t)c[C_NEXIT];
}

hipError_t launch_batched_init(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    hipLaunchKernelGGL(k_binit, dim3(hplan.count), dim3(256), 0, s, dplan);
    return hipGetLastError();
}

hipError_t launch_batched_rest(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    const dim3 grid(kBatchBlocksPerField, hplan.count);
    hipLaunchKernelGGL(k_bexit_init, grid, dim3(256), 0, s, dplan);
    for (int p = 0; p < hplan.tuning.passes; ++p) hipLaunchKernelGGL(k_bexit_jump, grid, dim3(256), 0, s, dplan, p);
    for (int p = 0; p < hplan.tuning.passes; ++p) hipLaunchKernelGGL(k_bfinal, grid, dim3(256), 0, s, dplan, p);
    hipLaunchKernelGGL(k_bload_maxima, grid, dim3(256), 0, s, dplan);
    hipLaunchKernelGGL(k_breps, grid, dim3(256), 0, s, dplan);
    uint64_t* sorted = nullptr;
    hipError_t e = launch_sort(hplan.keysA, hplan.keysB, &hplan.bctr[C_NKEYS], hplan.cap_keys,
                               hplan.fbits + 2 * hplan.bits + 2, hplan.hist, &sorted, s);
    if (e != hipSuccess) return e;
    // block sums, their scan (totals into the batch counters), segment starts, writes
    e = launch_csr_counts(sorted, &hplan.bctr[C_NKEYS], hplan.cap_keys, hplan.bits, hplan.hist, hplan.bctr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_bcsr<false>), dim3(kSortBlocks), dim3(256), 0, s, dplan, sorted);
    hipLaunchKernelGGL((k_bcsr<true>), dim3(kSortBlocks), dim3(256), 0, s, dplan, sorted);
    hipLaunchKernelGGL(k_bfinalize, dim3(hplan.count), dim3(64), 0, s, dplan);
    return hipGetLastError();
}

}  // namespace eg
