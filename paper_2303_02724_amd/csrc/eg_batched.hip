// eg_batched.hip -- the label pass for a batch of fields.
//
// Every kernel here covers all fields of the batch in one launch: the grid's
// y dimension is the field, x strides over that field's items.  Stage (d)
// of a batch runs the stage (d) kernels with the batch field selector.
#include "eg_internal.h"

namespace eg {

constexpr int kBatchBlocksPerField = 48;
constexpr int kBatchLateBlocksPerField = 2;

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
    if (t < EG_H_SLOTS) F.arc.header[t] = 0;
    if (blockIdx.x == 0 && t < C_SLOTS) plan->bctr[t] = 0;
}

// ------------------------------------------------------------------ labels

// Both exit-list kernels take four consecutive entries per thread when the
// field's list and results are 16-byte aligned (one 16-byte access, four
// independent gathers or chains in flight), as the single-field kernels do.
__device__ __forceinline__ bool aligned16(const void* a, const void* b)
{
    return ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
}

__global__ __launch_bounds__(256) void k_bexit_init(const BatchPlan* __restrict__ plan)
{
    const BatchField F = plan->fields[blockIdx.y];  // a copy: loop loads cannot alias it
    const uint32_t req = rd(&F.ta.ctr[C_NEXIT]);
    const uint32_t n = req < F.ta.cap_exit ? req : F.ta.cap_exit;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    const int32_t* lab = F.ta.lab;
    uint32_t done = 0;
    if (aligned16(F.ta.exits, F.exres)) {
        const uint32_t nq = n >> 2;
        const uint4* e4 = reinterpret_cast<const uint4*>(F.ta.exits);
        int4* r4 = reinterpret_cast<int4*>(F.exres);
        for (uint32_t q = t; q < nq; q += stride) {
            const uint4 e = e4[q];
            r4[q] = make_int4(lab[e.x], lab[e.y], lab[e.z], lab[e.w]);
        }
        done = nq << 2;
    }
    for (uint32_t i = done + t; i < n; i += stride) F.exres[i] = lab[F.ta.exits[i]];
}

__global__ __launch_bounds__(256) void k_bexit_jump(const BatchPlan* __restrict__ plan, int pass)
{
    if (!bgate(plan->bctr, C_JUMP, pass)) return;
    const BatchField F = plan->fields[blockIdx.y];  // a copy: loop loads cannot alias it
    const uint32_t req = rd(&F.ta.ctr[C_NEXIT]);
    const uint32_t n = req < F.ta.cap_exit ? req : F.ta.cap_exit;
    const int N = F.N;
    const int32_t* lab = F.ta.lab;
    int32_t* res = F.exres;
    const int hops = plan->tuning.hops;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    bool notdone = false;
    uint32_t done = 0;
    if (aligned16(F.ta.exits, res)) {
        const uint32_t nq = n >> 2;
        int4* r4 = reinterpret_cast<int4*>(res);
        for (uint32_t q = t; q < nq; q += stride) {
            const int4 x = r4[q];
            if ((x.x | x.y | x.z | x.w) >= 0) continue;  // all four final
            int y0 = x.x, y1 = x.y, y2 = x.z, y3 = x.w;
            for (int h = 0; (y0 < 0 || y1 < 0 || y2 < 0 || y3 < 0) && h < hops; ++h) {
                if (y0 < 0) y0 = next_link_b(lab, res, N, y0);
                if (y1 < 0) y1 = next_link_b(lab, res, N, y1);
                if (y2 < 0) y2 = next_link_b(lab, res, N, y2);
                if (y3 < 0) y3 = next_link_b(lab, res, N, y3);
            }
            r4[q] = make_int4(y0, y1, y2, y3);
            notdone |= (y0 < 0) | (y1 < 0) | (y2 < 0) | (y3 < 0);
        }
        done = nq << 2;
    }
    for (uint32_t i = done + t; i < n; i += stride) {
        int x = res[i];
        if (x >= 0) continue;
        int h = 0;
        do {
            x = next_link_b(lab, res, N, x);
            ++h;
        } while (x < 0 && h < hops);
        res[i] = x;
        notdone |= x < 0;
    }
    if (__ballot(notdone) != 0 && __lane_id() == 0) atomicOr(&plan->bctr[C_JUMP + pass], 1u);
}

__global__ __launch_bounds__(256) void k_bfinal(const BatchPlan* __restrict__ plan, int pass)
{
    if (!bgate(plan->bctr, C_FINAL, pass)) return;
    const BatchField F = plan->fields[blockIdx.y];  // a copy: loop loads cannot alias it
    const int N = F.N;
    int32_t* lab = F.ta.lab;
    const int32_t* res = F.exres;
    const int hops = plan->tuning.hops;
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
        for (int h = 0; y < 0 && h < hops; ++h) y = next_link_b(lab, res, N, y);
        lab[v] = y;
        notdone |= y < 0;
    }
    if (__ballot(notdone) != 0 && __lane_id() == 0) atomicOr(&plan->bctr[C_FINAL + pass], 1u);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&F.ta.ctr[C_PASSES], 1u);
}

hipError_t launch_batched_init(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    hipLaunchKernelGGL(k_binit, dim3(hplan.count), dim3(256), 0, s, dplan);
    return hipGetLastError();
}

hipError_t launch_batched_rest(const BatchPlan* dplan, const BatchPlan& hplan, hipStream_t s)
{
    const dim3 grid(kBatchBlocksPerField, hplan.count);
    // later passes run only when the pass before stopped short, which is
    // rare: their launches mostly return at once, so they get small grids
    const dim3 late(kBatchLateBlocksPerField, hplan.count);
    hipLaunchKernelGGL(k_bexit_init, grid, dim3(256), 0, s, dplan);
    for (int p = 0; p < hplan.tuning.passes; ++p)
        hipLaunchKernelGGL(k_bexit_jump, p == 0 ? grid : late, dim3(256), 0, s, dplan, p);
    // pass 0 in tile order, the rest linear (each gated by the pass before)
    hipError_t e = launch_final_tiled_batched(dplan, hplan, s);
    if (e != hipSuccess) return e;
    for (int p = 1; p < hplan.tuning.passes; ++p) hipLaunchKernelGGL(k_bfinal, late, dim3(256), 0, s, dplan, p);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_arcs_batched(dplan, hplan, s);
}

}  // namespace eg
