// rg_variants.hip - specialised count-only variants for matched pairs with at
// least one array or run container. All four cardinalities follow from
// |A n B| (Section 5.9 identities), so each variant computes the intersection
// size of one container pair and adds it to the pair's accumulator; the
// requested count is derived once per pair at the end.
//
//   RG_V_MERGE    array-array: both arrays staged in LDS, merge path split over
//                 256 threads, each thread merges its diagonal segment
//                 (the sorted-block merge of Section 4.2, made data-parallel).
//   RG_V_GALLOP   array-array: every element of the smaller array is searched
//                 (binary search) in the larger one in global memory, one wave
//                 per pair: O(min log max), the galloping regime of Section 2.2.
//   RG_V_PROBE    array-bitset (either order): one bit test per array value
//                 (Section 3.2 bit addressing), one wave per pair.
//   RG_V_THREAD   any pair with an array side: one thread per pair looks every
//                 value of the (smaller) array up in the other container;
//                 chosen for small array sides, where a wave or a workgroup
//                 per pair would idle. Wave-aggregated atomics per pair.
//   RG_V_RUNMERGE run-run: interval intersection, each run of the side with
//                 fewer runs searches the other run list; run-array: each array
//                 value searches the run list; run-bitset: population count of
//                 the bitset words under each run. One wave per pair.
// Materialised results and any other combination use the generic LDS kernel.
#include "rg_count_dev.h"

namespace rg {

// One wave per pair: probe / gallop / run-merge by container types.
__global__ void __launch_bounds__(256) k_wave_count(ComputeArgs a) {
    const uint32_t lane = lane_id();
    const uint32_t w = wave_index();
    if (w >= a.n) return;
    const uint32_t slot = uniform(a.list[w]);
    const Task t = uniform_task(a.tasks, slot);
    const uint64_t t0 = a.cost ? __builtin_amdgcn_s_memtime() : 0;
    const uint32_t inter = wave_inter(a.A, a.B, t, lane);
    if (lane == 0) acc_add(a.acc, t.pair, (long long)inter);
    if (a.cost && lane == 0) a.cost[slot] = (float)(__builtin_amdgcn_s_memtime() - t0);
}

// Array-array merge path: one 256-thread workgroup per pair, both arrays in LDS.
__global__ void __launch_bounds__(256) k_merge_count(ComputeArgs a) {
    __shared__ uint16_t sA[4096];
    __shared__ uint16_t sB[4096];
    __shared__ uint64_t tmp64[4];
    for (uint32_t it = blockIdx.x; it < a.n; it += gridDim.x) {
        const uint32_t slot = uniform(a.list[it]);
        const Task t = uniform_task(a.tasks, slot);
        const uint64_t t0 = a.cost ? __builtin_amdgcn_s_memtime() : 0;
        const uint32_t inter = merge_inter_wg(a.A, a.B, t, sA, sB, tmp64);
        if (threadIdx.x == 0) acc_add(a.acc, t.pair, (long long)inter);
        // cost in wave-cycles: four waves for the task's duration
        if (a.cost && threadIdx.x == 0) a.cost[slot] = 4.f * (float)(__builtin_amdgcn_s_memtime() - t0);
        __syncthreads();
    }
}

// One thread per pair.
__global__ void __launch_bounds__(256) k_thread_count(ComputeArgs a) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    uint32_t pair = NONE, inter = 0, slot = NONE;
    const uint64_t t0 = a.cost ? __builtin_amdgcn_s_memtime() : 0;
    if (i < a.n) {
        slot = a.list[i];
        const Task t = a.tasks[slot];
        inter = thread_inter(a.A, a.B, t);
        pair = t.pair;
    }
    wave_aggregate_add(a.acc, pair, inter);
    if (a.cost) {
        // the wave's time, shared by its active lanes
        const uint64_t dt = __builtin_amdgcn_s_memtime() - t0;
        const uint32_t act = (uint32_t)__popcll(__ballot(slot != NONE));
        if (slot != NONE) a.cost[slot] = (float)dt / (float)act;
    }
}

static void launch_wave_count(const ComputeArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_wave_count, dim3((a.n + 3) / 4), dim3(256), 0, st, a);
}

static void launch_merge_count(const ComputeArgs& a, hipStream_t st) {
    const uint32_t g = a.n < 65536u ? a.n : 65536u;
    hipLaunchKernelGGL(k_merge_count, dim3(g), dim3(256), 0, st, a);
}

// The classifier only routes count-only pairs of the right types here;
// materialising calls use the generic kernel.
void launch_aa(const ComputeArgs& a, hipStream_t st) {
    if (!a.n) return;
    if (a.materialize) launch_generic(a, st);
    else launch_merge_count(a, st);
}
void launch_gallop(const ComputeArgs& a, hipStream_t st) {
    if (!a.n) return;
    if (a.materialize) launch_generic(a, st);
    else launch_wave_count(a, st);
}
void launch_ab(const ComputeArgs& a, hipStream_t st) {
    if (!a.n) return;
    if (a.materialize) launch_generic(a, st);
    else launch_wave_count(a, st);
}
void launch_thread(const ComputeArgs& a, hipStream_t st) {
    if (!a.n) return;
    if (a.materialize) launch_generic(a, st);
    else hipLaunchKernelGGL(k_thread_count, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
}
void launch_rr(const ComputeArgs& a, hipStream_t st) {
    if (!a.n) return;
    if (a.materialize) launch_generic(a, st);
    else launch_wave_count(a, st);
}

}  // namespace rg
