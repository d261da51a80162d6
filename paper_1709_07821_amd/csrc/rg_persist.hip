// rg_persist.hip - one persistent kernel for the listed container pairs of a
// batched count-only call (a plan). Small-array pairs never get here: key
// matching counts them itself. A fixed grid (a few workgroups per CU) drains
// per-bin work counters with atomics, largest items first: workgroup-sized
// tasks (generic LDS expansion, merge path), then wave-sized tasks (bitset
// pairs, galloping search, bitset probes, run merges), each wave grabbing its
// own. Every wave exits when all counters are drained, so the grid always
// finishes.
//
// The kernel accumulates |A n B| per pair, whatever operation was asked for:
// union, symmetric difference and difference counts follow from it and the
// stored totals (Section 5.9), so one instantiation serves all four.
#include "rg_count_dev.h"

namespace rg {

// Next item index from a bin's work counter. Read-modify-writes of one
// address are serialised in its L2 channel, so thousands of waves asking an
// exhausted counter would queue behind each other: a coherent plain read
// first, and the atomic only while items remain. A stale read only costs the
// atomic; the atomic's result decides.
__device__ __forceinline__ uint32_t take_next(uint32_t* next, uint32_t cnt) {
    const uint32_t seen = __hip_atomic_load(next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return seen >= cnt ? seen : atomicAdd(next, 1u);
}

__global__ void __launch_bounds__(256) k_persist(PersistArgs a) {
    __shared__ WgShared sh;
    __shared__ uint32_t grab;
    const uint32_t lane = lane_id();
    // workgroup-sized tasks, largest first, taken from a counter
#pragma unroll 1
    for (int q = 0; q < 2; ++q) {
        const int b = q == 0 ? BIN_GEN : BIN_AA;
        const uint32_t cnt = uniform(a.bin_info[b]), off = uniform(a.bin_info[NBINS + b]);
        if (cnt == 0) continue;
        for (;;) {
            if (threadIdx.x == 0) grab = take_next(&a.next[b], cnt);
            __syncthreads();
            const uint32_t i = uniform(grab);
            __syncthreads();
            if (i >= cnt) break;
            const Task t = uniform_task(a.tasks, uniform(a.lists[off + i]));
            if (b == BIN_GEN) {
                const uint32_t c = generic_count_wg<RG_AND>(a.A, a.B, t, sh);
                if (threadIdx.x == 0) acc_add(a.acc, t.pair, (long long)c);
            } else {
                const uint32_t inter = merge_inter_wg(a.A, a.B, t, reinterpret_cast<uint16_t*>(sh.sa),
                                                      reinterpret_cast<uint16_t*>(sh.sb), sh.tmp64);
                if (threadIdx.x == 0) acc_add(a.acc, t.pair, (long long)inter);
            }
            __syncthreads();
        }
    }
    // wave-sized tasks: each wave grabs independently
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const int b = q == 0 ? BIN_BB : q == 1 ? BIN_GALLOP : q == 2 ? BIN_AB : BIN_RR;
        const uint32_t cnt = uniform(a.bin_info[b]), off = uniform(a.bin_info[NBINS + b]);
        if (cnt == 0) continue;
        for (;;) {
            // lane 0 takes the next item; readlane makes the index a scalar, so
            // the loop exit below is one branch for the whole wave
            uint32_t v = 0;
            if (lane == 0) v = take_next(&a.next[b], cnt);
            const uint32_t i = __builtin_amdgcn_readlane(v, 0);
            if (i >= cnt) break;
            const Task t = uniform_task(a.tasks, uniform(a.lists[off + i]));
            if (b == BIN_BB) {
                const uint32_t c = bb_count_wave<RG_AND>(a.A, a.B, t, lane);
                if (lane == 0) acc_add(a.acc, t.pair, (long long)c);
            } else {
                const uint32_t inter = wave_inter(a.A, a.B, t, lane);
                if (lane == 0) acc_add(a.acc, t.pair, (long long)inter);
            }
        }
    }
}

void launch_persist(const PersistArgs& a, uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(k_persist, dim3(grid), dim3(256), 0, st, a);
}

}  // namespace rg
