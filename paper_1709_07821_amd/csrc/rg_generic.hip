// rg_generic.hip - the universal variant: both containers of a pair, of any
// type, are expanded into 8 KiB LDS bitsets, combined word by word, and the
// result goes through the common output step (P1 type, payload). It handles
// every type pair; the specialised kernels only make some pairs cheaper. Run
// containers, for which the paper gives no algorithm (Section 5.10, Section 6),
// go through the ballot/prefix-XOR expansion of expand_container().
//
// One 256-thread workgroup per container pair, grid-stride over the list.
#include "rg_count_dev.h"

namespace rg {

template <int OP, bool MAT>
__global__ void __launch_bounds__(256) k_generic(ComputeArgs a) {
    __shared__ WgShared sh;
    const uint32_t n = a.n;
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t slot = uniform(a.list[i]);
        const Task t = uniform_task(a.tasks, slot);
        const uint64_t t0 = (!MAT && a.cost) ? __builtin_amdgcn_s_memtime() : 0;
        expand_container(sh.sa, a.A, t.ia, sh);
        expand_container(sh.sb, a.B, t.ib, sh);
        uint64_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = apply_op<OP>(sh.sa[4 * threadIdx.x + j], sh.sb[4 * threadIdx.x + j]);
        if (MAT) {
            finalize_words(w, slot, a.so, sh.sa, sh.sb, sh);
        } else {
            const uint32_t c = count_words(w, sh);
            if (threadIdx.x == 0) acc_add(a.acc, t.pair, (long long)c);
            if (a.cost && threadIdx.x == 0) a.cost[slot] = 4.f * (float)(__builtin_amdgcn_s_memtime() - t0);
        }
        __syncthreads();
    }
}

void launch_generic(const ComputeArgs& a, hipStream_t st) {
    uint32_t grid = a.n;
    if (!grid) return;
    if (grid > 65536u) grid = 65536u;
    // count-only calls accumulate the intersection for every operation; the
    // binned path materialises intersections only
    if (!a.materialize) hipLaunchKernelGGL((k_generic<RG_AND, false>), dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_generic<RG_AND, true>), dim3(grid), dim3(256), 0, st, a);
}

}  // namespace rg
