// rg_bitset.hip - bitset op bitset with fused population count (Section 4.1.2)
// and the on-the-fly output-type decision for the result (Section 1).
//
// One wave64 per container pair. Each lane loads 8 x 16 bytes from each
// input (coalesced dwordx4, 8 KiB per input per wave), combines the words in
// registers and counts them with the native per-lane popcount; the 64 lane
// counts are summed across the wave. The count-only form stops there (16 KiB
// read, 8 bytes of atomic add). The materialising form also counts the runs
// of the result, decides the P1 type, and writes the 8 KiB bitset straight
// from registers when the result is a bitset; the rare array/run results are
// handed to the LDS kernel (redo list), which recomputes them.
//
// Word order in registers: lane l, step k holds words 128k + 2l and
// 128k + 2l + 1 (lo, hi), so the word preceding (k, l, lo) is (k, l-1, hi),
// or (k-1, 63, hi) for lane 0.
#include "rg_count_dev.h"

namespace rg {

// Count-only form: |A n B| per bitset pair (every operation's count follows
// from it). One pair per wave: a grid-stride variant with a fixed 65536-block
// grid measured slower on MI355X (6.75 vs 6.4 ms for 2.56e6 pairs).

__global__ void __launch_bounds__(256) k_bb_count(ComputeArgs a) {
    const uint32_t lane = lane_id();
    const uint32_t stride = gridDim.x * 4;
    for (uint32_t w = wave_index(); w < a.n; w += stride) {
        const uint32_t slot = uniform(a.list[w]);
        const Task t = uniform_task(a.tasks, slot);
        const uint32_t c = bb_count_wave<RG_AND>(a.A, a.B, t, lane);
        if (lane == 0) acc_add(a.acc, t.pair, (long long)c);
    }
}

// Materialising form (intersection): words in registers, run count, P1 type,
// bitset results written from registers, other results to the redo list.
template <int OP>
__global__ void __launch_bounds__(256) k_bb_mat(ComputeArgs a) {
    const uint32_t lane = lane_id();
    const uint32_t w = wave_index();
    if (w >= a.n) return;
    const uint32_t slot = uniform(a.list[w]);
    const Task t = uniform_task(a.tasks, slot);
    const u32x4* pa = reinterpret_cast<const u32x4*>(a.A.payload + a.A.off[t.ia]);
    const u32x4* pb = reinterpret_cast<const u32x4*>(a.B.payload + a.B.off[t.ib]);
    u32x4 x[8], y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = __builtin_nontemporal_load(pa + k * 64 + lane);
        y[k] = __builtin_nontemporal_load(pb + k * 64 + lane);
    }
    uint64_t lo[8], hi[8];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint64_t xa = (uint64_t)x[k].x | ((uint64_t)x[k].y << 32);
        uint64_t xb = (uint64_t)x[k].z | ((uint64_t)x[k].w << 32);
        uint64_t ya = (uint64_t)y[k].x | ((uint64_t)y[k].y << 32);
        uint64_t yb = (uint64_t)y[k].z | ((uint64_t)y[k].w << 32);
        lo[k] = apply_op<OP>(xa, ya);
        hi[k] = apply_op<OP>(xb, yb);
        c += __popcll(lo[k]) + __popcll(hi[k]);
    }
    // run starts: bit set and the bit below it (previous word's MSB for bit 0) clear
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint64_t prev = __shfl_up(hi[k], 1);
        uint64_t wrap = k > 0 ? __shfl(hi[k > 0 ? k - 1 : 0], 63) : 0ull;
        if (lane == 0) prev = wrap;
        uint64_t s_lo = lo[k] & ~((lo[k] << 1) | (prev >> 63));
        uint64_t s_hi = hi[k] & ~((hi[k] << 1) | (lo[k] >> 63));
        r += __popcll(s_lo) + __popcll(s_hi);
    }
    uint64_t cr = wave_sum_u64((uint64_t)c | ((uint64_t)r << 32));
    c = (uint32_t)cr;
    r = (uint32_t)(cr >> 32);
    if (c == 0) return;  // empty result: slot stays empty
    const uint8_t type = p1_type(c, r);
    if (type == RG_BITSET) {
        u32x4* dst = reinterpret_cast<u32x4*>(a.so.payload + a.so.slot_off[slot]);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            u32x4 v;
            v.x = (uint32_t)lo[k];
            v.y = (uint32_t)(lo[k] >> 32);
            v.z = (uint32_t)hi[k];
            v.w = (uint32_t)(hi[k] >> 32);
            __builtin_nontemporal_store(v, dst + k * 64 + lane);
        }
        if (lane == 0) {
            a.so.res_card[slot] = c;
            a.so.res_type[slot] = RG_BITSET;
            a.so.res_size[slot] = 1024;
        }
    } else if (lane == 0) {
        uint32_t pos = atomicAdd(a.so.redo_count, 1u);
        a.so.redo_list[pos] = slot;
    }
}

void launch_bb(const ComputeArgs& a, hipStream_t st) {
    if (!a.n) return;
    const dim3 grid((a.n + 3) / 4);
    // count-only calls accumulate the intersection for every operation; the
    // binned path materialises intersections only (the other operations go
    // through the k-way path)
    if (!a.materialize) {
        hipLaunchKernelGGL(k_bb_count, grid, dim3(256), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_bb_mat<RG_AND>), grid, dim3(256), 0, st, a);
    }
}

}  // namespace rg
