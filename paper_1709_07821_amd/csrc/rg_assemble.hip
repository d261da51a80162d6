// rg_assemble.hip - output assembly and the cardinality / Jaccard step.
//
// Results are built as new bitmaps, inputs untouched (Section 5.7). Slots are
// in result key order; empty results are dropped (Section 2.2: no empty
// containers), the survivors are compacted by a prefix sum of non-empty
// flags. Payloads stay where their slot put them, so only the 19 bytes of
// metadata per container move.
//
// Counts: unmatched containers contribute their stored cardinality and
// matched pairs the population count of their result, so |A op B| needs no
// materialisation (Section 5.9); the Jaccard index follows from the
// identities |A u B| = |A| + |B| - |A n B|, |A \ B| = |A| - |A n B| and
// |A xor B| = |A| + |B| - 2|A n B| with one binary64 division.
#include "rg_internal.h"

namespace rg {

// A pair's slots are consecutive, so the 64 slots of a wave belong to a few
// runs of equal pair index: the per-bitmap totals are summed over each run
// (segmented scan over the lanes) and added by its last lane, one atomic per
// run instead of one per slot (thousands of slots of one pair otherwise
// serialise on its two counters).
__global__ void k_compact(CompactArgs c) {
    const uint32_t lane = lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < c.n_slots; base += stride) {
        const uint64_t s = base + lane;
        uint32_t card = 0, pair = 0xFFFFFFFFu;
        if (s < c.n_slots) {
            card = c.res_card[s];
            const Task t = c.tasks[s];
            pair = t.pair;
            if (card) {
                const uint64_t i = c.out_idx[s];
                c.keys[i] = t.key;
                c.types[i] = c.res_type[s];
                c.card[i] = card;
                c.size[i] = c.res_size[s];
                c.off[i] = c.slot_off[s];
            }
        }
        uint64_t sc = card, sw = card ? wbytes_of(card) : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t uc = __shfl_up(sc, o), uw = __shfl_up(sw, o);
            const uint32_t up = __shfl_up(pair, o);
            if (lane >= (uint32_t)o && up == pair) {  // pairs do not decrease along the slots
                sc += uc;
                sw += uw;
            }
        }
        const uint32_t next = __shfl_down(pair, 1);
        const bool last = lane == 63 || next != pair;
        if (last && pair != 0xFFFFFFFFu && sc) {
            atomicAdd(reinterpret_cast<unsigned long long*>(&c.bm_card[pair]), (unsigned long long)sc);
            if (c.bm_wbytes) atomicAdd(reinterpret_cast<unsigned long long*>(&c.bm_wbytes[pair]), (unsigned long long)sw);
        }
    }
}

void launch_compact(const CompactArgs& c, hipStream_t st) {
    if (!c.n_slots) return;
    uint64_t g = (c.n_slots + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_compact, dim3((uint32_t)g), dim3(256), 0, st, c);
}

// bm_begin of each pair of the wave: output index of its first slot
__global__ void k_bm_begin(const uint64_t* cand_off, const uint64_t* out_idx, uint64_t n_slots,
                           const uint64_t* out_total, uint32_t n_pairs, uint64_t pair0, uint64_t* bm_begin,
                           int last_wave) {
    uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_pairs) {
        uint64_t s = cand_off[p];
        bm_begin[pair0 + p] = s < n_slots ? out_idx[s] : *out_total;
    }
    if (last_wave && p == n_pairs) bm_begin[pair0 + n_pairs] = *out_total;
}

void launch_bm_begin(const uint64_t* cand_off, const uint64_t* out_idx, uint64_t n_slots, const uint64_t* out_total,
                     uint32_t n_pairs, uint64_t pair0, uint64_t* bm_begin, bool last_wave, hipStream_t st) {
    hipLaunchKernelGGL(k_bm_begin, dim3((n_pairs + 1 + 255) / 256), dim3(256), 0, st, cand_off, out_idx, n_slots,
                       out_total, n_pairs, pair0, bm_begin, (int)last_wave);
}

// Sums over the pairs of a batched call, for the host's sizing without reading
// the per-pair arrays back: out[0] candidate slots, out[1] result payload
// bound, out[2] result containers bound, out[3] the most slots of one pair
// (bound and min_cont may be null: count-only). out is zeroed by the launcher.
__global__ void __launch_bounds__(256) k_pair_totals(const uint32_t* n_cand, const uint64_t* bound,
                                                     const uint32_t* min_cont, uint64_t n, uint64_t* out) {
    uint64_t c = 0, b = 0, m = 0, most = 0;
    for (uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (uint64_t)gridDim.x * 256) {
        const uint64_t x = n_cand[p];
        c += x;
        most = x > most ? x : most;
        if (bound) b += bound[p];
        if (min_cont) m += min_cont[p];
    }
    c = wave_sum_u64(c);
    b = wave_sum_u64(b);
    m = wave_sum_u64(m);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(most, o);
        most = y > most ? y : most;
    }
    if (lane_id() == 0) {
        if (c) atomicAdd(reinterpret_cast<unsigned long long*>(&out[0]), (unsigned long long)c);
        if (b) atomicAdd(reinterpret_cast<unsigned long long*>(&out[1]), (unsigned long long)b);
        if (m) atomicAdd(reinterpret_cast<unsigned long long*>(&out[2]), (unsigned long long)m);
        if (most) atomicMax(reinterpret_cast<unsigned long long*>(&out[3]), (unsigned long long)most);
    }
}

void launch_pair_totals(const uint32_t* n_cand, const uint64_t* bound, const uint32_t* min_cont, uint64_t n,
                        uint64_t* out, hipStream_t st) {
    launch_fill_u64(out, 0, 4, st);
    if (!n) return;
    const uint64_t g = (n + 2047) / 2048;  // about eight pairs per thread
    hipLaunchKernelGGL(k_pair_totals, dim3(g < 1024 ? (uint32_t)g : 1024u), dim3(256), 0, st, n_cand, bound,
                       min_cont, n, out);
}

// |A n B| from |A op B| and the stored totals
__device__ __forceinline__ uint64_t inter_from(int op, uint64_t card, uint64_t na, uint64_t nb) {
    if (op == RG_AND) return card;
    if (op == RG_OR) return na + nb - card;
    if (op == RG_XOR) return (na + nb - card) / 2;
    return na - card;
}

__device__ __forceinline__ double jaccard_of(uint64_t inter, uint64_t na, uint64_t nb) {
    uint64_t uni = na + nb - inter;
    if (uni == 0) return 1.0;
    return (double)inter / (double)uni;
}

// |A op B| from |A n B| and the stored totals
__device__ __forceinline__ uint64_t card_from(int op, uint64_t inter, uint64_t na, uint64_t nb) {
    if (op == RG_AND) return inter;
    if (op == RG_OR) return na + nb - inter;
    if (op == RG_XOR) return na + nb - 2 * inter;
    return na - inter;
}

__global__ void k_finish_counts(int acc_op, int out_op, const long long* acc, PoolView A, PoolView B, uint32_t nA,
                                uint32_t nB, const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0,
                                uint64_t pair0, uint32_t n_pairs, uint64_t* d_cards, double* d_jacc) {
    uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    uint64_t p = pair0 + q;
    const uint64_t v = (uint64_t)acc[p];
    uint32_t a = ia ? ia[p] : ia0, b = ib ? ib[p] : ib0;
    if (a >= nA || b >= nB) {  // reported through the call's error flag
        if (d_cards) d_cards[p] = 0;
        if (d_jacc) d_jacc[p] = 0.0;
        return;
    }
    uint64_t na = A.bm_card[a], nb = B.bm_card[b];
    const uint64_t inter = inter_from(acc_op, v, na, nb);
    if (d_cards) d_cards[p] = acc_op == out_op ? v : card_from(out_op, inter, na, nb);
    if (d_jacc) d_jacc[p] = jaccard_of(inter, na, nb);
}

void launch_finish_counts(int acc_op, int out_op, const long long* acc, PoolView A, PoolView B, uint32_t nA,
                          uint32_t nB, const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0,
                          uint64_t pair0, uint32_t n_pairs, uint64_t* d_cards, double* d_jacc, hipStream_t st) {
    if (!n_pairs) return;
    hipLaunchKernelGGL(k_finish_counts, dim3((n_pairs + 255) / 256), dim3(256), 0, st, acc_op, out_op, acc, A, B,
                       nA, nB, ia, ib, ia0, ib0, pair0, n_pairs, d_cards, d_jacc);
}

__global__ void k_mat_counts(int op, const uint64_t* bm_card, PoolView A, PoolView B, const uint32_t* ia,
                             const uint32_t* ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs, uint64_t* d_cards,
                             double* d_jacc) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_pairs) return;
    uint64_t card = bm_card[p];
    if (d_cards) d_cards[p] = card;
    if (d_jacc) {
        uint32_t a = ia ? ia[p] : ia0, b = ib ? ib[p] : ib0;
        uint64_t na = A.bm_card[a], nb = B.bm_card[b];
        d_jacc[p] = jaccard_of(inter_from(op, card, na, nb), na, nb);
    }
}

void launch_mat_counts(int op, const uint64_t* bm_card, PoolView A, PoolView B, const uint32_t* ia,
                       const uint32_t* ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs, uint64_t* d_cards,
                       double* d_jacc, hipStream_t st) {
    if (!n_pairs) return;
    hipLaunchKernelGGL(k_mat_counts, dim3((uint32_t)((n_pairs + 255) / 256)), dim3(256), 0, st, op, bm_card, A, B,
                       ia, ib, ia0, ib0, n_pairs, d_cards, d_jacc);
}

}  // namespace rg
