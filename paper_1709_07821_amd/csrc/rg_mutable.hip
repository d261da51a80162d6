// rg_mutable.hip - in-place operations on mutable bitmaps (A op= B).
//
// The paper changes containers in place: array values are set, cleared or
// flipped in a bitset while its cardinality is kept (Section 3.2), and wide
// unions are built partly in place (Section 5.9). A mutable pool gives every
// bitmap a directory of all 65536 keys (the slot of each present container)
// and keeps containers in fixed 8 KiB slots, which hold any container in P1
// form, so a result never has to move: slots come from and go back to a device
// free list. A op= B touches only the keys of B (for intersection, also
// drops A's keys that B lacks):
//   classify: each key of B is present in A (evaluate in A's slot) or absent
//     (union, symmetric difference: a new slot);
//   check: the op is skipped, with a sticky capacity error, when there are
//     fewer free slots than keys to insert - before anything changes;
//   evaluate: one workgroup per present key expands A's container into LDS,
//     applies B's (set / flip / clear per value or run, word-wise for bitsets,
//     AND through a second expansion), and writes the P1 result back into the
//     same slot; an empty result frees the slot;
//   insert: one wave per absent key takes a slot and copies B's container.
// Slots are only freed (pushed) in the drop and evaluate kernels and only
// taken (popped) in the insert kernel, so the free list never sees both at
// once. Every kernel adds its keys' change of cardinality to the bitmap's
// total, so bm_card is maintained without a recount.
#include "rg_finalize.h"
#include "rg_mutable.h"

namespace rg {

__device__ __forceinline__ PoolView mut_view(const MutView& m) {
    PoolView v{};
    v.types = m.s_type;
    v.card = m.s_card;
    v.size = m.s_size;
    v.off = m.s_off;
    v.payload = m.slab;
    return v;
}

__device__ __forceinline__ PoolView view_of(const rg_pool& P) {
    PoolView v{};
    v.bm_begin = P.bm_begin;
    v.keys = P.keys;
    v.types = P.types;
    v.card = P.card;
    v.size = P.size;
    v.off = P.off;
    v.payload = P.payload;
    v.bm_card = P.bm_card;
    v.bm_wbytes = P.bm_wbytes;
    return v;
}

__device__ __forceinline__ void mut_free(const MutView& m, uint32_t slot) {
    const int32_t i = atomicAdd(&m.ctl[0], 1);
    m.free_list[i] = slot;
}

__device__ __forceinline__ void add_card(const MutView& m, uint32_t b, long long d) {
    if (d) atomicAdd(reinterpret_cast<unsigned long long*>(&m.bm_card[b]), (unsigned long long)d);
}

// ------------------------------------------------------------------ set-up
__global__ void k_mut_init(MutView m) {
    const uint64_t nd = (uint64_t)m.n_bitmaps * MUT_KEYS;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += stride) m.dir[i] = NONE;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m.n_slots; i += stride) {
        m.free_list[i] = (uint32_t)(m.n_slots - 1 - i);
        m.s_off[i] = i * MUT_SLOT_BYTES;
        m.s_card[i] = 0;
        m.s_type[i] = 0;
        m.s_size[i] = 0;
    }
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m.n_bitmaps; i += stride) m.bm_card[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        m.ctl[0] = (int32_t)m.n_slots;
        m.ctl[1] = 0;
        m.ctl[2] = 0;
        m.ctl[3] = 0;
    }
}

void launch_mut_init(const MutView& m, hipStream_t st) {
    hipLaunchKernelGGL(k_mut_init, dim3(4096), dim3(256), 0, st, m);
}

// ------------------------------------------------------------------ one operation
__global__ void k_mut_begin(MutView m) {
    m.counts[0] = 0;
    m.counts[1] = 0;
    m.ctl[3] = 0;
}

__global__ void k_mut_classify(MutView m, int op, uint32_t b, rg_pool P, uint32_t src) {
    const uint64_t c0 = P.bm_begin[src], c1 = P.bm_begin[src + 1];
    const uint32_t* dir = m.dir + (uint64_t)b * MUT_KEYS;
    for (uint64_t j = c0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < c1;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t slot = dir[P.keys[j]];
        if (slot != NONE) {
            const uint32_t i = atomicAdd(&m.counts[0], 1u);
            m.present[2 * i] = (uint32_t)j;
            m.present[2 * i + 1] = slot;
        } else if (op == RG_OR || op == RG_XOR) {
            m.absent[atomicAdd(&m.counts[1], 1u)] = (uint32_t)j;
        }
    }
}

// the keys to insert must fit the free slots, else the whole op is skipped
__global__ void k_mut_check(MutView m) {
    if ((int64_t)m.counts[1] > (int64_t)m.ctl[0]) {
        m.ctl[3] = 1;
        m.ctl[1] = 1;
    }
}

// intersection: A's keys that B lacks become empty
__global__ void k_mut_and_drop(MutView m, uint32_t b, rg_pool P, uint32_t src) {
    __shared__ unsigned long long sum;
    if (threadIdx.x == 0) sum = 0;
    __syncthreads();
    const uint32_t key = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t* dir = m.dir + (uint64_t)b * MUT_KEYS;
    const uint32_t slot = key < MUT_KEYS ? dir[key] : NONE;
    if (slot != NONE) {
        uint64_t lo = P.bm_begin[src], hi = P.bm_begin[src + 1];
        const uint64_t e = hi;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (P.keys[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        if (lo == e || P.keys[lo] != key) {
            atomicAdd(&sum, (unsigned long long)m.s_card[slot]);
            m.s_card[slot] = 0;
            dir[key] = NONE;
            mut_free(m, slot);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) add_card(m, b, -(long long)sum);
}

// B's array or run container folded into the LDS bitset s: FOP 0 sets its
// values, 1 flips them, 2 clears them (Section 3.2, one word update per value)
template <int FOP>
__device__ __forceinline__ void mut_fold(uint64_t* s, const uint8_t* pl, uint8_t type, uint32_t size) {
    auto apply = [&](uint32_t wi, uint64_t mk) {
        unsigned long long* d = reinterpret_cast<unsigned long long*>(&s[wi]);
        if (FOP == 0) atomicOr(d, mk);
        else if (FOP == 1) atomicXor(d, mk);
        else atomicAnd(d, ~mk);
    };
    if (type == RG_ARRAY) {
        const uint16_t* a = reinterpret_cast<const uint16_t*>(pl);
        for (uint32_t i = threadIdx.x; i < size; i += blockDim.x) apply(a[i] >> 6, 1ull << (a[i] & 63));
    } else {
        const uint32_t* r = reinterpret_cast<const uint32_t*>(pl);
        for (uint32_t i = threadIdx.x; i < size; i += blockDim.x) {
            const uint32_t first = r[i] & 0xFFFFu, last = first + (r[i] >> 16);
            for (uint32_t wi = first >> 6; wi <= last >> 6; ++wi) {
                const uint32_t lo = wi == first >> 6 ? first & 63 : 0;
                const uint32_t hi = wi == last >> 6 ? last & 63 : 63;
                apply(wi, (~0ull << lo) & (~0ull >> (63 - hi)));
            }
        }
    }
    __syncthreads();
}

// M[b]'s container in `slot` op= container j of P, in place (one workgroup):
// A's container is expanded into LDS, B's applied (set / flip / clear per
// value or run, word-wise for bitsets, AND through a second expansion), and
// the P1 result written back into the same slot; an empty result frees it.
// The bitmap's cardinality moves by the key's change.
__device__ void mut_eval_one(const MutView& m, int op, uint32_t b, const rg_pool& P, uint32_t j, uint32_t slot,
                             WgShared& sh) {
    const uint32_t tid = threadIdx.x;
    const PoolView A = mut_view(m);
    const PoolView B = view_of(P);
    const SlotOut so{m.s_off, m.slab, m.s_card, m.s_type, m.s_size};
    const uint32_t old_c = uniform(m.s_card[slot]);
    const uint16_t key = (uint16_t)uniform(P.keys[j]);
    expand_container(sh.sa, A, slot, sh);  // ends with a barrier
    const uint8_t tb = (uint8_t)uniform(P.types[j]);
    const uint32_t sb = uniform(P.size[j]);
    const uint8_t* pb = P.payload + uniform64(P.off[j]);
    uint64_t w[4];
    if (op == RG_AND || tb == RG_BITSET) {
        if (op == RG_AND) expand_container(sh.sb, B, j, sh);
        const uint64_t* bw = op == RG_AND ? sh.sb : reinterpret_cast<const uint64_t*>(pb);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t a = sh.sa[4 * tid + q], x = bw[4 * tid + q];
            w[q] = op == RG_AND ? (a & x) : op == RG_OR ? (a | x) : op == RG_XOR ? (a ^ x) : (a & ~x);
        }
    } else {
        if (op == RG_OR) mut_fold<0>(sh.sa, pb, tb, sb);
        else if (op == RG_XOR) mut_fold<1>(sh.sa, pb, tb, sb);
        else mut_fold<2>(sh.sa, pb, tb, sb);
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = sh.sa[4 * tid + q];
    }
    // the result goes back into A's slot (8 KiB: any P1 container fits);
    // A's payload was read into LDS above, so nothing still reads it
    const uint32_t c = finalize_words(w, slot, so, sh.sa, sh.sb, sh);
    if (tid == 0) {
        if (c == 0) {
            m.s_card[slot] = 0;
            m.dir[(uint64_t)b * MUT_KEYS + key] = NONE;
            mut_free(m, slot);
        }
        add_card(m, b, (long long)c - (long long)old_c);
    }
    __syncthreads();
}

__global__ void __launch_bounds__(256) k_mut_eval(MutView m, int op, uint32_t b, rg_pool P) {
    __shared__ WgShared sh;
    if (uniform((uint32_t)m.ctl[3])) return;  // skipped: not enough free slots
    const uint32_t n = uniform(m.counts[0]);
    for (uint32_t i = blockIdx.x; i < n; i += gridDim.x)
        mut_eval_one(m, op, b, P, uniform(m.present[2 * i]), uniform(m.present[2 * i + 1]), sh);
}

// union, symmetric difference: one wave per key A lacks takes a free slot and
// copies B's container (already in P1 form)
// container j of P copied into a free slot as M[b]'s container at its key (one wave)
__device__ __forceinline__ void mut_insert_one(const MutView& m, uint32_t b, const rg_pool& P, uint32_t j,
                                               uint32_t lane) {
    uint32_t slot = 0;
    if (lane == 0) slot = m.free_list[atomicSub(&m.ctl[0], 1) - 1];  // the check kept this >= 0
    slot = __builtin_amdgcn_readlane(slot, 0);
    const uint8_t t = (uint8_t)uniform(P.types[j]);
    const uint32_t sz = uniform(P.size[j]), c = uniform(P.card[j]);
    const uint32_t units = (payload_bytes_of(t, sz) + 15) / 16;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(P.payload + uniform64(P.off[j]));
    u32x4* d4 = reinterpret_cast<u32x4*>(m.slab + (uint64_t)slot * MUT_SLOT_BYTES);
    for (uint32_t u = lane; u < units; u += 64) d4[u] = s4[u];
    if (lane == 0) {
        m.s_type[slot] = t;
        m.s_size[slot] = sz;
        m.s_card[slot] = c;
        m.dir[(uint64_t)b * MUT_KEYS + P.keys[j]] = slot;
        add_card(m, b, (long long)c);
    }
}

__global__ void __launch_bounds__(256) k_mut_insert(MutView m, uint32_t b, rg_pool P) {
    const uint32_t lane = lane_id();
    if (uniform((uint32_t)m.ctl[3])) return;
    const uint32_t n = uniform(m.counts[1]);
    const uint32_t nwaves = gridDim.x * 4;
    for (uint32_t i = wave_index(); i < n; i += nwaves) mut_insert_one(m, b, P, uniform(m.absent[i]), lane);
}

void launch_mut_op(const MutView& m, int op, uint32_t b, const rg_pool& P, uint32_t src, hipStream_t st) {
    hipLaunchKernelGGL(k_mut_begin, dim3(1), dim3(1), 0, st, m);
    hipLaunchKernelGGL(k_mut_classify, dim3(64), dim3(256), 0, st, m, op, b, P, src);
    if (op == RG_OR || op == RG_XOR) hipLaunchKernelGGL(k_mut_check, dim3(1), dim3(1), 0, st, m);
    if (op == RG_AND) hipLaunchKernelGGL(k_mut_and_drop, dim3(MUT_KEYS / 256), dim3(256), 0, st, m, b, P, src);
    hipLaunchKernelGGL(k_mut_eval, dim3(1024), dim3(256), 0, st, m, op, b, P);
    if (op == RG_OR || op == RG_XOR) hipLaunchKernelGGL(k_mut_insert, dim3(512), dim3(256), 0, st, m, b, P);
}

// ------------------------------------------------------------------ batches
// Positions t < bbase[n] of a batch enumerate (operation i, key j of its B
// operand): t - bbase[i] is j's position in P[src[i]]'s keys.
__device__ __forceinline__ uint32_t batch_op_of(const MutBatch& bt, const uint64_t* bbase, uint64_t t) {
    uint32_t lo = 0, hi = bt.n - 1;  // last i with bbase[i] <= t
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (bbase[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void k_mutb_prep(MutView m, MutBatch bt, rg_pool P) {
    __shared__ uint64_t cnt[MUT_BATCH_MAX];
    const uint32_t i = threadIdx.x;
    if (i < bt.n) cnt[i] = P.bm_begin[bt.src[i] + 1] - P.bm_begin[bt.src[i]];
    __syncthreads();
    if (i == 0) {
        uint64_t o = 0;
        for (uint32_t q = 0; q < bt.n; ++q) {
            m.bbase[q] = o;
            o += cnt[q];
        }
        m.bbase[bt.n] = o;
        m.ctl[2] = 0;
        m.ctl[3] = 0;
    }
}

// per (operation, key of B): whether A lacks the key (a bit in tbits, one
// 64-bit word per wave and round), and the keys unions and symmetric
// differences will insert (one atomic per wave)
__global__ void __launch_bounds__(256) k_mutb_classify(MutView m, MutBatch bt, rg_pool P) {
    const uint32_t lane = lane_id();
    const uint64_t total = m.bbase[bt.n];
    const uint64_t step = (uint64_t)gridDim.x * 4 * 64;
    for (uint64_t t0 = (uint64_t)wave_index() * 64; t0 < total; t0 += step) {
        const uint64_t t = t0 + lane;
        bool absent = false, ins = false;
        if (t < total) {
            const uint32_t i = batch_op_of(bt, m.bbase, t);
            const uint64_t j = P.bm_begin[bt.src[i]] + (t - m.bbase[i]);
            absent = m.dir[(uint64_t)bt.b[i] * MUT_KEYS + P.keys[j]] == NONE;
            ins = absent && (bt.op[i] == RG_OR || bt.op[i] == RG_XOR);
        }
        const uint64_t word = __ballot(absent);
        const uint64_t ni = __popcll(__ballot(ins));
        if (lane == 0) {
            m.tbits[t0 >> 6] = word;
            if (ni) atomicAdd(&m.ctl[2], (int32_t)ni);
        }
    }
}

// the batch's insertions must fit the free slots, else the batch is skipped
__global__ void k_mutb_check(MutView m) {
    if (m.ctl[2] > m.ctl[0]) {
        m.ctl[3] = 1;
        m.ctl[1] = 1;
    }
}

// intersections: A's keys that B lacks become empty (blockIdx.y: the operation)
__global__ void k_mutb_drop(MutView m, MutBatch bt, rg_pool P) {
    __shared__ unsigned long long sum;
    const uint32_t i = blockIdx.y;
    if (bt.op[i] != RG_AND || uniform((uint32_t)m.ctl[3])) return;
    if (threadIdx.x == 0) sum = 0;
    __syncthreads();
    const uint32_t b = bt.b[i], key = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t* dir = m.dir + (uint64_t)b * MUT_KEYS;
    const uint32_t slot = dir[key];
    if (slot != NONE) {
        uint64_t lo = P.bm_begin[bt.src[i]], hi = P.bm_begin[bt.src[i] + 1];
        const uint64_t e = hi;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (P.keys[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        if (lo == e || P.keys[lo] != key) {
            atomicAdd(&sum, (unsigned long long)m.s_card[slot]);
            m.s_card[slot] = 0;
            dir[key] = NONE;
            mut_free(m, slot);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) add_card(m, b, -(long long)sum);
}

// keys A held before the batch: one workgroup each
__global__ void __launch_bounds__(256) k_mutb_eval(MutView m, MutBatch bt, rg_pool P) {
    __shared__ WgShared sh;
    if (uniform((uint32_t)m.ctl[3])) return;
    const uint64_t total = uniform64(m.bbase[bt.n]);
    for (uint64_t t = blockIdx.x; t < total; t += gridDim.x) {
        if ((m.tbits[t >> 6] >> (t & 63)) & 1ull) continue;  // absent before the batch
        const uint32_t i = uniform(batch_op_of(bt, m.bbase, t));
        const uint32_t j = uniform((uint32_t)(P.bm_begin[bt.src[i]] + (t - m.bbase[i])));
        const uint32_t slot = uniform(m.dir[(uint64_t)bt.b[i] * MUT_KEYS + P.keys[j]]);
        mut_eval_one(m, bt.op[i], bt.b[i], P, j, slot, sh);
    }
}

// keys A lacked before the batch (unions, symmetric differences): one wave each
__global__ void __launch_bounds__(256) k_mutb_insert(MutView m, MutBatch bt, rg_pool P) {
    const uint32_t lane = lane_id();
    if (uniform((uint32_t)m.ctl[3])) return;
    const uint64_t total = uniform64(m.bbase[bt.n]);
    const uint64_t nwaves = (uint64_t)gridDim.x * 4;
    for (uint64_t t = wave_index(); t < total; t += nwaves) {
        if (!((m.tbits[t >> 6] >> (t & 63)) & 1ull)) continue;
        const uint32_t i = uniform(batch_op_of(bt, m.bbase, t));
        if (bt.op[i] != RG_OR && bt.op[i] != RG_XOR) continue;
        mut_insert_one(m, bt.b[i], P, uniform((uint32_t)(P.bm_begin[bt.src[i]] + (t - m.bbase[i]))), lane);
    }
}

void launch_mut_batch(const MutView& m, const MutBatch& bt, const rg_pool& P, hipStream_t st) {
    if (!bt.n) return;
    bool any_and = false;
    for (uint32_t i = 0; i < bt.n; ++i) any_and |= bt.op[i] == RG_AND;
    hipLaunchKernelGGL(k_mutb_prep, dim3(1), dim3(MUT_BATCH_MAX), 0, st, m, bt, P);
    hipLaunchKernelGGL(k_mutb_classify, dim3(1024), dim3(256), 0, st, m, bt, P);
    hipLaunchKernelGGL(k_mutb_check, dim3(1), dim3(1), 0, st, m);
    if (any_and) hipLaunchKernelGGL(k_mutb_drop, dim3(MUT_KEYS / 256, bt.n), dim3(256), 0, st, m, bt, P);
    hipLaunchKernelGGL(k_mutb_eval, dim3(2048), dim3(256), 0, st, m, bt, P);
    hipLaunchKernelGGL(k_mutb_insert, dim3(1024), dim3(256), 0, st, m, bt, P);
}

// ------------------------------------------------------------------ clear
__global__ void k_mut_clear(MutView m, uint32_t b) {
    const uint32_t key = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t* dir = m.dir + (uint64_t)b * MUT_KEYS;
    if (key == 0) m.bm_card[b] = 0;
    if (key >= MUT_KEYS) return;
    const uint32_t slot = dir[key];
    if (slot == NONE) return;
    m.s_card[slot] = 0;
    dir[key] = NONE;
    mut_free(m, slot);
}

void launch_mut_clear(const MutView& m, uint32_t b, hipStream_t st) {
    hipLaunchKernelGGL(k_mut_clear, dim3(MUT_KEYS / 256), dim3(256), 0, st, m, b);
}

// ------------------------------------------------------------------ export
__device__ __forceinline__ uint32_t slot_bytes(const MutView& m, uint32_t slot) {
    return (payload_bytes_of(m.s_type[slot], m.s_size[slot]) + 15u) & ~15u;
}

__global__ void __launch_bounds__(256) k_mut_measure(MutView m, uint32_t b0, uint64_t* cnt, uint64_t* bytes) {
    __shared__ uint64_t tmp[4];
    const uint32_t* dir = m.dir + (uint64_t)(b0 + blockIdx.x) * MUT_KEYS;
    uint64_t c = 0, by = 0;
    for (uint32_t k = threadIdx.x; k < MUT_KEYS; k += 256) {
        const uint32_t slot = dir[k];
        if (slot != NONE) {
            ++c;
            by += slot_bytes(m, slot);
        }
    }
    c = block_sum_u64(c, tmp);
    by = block_sum_u64(by, tmp);
    if (threadIdx.x == 0) {
        cnt[blockIdx.x] = c;
        bytes[blockIdx.x] = by;
    }
}

void launch_mut_measure(const MutView& m, uint32_t b0, uint32_t n, uint64_t* cnt, uint64_t* bytes, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_mut_measure, dim3(n), dim3(256), 0, st, m, b0, cnt, bytes);
}

// one workgroup per bitmap: its keys in ascending order, 256 at a time
__global__ void __launch_bounds__(256) k_mut_write(MutView m, uint32_t b0, uint32_t n, const uint64_t* cbase,
                                                   const uint64_t* pbase, uint32_t* src_slot, rg_out out) {
    __shared__ uint32_t tmp[8];
    __shared__ uint64_t tmp64[4];
    const uint32_t j = blockIdx.x, b = b0 + j;
    const uint32_t* dir = m.dir + (uint64_t)b * MUT_KEYS;
    uint64_t ci = cbase[j], po = pbase[j], wb = 0;
    for (uint32_t k0 = 0; k0 < MUT_KEYS; k0 += 256) {
        const uint32_t key = k0 + threadIdx.x;
        const uint32_t slot = dir[key];
        const uint32_t here = slot != NONE ? 1u : 0u;
        const uint32_t nb = here ? slot_bytes(m, slot) : 0u;
        uint32_t tc, tb;
        const uint32_t pos = block_excl_scan_u32(here, tmp, &tc);
        const uint32_t bpos = block_excl_scan_u32(nb, tmp, &tb);
        if (here) {
            const uint64_t i = ci + pos;
            const uint32_t card = m.s_card[slot];
            out.keys[i] = (uint16_t)key;
            out.types[i] = m.s_type[slot];
            out.card[i] = card;
            out.size[i] = m.s_size[slot];
            out.off[i] = po + bpos;
            src_slot[i] = slot;
            wb += wbytes_of(card);
        }
        ci += tc;
        po += tb;
    }
    wb = block_sum_u64(wb, tmp64);
    if (threadIdx.x == 0) {
        out.bm_begin[j] = cbase[j];
        if (j + 1 == n) out.bm_begin[n] = ci;
        out.bm_card[j] = m.bm_card[b];
        if (out.bm_wbytes) out.bm_wbytes[j] = wb;
    }
}

__global__ void __launch_bounds__(256) k_mut_copy(MutView m, uint64_t n_out, const uint32_t* src_slot, rg_out out) {
    const uint32_t lane = lane_id();
    const uint64_t nwaves = (uint64_t)gridDim.x * 4;
    for (uint64_t i = wave_index(); i < n_out; i += nwaves) {
        const uint32_t slot = uniform(src_slot[i]);
        const uint32_t units = slot_bytes(m, slot) / 16;
        const u32x4* s4 = reinterpret_cast<const u32x4*>(m.slab + (uint64_t)slot * MUT_SLOT_BYTES);
        u32x4* d4 = reinterpret_cast<u32x4*>(out.payload + uniform64(out.off[i]));
        for (uint32_t u = lane; u < units; u += 64) d4[u] = s4[u];
    }
}

void launch_mut_export(const MutView& m, uint32_t b0, uint32_t n, const uint64_t* cbase, const uint64_t* pbase,
                       uint64_t n_out, uint32_t* src_slot, const rg_out& out, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_mut_write, dim3(n), dim3(256), 0, st, m, b0, n, cbase, pbase, src_slot, out);
    if (n_out) {
        uint64_t g = (n_out + 3) / 4;
        if (g > 65536) g = 65536;
        hipLaunchKernelGGL(k_mut_copy, dim3((uint32_t)g), dim3(256), 0, st, m, n_out, src_slot, out);
    }
}

}  // namespace rg
