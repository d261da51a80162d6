// rg_bitset.hip - bitset op bitset with fused population count (Section 4.1.2)
// and the on-the-fly output-type decision for the result (Section 1).
//
// One wave64 per container pair. Each lane loads 8 x 16 bytes from each
// input (coalesced dwordx4, 8 KiB per input per wave), combines the words in
// registers and counts them with the native per-lane popcount; the 64 lane
// counts are summed across the wave. The count-only form stops there (16 KiB
// read, 8 bytes of atomic add). The materialising form also counts the runs
// of the result, decides the P1 type, and writes the result from registers:
// the 8 KiB bitset as it is; an array by extracting the set bits (Section
// 3.1: each lane's values go after the values of the words before its own,
// a prefix sum over the lanes per step); runs from the run-start and run-end
// masks, staged in LDS so that each run's start and end meet.
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

// Result words of one bitset pair in registers (see the word order above),
// with their population count c and run count r summed over the wave. A side
// given as nullptr is absent (all words zero).
struct BbWords {
    uint64_t lo[8], hi[8];
    uint32_t c, r;
};

__device__ __forceinline__ uint64_t bb_op(int op, uint64_t x, uint64_t y) {
    return op == RG_AND ? (x & y) : op == RG_OR ? (x | y) : op == RG_XOR ? (x ^ y) : (x & ~y);
}

__device__ __forceinline__ void bb_count(BbWords& w, uint32_t lane);

// the lane's 16 words of a bitset container (zeros for an absent one)
__device__ __forceinline__ void bb_load(const u32x4* p, uint32_t lane, u32x4 (&x)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = p ? __builtin_nontemporal_load(p + k * 64 + lane) : u32x4{0, 0, 0, 0};
}

// A's words already loaded (x), B's loaded here, combined by op
__device__ __forceinline__ void bb_words_x(int op, const u32x4 (&x)[8], const u32x4* pb, uint32_t lane,
                                           BbWords& w) {
    u32x4 y[8];
    bb_load(pb, lane, y);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint64_t xa = (uint64_t)x[k].x | ((uint64_t)x[k].y << 32);
        const uint64_t xb = (uint64_t)x[k].z | ((uint64_t)x[k].w << 32);
        const uint64_t ya = (uint64_t)y[k].x | ((uint64_t)y[k].y << 32);
        const uint64_t yb = (uint64_t)y[k].z | ((uint64_t)y[k].w << 32);
        w.lo[k] = bb_op(op, xa, ya);
        w.hi[k] = bb_op(op, xb, yb);
    }
    bb_count(w, lane);
}

__device__ __forceinline__ void bb_words(int op, const u32x4* pa, const u32x4* pb, uint32_t lane, BbWords& w) {
    u32x4 x[8];
    bb_load(pa, lane, x);
    bb_words_x(op, x, pb, lane, w);
}

// The result's cardinality w.c and run count w.r from the words in registers
// (lane l holds words 128k + 2l and 128k + 2l + 1 of the bitset in lo[k], hi[k]).
__device__ __forceinline__ void bb_count(BbWords& w, uint32_t lane) {
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) c += __popcll(w.lo[k]) + __popcll(w.hi[k]);
    // run starts: bit set and the bit below it (previous word's MSB for bit 0) clear
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint64_t prev = __shfl_up(w.hi[k], 1);
        const uint64_t wrap = k > 0 ? __shfl(w.hi[k > 0 ? k - 1 : 0], 63) : 0ull;
        if (lane == 0) prev = wrap;
        const uint64_t s_lo = w.lo[k] & ~((w.lo[k] << 1) | (prev >> 63));
        const uint64_t s_hi = w.hi[k] & ~((w.hi[k] << 1) | (w.lo[k] >> 63));
        r += __popcll(s_lo) + __popcll(s_hi);
    }
    const uint64_t cr = wave_sum_u64((uint64_t)c | ((uint64_t)r << 32));
    w.c = (uint32_t)cr;
    w.r = (uint32_t)(cr >> 32);
}

// writes the result words as an 8 KiB bitset container
__device__ __forceinline__ void bb_store(const BbWords& w, uint8_t* dst8, uint32_t lane) {
    u32x4* dst = reinterpret_cast<u32x4*>(dst8);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        u32x4 v;
        v.x = (uint32_t)w.lo[k];
        v.y = (uint32_t)(w.lo[k] >> 32);
        v.z = (uint32_t)w.hi[k];
        v.w = (uint32_t)(w.hi[k] >> 32);
        __builtin_nontemporal_store(v, dst + k * 64 + lane);
    }
}

// exclusive prefix sum over the lanes, and the total
__device__ __forceinline__ uint32_t bb_excl_sum(uint32_t v, uint32_t& total) {
    const uint32_t incl = wave_incl_scan_u32(v);
    total = uniform(__shfl(incl, 63));
    return incl - v;
}

// writes the set bits of the word pair (x0, x1) = words wi, wi + 1 as 16-bit
// values from position pos on
__device__ __forceinline__ void bb_extract(uint64_t x0, uint64_t x1, uint32_t wi, uint16_t* d16, uint32_t pos) {
    while (x0) {
        d16[pos++] = (uint16_t)(wi * 64 + __builtin_ctzll(x0));
        x0 &= x0 - 1;
    }
    while (x1) {
        d16[pos++] = (uint16_t)((wi + 1) * 64 + __builtin_ctzll(x1));
        x1 &= x1 - 1;
    }
}

// Writes the result words as an array container (type RG_ARRAY, c <= 4096
// values) or run container (RG_RUN, r <= 2048 runs) at dst. lds: this wave's
// 2 x 2048 16-bit entries (run starts, run ends).
__device__ void bb_store_sparse(const BbWords& w, uint8_t type, uint8_t* dst, uint16_t* lds, uint32_t lane) {
    uint16_t* d16 = reinterpret_cast<uint16_t*>(dst);
    if (type == RG_ARRAY) {
        uint32_t base = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            uint32_t tot;
            const uint32_t pre = bb_excl_sum(__popcll(w.lo[k]) + __popcll(w.hi[k]), tot);
            bb_extract(w.lo[k], w.hi[k], 128 * k + 2 * lane, d16, base + pre);
            base += tot;
        }
        return;
    }
    // run starts: bit set, the bit below clear; run ends: bit set, the bit above clear
    uint16_t* ls = lds;
    uint16_t* le = lds + 2048;
    uint32_t bs = 0, be = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint64_t prev = __shfl_up(w.hi[k], 1);
        const uint64_t wrap = k > 0 ? __shfl(w.hi[k > 0 ? k - 1 : 0], 63) : 0ull;
        if (lane == 0) prev = wrap;
        uint64_t next = __shfl_down(w.lo[k], 1);
        const uint64_t wrap_n = k < 7 ? __shfl(w.lo[k < 7 ? k + 1 : 7], 0) : 0ull;
        if (lane == 63) next = wrap_n;
        const uint64_t st_lo = w.lo[k] & ~((w.lo[k] << 1) | (prev >> 63));
        const uint64_t st_hi = w.hi[k] & ~((w.hi[k] << 1) | (w.lo[k] >> 63));
        const uint64_t en_lo = w.lo[k] & ~((w.lo[k] >> 1) | (w.hi[k] << 63));
        const uint64_t en_hi = w.hi[k] & ~((w.hi[k] >> 1) | (next << 63));
        uint32_t ts, te;
        const uint32_t ps = bb_excl_sum(__popcll(st_lo) + __popcll(st_hi), ts);
        const uint32_t pe = bb_excl_sum(__popcll(en_lo) + __popcll(en_hi), te);
        bb_extract(st_lo, st_hi, 128 * k + 2 * lane, ls, bs + ps);
        bb_extract(en_lo, en_hi, 128 * k + 2 * lane, le, be + pe);
        bs += ts;
        be += te;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
    for (uint32_t i = lane; i < bs; i += 64) d32[i] = (uint32_t)ls[i] | ((uint32_t)(le[i] - ls[i]) << 16);
    __builtin_amdgcn_wave_barrier();  // the LDS is read before the wave's next result
}

// Writes a non-empty result of the words in P1 form into slot `slot` (bitset
// from registers, array or runs through bb_store_sparse) and records it;
// false (nothing written, *err bit 2) when it would end past the arena.
__device__ bool bb_store_result(const BbWords& w, uint32_t slot, const SlotOut& so, uint16_t* lds, uint32_t lane) {
    const uint8_t type = p1_type(w.c, w.r);
    const uint64_t nbytes = type == RG_ARRAY ? 2ull * w.c : type == RG_BITSET ? 8192ull : 4ull * w.r;
    const uint64_t soff = so.slot_off[slot];
    if (soff + nbytes > so.cap) {
        if (lane == 0 && so.err) atomicOr(so.err, 2u);
        return false;
    }
    if (type == RG_BITSET) bb_store(w, so.payload + soff, lane);
    else bb_store_sparse(w, type, so.payload + soff, lds, lane);
    if (lane == 0) {
        so.res_card[slot] = w.c;
        so.res_type[slot] = type;
        so.res_size[slot] = type == RG_ARRAY ? w.c : type == RG_BITSET ? 1024u : w.r;
    }
    return true;
}

// Materialising form (intersection): words in registers, run count, P1 type,
// the result written from registers.
__global__ void __launch_bounds__(256) k_bb_mat(ComputeArgs a) {
    __shared__ uint16_t lds[4][4096];
    const uint32_t lane = lane_id();
    const uint32_t wv = wave_index();
    if (wv >= a.n) return;
    const uint32_t slot = uniform(a.list[wv]);
    const Task t = uniform_task(a.tasks, slot);
    BbWords w;
    bb_words(a.op, reinterpret_cast<const u32x4*>(a.A.payload + a.A.off[t.ia]),
             reinterpret_cast<const u32x4*>(a.B.payload + a.B.off[t.ib]), lane, w);
    if (w.c == 0) return;  // empty result: slot stays empty
    bb_store_result(w, slot, a.so, lds[threadIdx.x >> 6], lane);
}

// k-way slots marked KW_TASK_BB (queries of one or two bitmaps whose
// containers at the key are bitsets, or a bitset and nothing), BB_CHUNK slots
// per wave: lane i loads slot i's task, op and payload offsets in parallel,
// then the wave builds the slots' results one after another as k_bb_mat
// does, in any P1 form, and marks each task KW_TASK_DONE.
constexpr uint32_t BB_CHUNK = 8;

__global__ void __launch_bounds__(256) k_kw_bb(KwArgs a) {
    __shared__ uint16_t lds[4][4096];
    const uint32_t lane = lane_id();
    const uint64_t step = (uint64_t)gridDim.x * 4 * BB_CHUNK;
    for (uint64_t c0 = (uint64_t)wave_index() * BB_CHUNK; c0 < a.n_slots; c0 += step) {
        bool mine = false;
        uint32_t op = 0, has = 0;
        uint64_t oa = 0, ob = 0;
        if (lane < BB_CHUNK && c0 + lane < a.n_slots) {
            const Task t = a.tasks[c0 + lane];
            mine = t.kind == KIND_MATCH && t.bin == KW_TASK_BB;
            if (mine) {
                op = a.queries[t.pair - a.pair_base].op;
                has = (t.ia != NONE ? 1u : 0u) | (t.ib != NONE ? 2u : 0u);
                if (t.ia != NONE) oa = a.P0.off[t.ia];
                if (t.ib != NONE) ob = a.P1.off[t.ib];
            }
        }
        uint64_t m = __ballot(mine);
        // software pipeline: the next slot's A-side words are loaded while the
        // current slot's result is built and written
        auto a_words = [&](uint32_t l) {
            const uint32_t hl = __builtin_amdgcn_readlane(has, l);
            return (hl & 1u) ? reinterpret_cast<const u32x4*>(a.P0.payload + readlane64(oa, l)) : nullptr;
        };
        u32x4 xn[8];
        uint32_t ln = m ? (uint32_t)__builtin_ctzll(m) : 0u;
        if (m) bb_load(a_words(ln), lane, xn);
        while (m) {
            const uint32_t l = ln;
            m &= m - 1;
            u32x4 x[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = xn[k];
            if (m) {
                ln = (uint32_t)__builtin_ctzll(m);
                bb_load(a_words(ln), lane, xn);
            }
            const uint32_t slot = (uint32_t)(c0 + l);
            const uint32_t hl = __builtin_amdgcn_readlane(has, l);
            const u32x4* pb = (hl & 2u) ? reinterpret_cast<const u32x4*>(a.P1.payload + readlane64(ob, l)) : nullptr;
            BbWords w;
            bb_words_x((int)__builtin_amdgcn_readlane(op, l), x, pb, lane, w);
            if (w.c) bb_store_result(w, slot, a.so, lds[threadIdx.x >> 6], lane);
            if (lane == 0) a.tasks[slot].bin = KW_TASK_DONE;
        }
    }
}

// Unions and symmetric differences of more than two bitmaps (k <= 64 per
// result key, slots marked KW_TASK_WAVE by the bounds kernel), one wave per
// result key: lane j finds the key's container in bitmap j (presence bit and
// rank, or binary search); bitset containers are combined in registers, two at
// a time with all their loads in flight; the values and runs of array and run
// containers are set (union) or flipped (symmetric difference) in the wave's
// 8 KiB LDS bitset, WAVE_UNROLL units per lane per round, each lane finding
// its unit's container by a search over the lanes' unit offsets. The LDS words
// then join the register words, and the P1 result is written from registers
// (bb_store_result) or, count-only, its cardinality added to the query's.
// Against the workgroup kernel: no block barriers, and four keys per
// workgroup's LDS instead of one.
constexpr uint32_t WAVE_CHUNK = 8;  // most slots whose tasks a wave reads at once
constexpr int WAVE_UNROLL = 4;

// exclusive prefix sum over the wave's lanes, and the total
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
    const uint32_t incl = wave_incl_scan_u32(v);
    total = uniform((uint32_t)__shfl((int)incl, 63));
    return incl - v;
}

// lane j's 64-bit value, j chosen per lane
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, uint32_t j) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, (int)j);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), (int)j);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__global__ void __launch_bounds__(256) k_kw_wave(KwArgs a, uint32_t chunk) {
    __shared__ uint64_t bits[4][1024];
    const uint32_t lane = lane_id();
    uint64_t* L = bits[threadIdx.x >> 6];
    const uint64_t step = (uint64_t)gridDim.x * 4 * chunk;
    for (uint64_t c0 = (uint64_t)wave_index() * chunk; c0 < a.n_slots; c0 += step) {
        bool mine = false;
        uint32_t pair = 0, key = 0;
        if (lane < chunk && c0 + lane < a.n_slots) {
            const Task t = a.tasks[c0 + lane];
            mine = t.kind == KIND_MATCH && t.bin == KW_TASK_WAVE;
            pair = t.pair;
            key = t.key;
        }
        uint64_t m = __ballot(mine);
        while (m) {
            const uint32_t l = (uint32_t)__builtin_ctzll(m);
            m &= m - 1;
            const uint32_t slot = (uint32_t)(c0 + l);
            const uint32_t q = __builtin_amdgcn_readlane(pair, l) - a.pair_base;
            const uint16_t kk = (uint16_t)__builtin_amdgcn_readlane(key, l);
            const KwQuery& Q = a.queries[q];
            const uint32_t op = uniform(Q.op), k = uniform(Q.k), ids0 = uniform(Q.ids_off);
            const bool mat = (uniform(Q.flags) & KW_MATERIALIZE) != 0;
            const bool xr = op == RG_XOR;
            // lane j: the key's container in bitmap j
            uint32_t ty = 0, sz = 0;
            uint64_t off = 0;
            if (lane < k) {
                const bool second = lane != 0;
                const uint32_t ci = kw_find_key(second ? a.P1.bm_begin : a.P0.bm_begin, second ? a.P1.keys : a.P0.keys,
                                                second ? a.P1.kidx : a.P0.kidx, a.ids[ids0 + lane], kk);
                if (ci != NONE) {
                    ty = second ? a.P1.types[ci] : a.P0.types[ci];
                    sz = second ? a.P1.size[ci] : a.P0.size[ci];
                    // the payload's address
                    off = reinterpret_cast<uint64_t>((second ? a.P1.payload : a.P0.payload) +
                                                     (second ? a.P1.off[ci] : a.P0.off[ci]));
                }
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) L[lane + 64 * i] = 0;
            // bitsets, combined in registers
            BbWords w;
#pragma unroll
            for (int i = 0; i < 8; ++i) w.lo[i] = w.hi[i] = 0;
            uint64_t bm = __ballot(ty == RG_BITSET);
            while (bm) {
                const uint32_t j0 = (uint32_t)__builtin_ctzll(bm);
                bm &= bm - 1;
                const bool two = bm != 0;
                const uint32_t j1 = two ? (uint32_t)__builtin_ctzll(bm) : j0;
                if (two) bm &= bm - 1;
                const u32x4* p0 = reinterpret_cast<const u32x4*>(readlane64(off, j0));
                const u32x4* p1 = reinterpret_cast<const u32x4*>(readlane64(off, j1));
                u32x4 x[8], y[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    x[i] = __builtin_nontemporal_load(p0 + i * 64 + lane);
                    y[i] = two ? __builtin_nontemporal_load(p1 + i * 64 + lane) : u32x4{0, 0, 0, 0};
                }
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const uint64_t xa = (uint64_t)x[i].x | ((uint64_t)x[i].y << 32);
                    const uint64_t xb = (uint64_t)x[i].z | ((uint64_t)x[i].w << 32);
                    const uint64_t ya = (uint64_t)y[i].x | ((uint64_t)y[i].y << 32);
                    const uint64_t yb = (uint64_t)y[i].z | ((uint64_t)y[i].w << 32);
                    w.lo[i] = xr ? (w.lo[i] ^ xa ^ ya) : (w.lo[i] | xa | ya);
                    w.hi[i] = xr ? (w.hi[i] ^ xb ^ yb) : (w.hi[i] | xb | yb);
                }
            }
            // array values and runs, into the LDS bitset
            const uint32_t units = (ty == RG_ARRAY || ty == RG_RUN) ? sz : 0u;
            uint32_t total;
            const uint32_t upos = wave_excl_scan(units, total);
            __builtin_amdgcn_wave_barrier();  // the LDS bitset is cleared
            for (uint32_t base = 0; base < total; base += 64 * WAVE_UNROLL) {
                uint32_t raw[WAVE_UNROLL];
                bool run[WAVE_UNROLL], live[WAVE_UNROLL];
#pragma unroll
                for (int r = 0; r < WAVE_UNROLL; ++r) {
                    const uint32_t u = base + r * 64 + lane;
                    // the unit's container: the last lane whose offset is <= u
                    uint32_t j = 0;
#pragma unroll
                    for (uint32_t sstep = 32; sstep; sstep >>= 1)
                        if ((uint32_t)__shfl((int)upos, (int)(j + sstep)) <= u) j += sstep;
                    const uint32_t tj = (uint32_t)__shfl((int)ty, (int)j);
                    const uint64_t oj = shfl_u64(off, j);
                    const uint32_t loc = u - (uint32_t)__shfl((int)upos, (int)j);
                    live[r] = u < total;
                    run[r] = tj == RG_RUN;
                    raw[r] = 0;
                    if (live[r]) {
                        const uint8_t* pl = reinterpret_cast<const uint8_t*>(oj);
                        raw[r] = run[r] ? reinterpret_cast<const uint32_t*>(pl)[loc]
                                        : (uint32_t)reinterpret_cast<const uint16_t*>(pl)[loc];
                    }
                }
#pragma unroll
                for (int r = 0; r < WAVE_UNROLL; ++r) {
                    if (!live[r]) continue;
                    if (!run[r]) {
                        unsigned long long* dst = reinterpret_cast<unsigned long long*>(&L[raw[r] >> 6]);
                        const unsigned long long bit = 1ull << (raw[r] & 63);
                        if (xr) atomicXor(dst, bit);
                        else atomicOr(dst, bit);
                    } else {
                        // (a run past the chunk's end in a malformed pool stops at its end)
                        const uint32_t first = raw[r] & 0xFFFFu, end = first + (raw[r] >> 16);
                        const uint32_t last = end < 65535u ? end : 65535u;
                        for (uint32_t wi = first >> 6; wi <= last >> 6; ++wi) {
                            const uint32_t lo = wi == first >> 6 ? first & 63 : 0;
                            const uint32_t hi = wi == last >> 6 ? last & 63 : 63;
                            const unsigned long long mask = (~0ull << lo) & (~0ull >> (63 - hi));
                            unsigned long long* dst = reinterpret_cast<unsigned long long*>(&L[wi]);
                            if (xr) atomicXor(dst, mask);
                            else atomicOr(dst, mask);
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();  // every unit is in the LDS bitset
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint64_t la = L[2 * (i * 64 + lane)], lb = L[2 * (i * 64 + lane) + 1];
                w.lo[i] = xr ? (w.lo[i] ^ la) : (w.lo[i] | la);
                w.hi[i] = xr ? (w.hi[i] ^ lb) : (w.hi[i] | lb);
            }
            __builtin_amdgcn_wave_barrier();  // the LDS is read before the output step reuses it
            bb_count(w, lane);
            if (mat) {
                if (w.c) bb_store_result(w, slot, a.so, reinterpret_cast<uint16_t*>(L), lane);
            } else if (lane == 0 && w.c) {
                atomicAdd(reinterpret_cast<unsigned long long*>(&a.acc[q]), (unsigned long long)w.c);
            }
            if (lane == 0) a.tasks[slot].bin = KW_TASK_DONE;
            __builtin_amdgcn_wave_barrier();  // the LDS is free for the next key
        }
    }
}

void launch_kw_wave(const KwArgs& a, hipStream_t st) {
    if (!a.n_slots || !a.wave) return;
    // a wave's slots are built one after another: as many per wave as it
    // takes to give every resident wave (about 3072) work, at most WAVE_CHUNK
    uint64_t chunk = a.n_slots / 3072;
    chunk = chunk < 1 ? 1 : chunk > WAVE_CHUNK ? WAVE_CHUNK : chunk;
    const uint64_t g = (a.n_slots + 4 * chunk - 1) / (4 * chunk);
    hipLaunchKernelGGL(k_kw_wave, dim3(g < 16384 ? (uint32_t)g : 16384u), dim3(256), 0, st, a, (uint32_t)chunk);
}

void launch_kw_bb(const KwArgs& a, hipStream_t st) {
    if (!a.n_slots || !a.small) return;
    const uint64_t g = (a.n_slots + 4 * BB_CHUNK - 1) / (4 * BB_CHUNK);
    hipLaunchKernelGGL(k_kw_bb, dim3(g < 16384 ? (uint32_t)g : 16384u), dim3(256), 0, st, a);
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
        hipLaunchKernelGGL(k_bb_mat, grid, dim3(256), 0, st, a);
    }
}

}  // namespace rg
