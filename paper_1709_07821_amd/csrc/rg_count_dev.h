// rg_count_dev.h - per-pair count bodies shared by the per-bin kernels and the
// persistent work-stealing kernel. Each returns a value summed over the wave
// (or workgroup) that executes it.
#pragma once
#include "rg_finalize.h"

namespace rg {

// Count-only kernels add |A_k n B_k| of each matched container pair to the
// pair's accumulator; the requested cardinality is derived per pair at the end.
__device__ __forceinline__ void acc_add(long long* acc, uint32_t pair, long long d) {
    if (d) atomicAdd(reinterpret_cast<unsigned long long*>(&acc[pair]), (unsigned long long)d);
}

// ---------------------------------------------------------------- bitset pair
// |a op b| of two 1024-word bitsets by one wave: 8 x 16-byte loads per lane per
// input, coalesced; native popcount; wave sum (every lane gets the total).
template <int OP>
__device__ __forceinline__ uint32_t bb_count_wave(const PoolView& A, const PoolView& B, const Task& t,
                                                  uint32_t lane) {
    const u32x4* pa = reinterpret_cast<const u32x4*>(A.payload + uniform64(A.off[t.ia]));
    const u32x4* pb = reinterpret_cast<const u32x4*>(B.payload + uniform64(B.off[t.ib]));
    u32x4 x[8], y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        x[k] = __builtin_nontemporal_load(pa + k * 64 + lane);
        y[k] = __builtin_nontemporal_load(pb + k * 64 + lane);
    }
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        uint64_t xa = (uint64_t)x[k].x | ((uint64_t)x[k].y << 32);
        uint64_t xb = (uint64_t)x[k].z | ((uint64_t)x[k].w << 32);
        uint64_t ya = (uint64_t)y[k].x | ((uint64_t)y[k].y << 32);
        uint64_t yb = (uint64_t)y[k].z | ((uint64_t)y[k].w << 32);
        c += __popcll(apply_op<OP>(xa, ya)) + __popcll(apply_op<OP>(xb, yb));
    }
    return wave_sum_u32(c);
}

// ---------------------------------------------------------------- array / run pairs
struct CView {
    uint8_t type;
    uint32_t size;
    uint32_t card;
    const uint8_t* pl;
};

__device__ __forceinline__ CView cview(const PoolView& P, uint32_t idx) {
    CView v;
    v.type = (uint8_t)uniform(P.types[idx]);
    v.size = uniform(P.size[idx]);
    v.card = uniform(P.card[idx]);
    v.pl = P.payload + uniform64(P.off[idx]);
    return v;
}

__device__ __forceinline__ bool search_u16(const uint16_t* a, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && a[lo] == x;
}

// index of the last run with start <= x, or -1
__device__ __forceinline__ int last_run_start_le(const uint32_t* runs, uint32_t r, uint32_t x) {
    uint32_t lo = 0, hi = r;  // first run with start > x
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if ((runs[mid] & 0xFFFFu) <= x) lo = mid + 1;
        else hi = mid;
    }
    return (int)lo - 1;
}

__device__ __forceinline__ bool in_runs(const uint32_t* runs, uint32_t r, uint32_t x) {
    int k = last_run_start_le(runs, r, x);
    if (k < 0) return false;
    uint32_t pr = runs[k];
    return x <= (pr & 0xFFFFu) + (pr >> 16);
}

// |S n L| where S is an array container: each lane takes values of S and tests
// them against L (bit test for a bitset, binary search for an array or runs)
__device__ __forceinline__ uint32_t array_probe(const CView& s, const CView& l, uint32_t lane) {
    const uint16_t* sv = reinterpret_cast<const uint16_t*>(s.pl);
    uint32_t hits = 0;
    if (l.type == RG_BITSET) {
        const uint64_t* w = reinterpret_cast<const uint64_t*>(l.pl);
        for (uint32_t i = lane; i < s.size; i += 64) {
            uint32_t x = sv[i];
            hits += (uint32_t)(w[x >> 6] >> (x & 63)) & 1u;
        }
    } else if (l.type == RG_ARRAY) {
        const uint16_t* lv = reinterpret_cast<const uint16_t*>(l.pl);
        for (uint32_t i = lane; i < s.size; i += 64) hits += search_u16(lv, l.size, sv[i]) ? 1u : 0u;
    } else {
        const uint32_t* lr = reinterpret_cast<const uint32_t*>(l.pl);
        for (uint32_t i = lane; i < s.size; i += 64) hits += in_runs(lr, l.size, sv[i]) ? 1u : 0u;
    }
    return hits;
}

// |R n Q| for two run containers: each lane takes runs of R
__device__ __forceinline__ uint32_t run_run(const CView& R, const CView& Q, uint32_t lane) {
    const uint32_t* rr = reinterpret_cast<const uint32_t*>(R.pl);
    const uint32_t* qr = reinterpret_cast<const uint32_t*>(Q.pl);
    uint32_t inter = 0;
    for (uint32_t i = lane; i < R.size; i += 64) {
        uint32_t s = rr[i] & 0xFFFFu, e = s + (rr[i] >> 16);
        int k = last_run_start_le(qr, Q.size, s);
        uint32_t q = k < 0 ? 0u : (uint32_t)k;
        for (; q < Q.size; ++q) {
            uint32_t qs = qr[q] & 0xFFFFu, qe = qs + (qr[q] >> 16);
            if (qs > e) break;
            uint32_t lo = s > qs ? s : qs, hi = e < qe ? e : qe;
            if (lo <= hi) inter += hi - lo + 1;
        }
    }
    return inter;
}

// |R n W| for a run container and a bitset: popcount of the words under each run
__device__ __forceinline__ uint32_t run_bitset(const CView& R, const CView& B, uint32_t lane) {
    const uint32_t* rr = reinterpret_cast<const uint32_t*>(R.pl);
    const uint64_t* w = reinterpret_cast<const uint64_t*>(B.pl);
    uint32_t inter = 0;
    for (uint32_t i = lane; i < R.size; i += 64) {
        uint32_t s = rr[i] & 0xFFFFu, e = s + (rr[i] >> 16);
        uint32_t ws = s >> 6, we = e >> 6;
        for (uint32_t k = ws; k <= we; ++k) {
            uint64_t m = ~0ull;
            if (k == ws) m &= ~0ull << (s & 63);
            if (k == we) m &= ~0ull >> (63 - (e & 63));
            inter += __popcll(w[k] & m);
        }
    }
    return inter;
}

// |A n B| of one non-bitset-bitset pair by one wave (summed over the wave)
__device__ __forceinline__ uint32_t wave_inter(const PoolView& PA, const PoolView& PB, const Task& t,
                                               uint32_t lane) {
    const CView A = cview(PA, t.ia), B = cview(PB, t.ib);
    uint32_t inter;
    if (A.type == RG_ARRAY && (B.type != RG_ARRAY || A.size <= B.size)) inter = array_probe(A, B, lane);
    else if (B.type == RG_ARRAY) inter = array_probe(B, A, lane);
    else if (A.type == RG_RUN && B.type == RG_RUN)
        inter = A.size <= B.size ? run_run(A, B, lane) : run_run(B, A, lane);
    else if (A.type == RG_RUN) inter = run_bitset(A, B, lane);
    else inter = run_bitset(B, A, lane);
    return wave_sum_u32(inter);
}

// |A n B| of one pair by one thread: every value of the smaller array side is
// looked up in the other container (bit test, binary search in an array or
// in the run starts). For small array sides only. Per-lane values throughout.
// The form taking what the caller has read already: types, sizes (array:
// cardinality, run: run count; unused for a bitset) and payload addresses.
__device__ __forceinline__ uint32_t thread_inter_at(uint8_t ta, uint8_t tb, uint32_t sa, uint32_t sb,
                                                    const uint8_t* pa, const uint8_t* pb) {
    // s: the array side (the smaller one when both are arrays); l: the other
    const bool a_is_s = ta == RG_ARRAY && (tb != RG_ARRAY || sa <= sb);
    const uint16_t* sv = reinterpret_cast<const uint16_t*>(a_is_s ? pa : pb);
    const uint32_t n = a_is_s ? sa : sb;
    const uint8_t lt = a_is_s ? tb : ta;
    const uint32_t ln = a_is_s ? sb : sa;
    const uint8_t* lp = a_is_s ? pb : pa;
    uint32_t hits = 0;
    if (lt == RG_BITSET) {
        const uint64_t* w = reinterpret_cast<const uint64_t*>(lp);
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t x = sv[i];
            hits += (uint32_t)(w[x >> 6] >> (x & 63)) & 1u;
        }
    } else if (lt == RG_ARRAY) {
        const uint16_t* lv = reinterpret_cast<const uint16_t*>(lp);
        uint32_t lo = 0;  // values of s are increasing: each search starts where the last ended
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t x = sv[i];
            uint32_t hi = ln;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (lv[mid] < x) lo = mid + 1;
                else hi = mid;
            }
            if (lo < ln && lv[lo] == x) ++hits;
        }
    } else {
        const uint32_t* lr = reinterpret_cast<const uint32_t*>(lp);
        for (uint32_t i = 0; i < n; ++i) hits += in_runs(lr, ln, sv[i]) ? 1u : 0u;
    }
    return hits;
}

// The form taking two packed metadata records' contents (PoolView::meta):
// data is a payload offset, or the values of an array of at most
// META_INLINE_MAX values when its inline flag is set.
__device__ __forceinline__ uint32_t thread_inter_rec(uint8_t ta, uint8_t tb, uint32_t sa, uint32_t sb, bool ina,
                                                     bool inb, uint64_t da, uint64_t db, const uint8_t* payA,
                                                     const uint8_t* payB) {
    if (!ina && !inb) return thread_inter_at(ta, tb, sa, sb, payA + da, payB + db);
    const bool a_is_s = ta == RG_ARRAY && (tb != RG_ARRAY || sa <= sb);
    const uint32_t n = a_is_s ? sa : sb;
    const bool s_in = a_is_s ? ina : inb;
    const uint64_t s_data = a_is_s ? da : db;
    const uint16_t* sv = s_in ? nullptr : reinterpret_cast<const uint16_t*>((a_is_s ? payA : payB) + s_data);
    const uint8_t lt = a_is_s ? tb : ta;
    const uint32_t ln = a_is_s ? sb : sa;
    const bool l_in = a_is_s ? inb : ina;
    const uint64_t l_data = a_is_s ? db : da;
    const uint8_t* lp = l_in ? nullptr : (a_is_s ? payB : payA) + l_data;
    uint32_t hits = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t x = s_in ? (uint32_t)(s_data >> (16 * i)) & 0xFFFFu : sv[i];
        if (lt == RG_BITSET) {
            hits += (uint32_t)(reinterpret_cast<const uint64_t*>(lp)[x >> 6] >> (x & 63)) & 1u;
        } else if (lt == RG_ARRAY) {
            if (l_in) {
                for (uint32_t t = 0; t < ln; ++t) hits += ((uint32_t)(l_data >> (16 * t)) & 0xFFFFu) == x ? 1u : 0u;
            } else {
                hits += search_u16(reinterpret_cast<const uint16_t*>(lp), ln, x) ? 1u : 0u;
            }
        } else {
            hits += in_runs(reinterpret_cast<const uint32_t*>(lp), ln, x) ? 1u : 0u;
        }
    }
    return hits;
}

// The container types are passed in when the caller has read them already.
__device__ __forceinline__ uint32_t thread_inter_typed(const PoolView& PA, const PoolView& PB, uint32_t ia,
                                                       uint32_t ib, uint8_t ta, uint8_t tb) {
    return thread_inter_at(ta, tb, PA.size[ia], PB.size[ib], PA.payload + PA.off[ia], PB.payload + PB.off[ib]);
}

__device__ __forceinline__ uint32_t thread_inter(const PoolView& PA, const PoolView& PB, const Task& t) {
    return thread_inter_typed(PA, PB, t.ia, t.ib, PA.types[t.ia], PB.types[t.ib]);
}

// Adds each lane's value v to acc[pair] (lanes with pair == NONE add nothing)
// with one atomic per distinct pair in the wave: neighbouring items mostly
// belong to the same pair. Call with the whole wave active.
__device__ __forceinline__ void wave_aggregate_add(long long* acc, uint32_t pair, uint32_t v) {
    const uint32_t lane = lane_id();
    uint64_t pending = __ballot(pair != NONE);
    while (pending) {
        const uint32_t leader = (uint32_t)__builtin_ctzll(pending);
        const uint32_t p = __builtin_amdgcn_readlane(pair, leader);
        const bool mine = pair == p;
        const uint64_t m = __ballot(mine);
        const uint32_t s = wave_sum_u32(mine ? v : 0u);
        if (lane == leader && s) atomicAdd(reinterpret_cast<unsigned long long*>(&acc[p]), (unsigned long long)s);
        pending &= ~m;
    }
}

// |A n B| of two array containers by a 256-thread workgroup: both arrays staged
// in LDS, merge path split of the merged sequence over the threads; a B value
// equal to the A value merged just before it is a match. Contains barriers.
__device__ __forceinline__ uint32_t merge_inter_wg(const PoolView& PA, const PoolView& PB, const Task& t,
                                                   uint16_t* sA, uint16_t* sB, uint64_t* tmp64) {
    const CView A = cview(PA, t.ia), B = cview(PB, t.ib);
    const uint32_t na = A.size, nb = B.size;
    const uint16_t* ga = reinterpret_cast<const uint16_t*>(A.pl);
    const uint16_t* gb = reinterpret_cast<const uint16_t*>(B.pl);
    for (uint32_t i = threadIdx.x; i < na; i += 256) sA[i] = ga[i];
    for (uint32_t i = threadIdx.x; i < nb; i += 256) sB[i] = gb[i];
    __syncthreads();
    const uint32_t total = na + nb;
    const uint32_t per = (total + 255) / 256;
    const uint32_t d0 = threadIdx.x * per;
    uint32_t hits = 0;
    if (d0 < total) {
        const uint32_t d1 = d0 + per < total ? d0 + per : total;
        uint32_t lo = d0 > nb ? d0 - nb : 0, hi = d0 < na ? d0 : na;
        while (lo < hi) {  // merge-path split of diagonal d0, A first on ties
            uint32_t mid = (lo + hi) >> 1;
            if (sA[mid] <= sB[d0 - mid - 1]) lo = mid + 1;
            else hi = mid;
        }
        uint32_t i = lo, j = d0 - lo;
        for (uint32_t d = d0; d < d1; ++d) {
            if (j >= nb || (i < na && sA[i] <= sB[j])) {
                ++i;
            } else {
                if (i > 0 && sA[i - 1] == sB[j]) ++hits;
                ++j;
            }
        }
    }
    return (uint32_t)block_sum_u64(hits, tmp64);
}

// |A op B| of any pair by a 256-thread workgroup through LDS bitsets
template <int OP>
__device__ __forceinline__ uint32_t generic_count_wg(const PoolView& PA, const PoolView& PB, const Task& t,
                                                     WgShared& sh) {
    expand_container(sh.sa, PA, t.ia, sh);
    expand_container(sh.sb, PB, t.ib, sh);
    uint64_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = apply_op<OP>(sh.sa[4 * threadIdx.x + j], sh.sb[4 * threadIdx.x + j]);
    return count_words(w, sh);
}

}  // namespace rg
