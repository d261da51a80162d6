// rg_small.hip - materialised results of pairs with an array side, one wave per
// result container, no LDS bitset.
//
// The paper builds array results by merging or searching sorted arrays
// (Sections 4.2-4.5: intersection, union, difference and symmetric difference
// of arrays; galloping for unequal sizes, Section 2.2) and tests array values
// against a bitset bit by bit (Section 3.2). The workgroup kernels expand both
// containers into 8 KiB LDS bitsets whatever their size; for a pair of small
// arrays that clear-fill-scan is most of the work. Here the result is built
// from the sorted values themselves, in one of two forms:
//  * filter - the result is a subset of one array X (intersection with an
//    array side: X is the array side with fewer values; difference with an
//    array first operand: X is that array). Each value of X is looked up in
//    the other container Y: binary search over Y's values or runs staged in
//    LDS, or a bit test of Y's bitset words, and kept or dropped.
//    The kept values come in ascending order, 64 per round; a ballot gives
//    each its output position and the kept value before it, which says
//    whether it starts a run. They are written as an array container as they
//    come; when the run form is the smaller one (P1: 2r < c) a second pass
//    writes the runs over them.
//  * merge - union and symmetric difference of two arrays (either may be
//    absent) with at most SMALL_MAX values together. Both are staged in LDS;
//    the merged order (ties: the first operand's copy first) is cut into 64
//    equal segments, each lane finds where its segment starts with one
//    merge-path search and walks it with two cursors, seeing for each value
//    whether the other array holds it (the equal value is the other cursor's
//    next one, or the value just passed). A first walk counts the kept
//    values and their runs; prefix sums over the lanes give each lane its
//    output position, run number and the last kept value and run start before
//    it; a second walk writes the chosen form.
#include "rg_count_dev.h"

namespace rg {

struct SmallSide {
    uint8_t type;  // 0: absent
    uint32_t size;
    const uint8_t* pl;
};

__device__ __forceinline__ SmallSide small_side(const PoolView& P, uint32_t idx) {
    SmallSide s;
    s.type = 0;
    s.size = 0;
    s.pl = nullptr;
    if (idx != NONE) {
        s.type = (uint8_t)uniform(P.types[idx]);
        s.size = uniform(P.size[idx]);
        s.pl = P.payload + uniform64(P.off[idx]);
    }
    return s;
}

// Copies n 16-bit values from global memory into this wave's LDS (16-byte
// loads for the whole 16-byte groups, the tail one value at a time).
__device__ __forceinline__ void stage_u16(uint16_t* dst, const uint8_t* src, uint32_t n, uint32_t lane) {
    const uint32_t n8 = n >> 3;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
    u32x4* d4 = reinterpret_cast<u32x4*>(dst);
    for (uint32_t i = lane; i < n8; i += 64) d4[i] = s4[i];
    const uint16_t* s16 = reinterpret_cast<const uint16_t*>(src);
    for (uint32_t i = (n8 << 3) + lane; i < n; i += 64) dst[i] = s16[i];
}

// lanes below this one
__device__ __forceinline__ uint64_t lanes_below(uint32_t lane) { return (1ull << lane) - 1ull; }

// highest set lane of a non-empty mask
__device__ __forceinline__ uint32_t top_lane(uint64_t m) { return 63u - (uint32_t)__builtin_clzll(m); }

// What one wave computes for one result container.
struct SmallJob {
    bool merge;        // union / symmetric difference of two arrays (merge_pair)
    bool keep_in;      // filter: keep the values of X that Y holds (else those it lacks)
    bool xor_op;       // merge: symmetric difference (else union)
    SmallSide X, Y;    // filter: X is probed in Y
    uint32_t n;        // filter: |X|
    bool y_lds;        // filter: Y's values or runs are staged in LDS
};

// Filter: value p of X and whether it is kept. lds: Y's values (array) or
// runs (u32), when y_lds.
__device__ __forceinline__ bool small_value(const SmallJob& j, const uint16_t* lds, uint32_t p, uint32_t& x) {
    x = reinterpret_cast<const uint16_t*>(j.X.pl)[p];
    bool member = false;
    if (j.Y.type == RG_ARRAY) {
        member = search_u16(lds, j.Y.size, x);
    } else if (j.Y.type == RG_BITSET) {
        const uint64_t w = reinterpret_cast<const uint64_t*>(j.Y.pl)[x >> 6];
        member = (w >> (x & 63u)) & 1ull;
    } else if (j.Y.type == RG_RUN) {
        const uint32_t* runs = j.y_lds ? reinterpret_cast<const uint32_t*>(lds) : reinterpret_cast<const uint32_t*>(j.Y.pl);
        member = in_runs(runs, j.Y.size, x);
    }
    return member == j.keep_in;
}

// exclusive prefix sum over the lanes, and the total
__device__ __forceinline__ uint32_t wave_excl_sum(uint32_t v, uint32_t& total) {
    const uint32_t incl = wave_incl_scan_u32(v);
    total = uniform(__shfl(incl, 63));
    return incl - v;
}

// exclusive prefix maximum over the lanes (-1 before lane 0)
__device__ __forceinline__ int wave_excl_max(int v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o);
        if (lane >= (uint32_t)o) v = t > v ? t : v;
    }
    const int ex = __shfl_up(v, 1);
    return lane ? ex : -1;
}

constexpr uint32_t PAST_END = 0x10000u;  // cursor past its array: above every 16-bit value

// One lane's segment [d0, d1) of the merged order of A (ca values) and B (cb
// values) in LDS, from cursor positions (i, k); calls keep_fn(x) for each value
// the operation keeps (union: every value once; symmetric difference: the
// values only one array holds).
template <class F>
__device__ __forceinline__ void merge_walk(bool xor_op, const uint16_t* A, uint32_t ca, const uint16_t* B, uint32_t cb,
                                           uint32_t i, uint32_t k, uint32_t len, F&& keep_fn) {
    uint32_t av = i < ca ? A[i] : PAST_END, bv = k < cb ? B[k] : PAST_END;
    uint32_t pa = i > 0 ? A[i - 1] : 0xFFFFFFFFu;  // A's value just passed
    for (uint32_t t = 0; t < len; ++t) {
        if (av <= bv) {  // A's copy first on ties
            const uint32_t x = av;
            if (!xor_op || bv != x) keep_fn(x);
            pa = av;
            ++i;
            av = i < ca ? A[i] : PAST_END;
        } else {
            const uint32_t x = bv;
            if (pa != x) keep_fn(x);  // else A's copy was kept (union) or both dropped (xor)
            ++k;
            bv = k < cb ? B[k] : PAST_END;
        }
    }
}

__device__ void merge_pair(bool xor_op, const uint16_t* A, uint32_t ca, const uint16_t* B, uint32_t cb, uint32_t slot,
                           const SlotOut& so) {
    const uint32_t lane = lane_id();
    const uint32_t n = ca + cb, seg = (n + 63) >> 6;
    const uint32_t d0 = lane * seg < n ? lane * seg : n;
    const uint32_t len = (d0 + seg < n ? d0 + seg : n) - d0;
    // merge path: values of A among the first d0 of the merged order
    uint32_t lo = d0 > cb ? d0 - cb : 0u, hi = d0 < ca ? d0 : ca;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[d0 - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t i0 = lo, k0 = d0 - lo;
    // first walk: kept values, runs starting inside the segment
    uint32_t cnt = 0, inner = 0;
    int first = -1, last = -1, last_inner_start = -1;
    merge_walk(xor_op, A, ca, B, cb, i0, k0, len, [&](uint32_t x) {
        if (last < 0) {
            first = (int)x;
        } else if ((uint32_t)last + 1u != x) {
            ++inner;
            last_inner_start = (int)x;
        }
        last = (int)x;
        ++cnt;
    });
    const int prev_last = wave_excl_max(last);  // last kept value before this lane's segment
    const bool first_start = first >= 0 && !(prev_last >= 0 && prev_last + 1 == first);
    uint32_t c, r;
    const uint32_t pos0 = wave_excl_sum(cnt, c);
    const uint32_t rbase = wave_excl_sum(inner + (first_start ? 1u : 0u), r);
    if (c == 0) return;
    const uint8_t type = p1_type(c, r);  // c <= SMALL_MAX: an array or runs
    const uint64_t soff = so.slot_off[slot];
    const uint64_t nbytes = type == RG_ARRAY ? 2ull * c : 4ull * r;
    if (soff + nbytes > so.cap) {
        if (lane == 0 && so.err) atomicOr(so.err, 2u);
        return;
    }
    uint16_t* d16 = reinterpret_cast<uint16_t*>(so.payload + soff);
    if (type == RG_ARRAY) {
        uint32_t at = pos0;
        merge_walk(xor_op, A, ca, B, cb, i0, k0, len, [&](uint32_t x) { d16[at++] = (uint16_t)x; });
    } else {
        // run i is (start, length - 1) in 16-bit halves 2i, 2i + 1; a run's
        // length is written when the next run starts, the last one's after
        const int lane_start = last_inner_start >= 0 ? last_inner_start : (first_start ? first : -1);
        int run_start = wave_excl_max(lane_start);  // start of the run open before this segment
        int pv = prev_last;
        uint32_t ri = rbase;
        merge_walk(xor_op, A, ca, B, cb, i0, k0, len, [&](uint32_t x) {
            if (!(pv >= 0 && (uint32_t)pv + 1u == x)) {
                d16[2 * ri] = (uint16_t)x;
                if (ri > 0) d16[2 * ri - 1] = (uint16_t)(pv - run_start);
                run_start = (int)x;
                ++ri;
            }
            pv = (int)x;
        });
        const uint64_t has = __ballot(cnt > 0);
        if (lane == top_lane(has)) d16[2 * r - 1] = (uint16_t)(pv - run_start);
    }
    if (lane == 0) {
        so.res_card[slot] = c;
        so.res_type[slot] = type;
        so.res_size[slot] = type == RG_ARRAY ? c : r;
    }
}

// A lone run container R (the other operand absent) in P1 form (Section 1):
// a first pass sums the values c and counts the merged runs (a run that
// starts one past its predecessor's end continues it); then the P1 form is
// written: merged runs (their starts and ends staged in LDS, paired by merged
// run number), an array (each lane expands its runs at the prefix of the
// lengths before them), or a bitset (the runs' bits set in an LDS bitset,
// then copied out). lds: this wave's SMALL_LDS 16-bit entries (8 KiB).
__device__ void lone_runs(const SmallSide& R, uint32_t slot, const SlotOut& so, uint16_t* lds) {
    const uint32_t lane = lane_id();
    const uint32_t* rp = reinterpret_cast<const uint32_t*>(R.pl);
    const uint32_t r = R.size;
    uint32_t c = 0, rm = 0;
    for (uint32_t base = 0; base < r; base += 64) {
        const uint32_t i = base + lane;
        uint32_t len = 0;
        bool head = false;
        if (i < r) {
            const uint32_t pr = rp[i];
            len = (pr >> 16) + 1;
            head = i == 0 || ((rp[i - 1] & 0xFFFFu) + (rp[i - 1] >> 16) + 1u) != (pr & 0xFFFFu);
        }
        c += wave_sum_u32(len);
        rm += (uint32_t)__popcll(__ballot(head));
    }
    c = uniform(c);
    rm = uniform(rm);
    if (c == 0) return;
    const uint8_t type = p1_type(c, rm);
    const uint64_t soff = so.slot_off[slot];
    const uint64_t nbytes = type == RG_ARRAY ? 2ull * c : type == RG_BITSET ? 8192ull : 4ull * rm;
    if (soff + nbytes > so.cap) {
        if (lane == 0 && so.err) atomicOr(so.err, 2u);
        return;
    }
    uint8_t* dst = so.payload + soff;
    if (type == RG_RUN) {
        // rm <= 2048 here: starts in lds[0, 2048), ends in lds[2048, 4096)
        uint32_t hb = 0;  // merged runs started in earlier rounds
        for (uint32_t base = 0; base < r; base += 64) {
            const uint32_t i = base + lane;
            bool head = false, tail = false;
            uint32_t s = 0, e = 0;
            if (i < r) {
                const uint32_t pr = rp[i];
                s = pr & 0xFFFFu;
                e = s + (pr >> 16);
                head = i == 0 || ((rp[i - 1] & 0xFFFFu) + (rp[i - 1] >> 16) + 1u) != s;
                tail = i + 1 == r || (rp[i + 1] & 0xFFFFu) != e + 1u;
            }
            const uint64_t heads = __ballot(head);
            const uint32_t upto = hb + (uint32_t)__popcll(heads & ((2ull << lane) - 1ull));  // heads at or before i
            if (head) lds[upto - 1] = (uint16_t)s;
            if (tail) lds[2048 + upto - 1] = (uint16_t)e;
            hb += (uint32_t)__popcll(heads);
        }
        __builtin_amdgcn_wave_barrier();
        uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
        for (uint32_t j = lane; j < rm; j += 64)
            d32[j] = (uint32_t)lds[j] | ((uint32_t)(lds[2048 + j] - lds[j]) << 16);
    } else if (type == RG_ARRAY) {
        uint16_t* d16 = reinterpret_cast<uint16_t*>(dst);
        uint32_t cb = 0;  // values of earlier rounds
        for (uint32_t base = 0; base < r; base += 64) {
            const uint32_t i = base + lane;
            uint32_t s = 0, len = 0;
            if (i < r) {
                s = rp[i] & 0xFFFFu;
                len = (rp[i] >> 16) + 1;
            }
            uint32_t tot;
            const uint32_t at = cb + wave_excl_sum(len, tot);
            for (uint32_t q = 0; q < len; ++q) d16[at + q] = (uint16_t)(s + q);
            cb += tot;
        }
    } else {
        uint64_t* bits = reinterpret_cast<uint64_t*>(lds);  // 1024 words
        for (uint32_t j = lane; j < 1024; j += 64) bits[j] = 0;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < r; i += 64) {
            const uint32_t first = rp[i] & 0xFFFFu, last = first + (rp[i] >> 16);
            for (uint32_t wi = first >> 6; wi <= last >> 6; ++wi) {
                const uint32_t lo = wi == first >> 6 ? first & 63 : 0;
                const uint32_t hi = wi == last >> 6 ? last & 63 : 63;
                atomicOr(reinterpret_cast<unsigned long long*>(&bits[wi]), (~0ull << lo) & (~0ull >> (63 - hi)));
            }
        }
        __builtin_amdgcn_wave_barrier();
        const u32x4* s4 = reinterpret_cast<const u32x4*>(bits);
        u32x4* d4 = reinterpret_cast<u32x4*>(dst);
        for (uint32_t j = lane; j < 512; j += 64) d4[j] = s4[j];
    }
    __builtin_amdgcn_wave_barrier();  // the LDS is read before the wave's next slot
    if (lane == 0) {
        so.res_card[slot] = c;
        so.res_type[slot] = type;
        so.res_size[slot] = type == RG_ARRAY ? c : type == RG_BITSET ? 1024u : rm;
    }
}

// Builds the result of one pair into slot `slot` of `so`. `lds`: this wave's
// SMALL_LDS 16-bit values, 16-byte aligned. Every lane of the wave calls it with the same
// arguments.
__device__ void small_pair(int op, SmallSide A, SmallSide B, uint32_t slot, const SlotOut& so, uint16_t* lds) {
    const uint32_t lane = lane_id();
    if (lone_run(op, A.type, B.type)) {
        lone_runs(A.type == RG_RUN ? A : B, slot, so, lds);
        return;
    }
    // Pairs come here by their cardinalities (small_mat_ok). A pool whose
    // array sizes disagree with them is malformed (rg_pool_validate reports
    // it); its sizes are cut to the staging area, so nothing is read or
    // written outside it and every result stays within SMALL_MAX values.
    if (A.type == RG_ARRAY && A.size > SMALL_MAX) A.size = SMALL_MAX;
    if (B.type == RG_ARRAY && B.size > SMALL_MAX) B.size = SMALL_MAX;
    if ((op == RG_OR || op == RG_XOR) && A.size + B.size > SMALL_MAX) B.size = SMALL_MAX - A.size;
    SmallJob j;
    j.merge = op == RG_OR || op == RG_XOR;
    j.xor_op = op == RG_XOR;
    j.keep_in = op == RG_AND;
    j.y_lds = false;
    if (j.merge) {
        // B after A, 16-byte aligned for the vector copy when that still fits
        // in SMALL_LDS entries; otherwise (A + B within 7 of the limit) right
        // after A, copied value by value
        const uint32_t ob = (A.size + 7u) & ~7u;
        const bool aligned = ob + B.size <= SMALL_LDS;
        uint16_t* lb = lds + (aligned ? ob : A.size);
        stage_u16(lds, A.pl, A.size, lane);
        if (aligned) {
            stage_u16(lb, B.pl, B.size, lane);
        } else {
            const uint16_t* s16 = reinterpret_cast<const uint16_t*>(B.pl);
            for (uint32_t i = lane; i < B.size; i += 64) lb[i] = s16[i];
        }
        __builtin_amdgcn_wave_barrier();
        merge_pair(j.xor_op, lds, A.size, lb, B.size, slot, so);
        return;
    } else {
        // intersection: probe the array side with fewer values; difference: the first operand
        const bool a_probe = op == RG_ANDNOT || (A.type == RG_ARRAY && (B.type != RG_ARRAY || A.size <= B.size));
        j.X = a_probe ? A : B;
        j.Y = a_probe ? B : A;
        j.n = j.X.size;
        if (j.Y.type == RG_ARRAY) {
            stage_u16(lds, j.Y.pl, j.Y.size, lane);
            j.y_lds = true;
        } else if (j.Y.type == RG_RUN && 2 * j.Y.size <= SMALL_MAX) {
            stage_u16(lds, j.Y.pl, 2 * j.Y.size, lane);
            j.y_lds = true;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const uint64_t soff = so.slot_off[slot];
    uint16_t* d16 = reinterpret_cast<uint16_t*>(so.payload + soff);
    const uint64_t room = so.cap > soff ? (so.cap - soff) >> 1 : 0ull;  // values that fit before the arena's end
    // pass 1: count values and runs, write the values
    uint32_t c = 0, r = 0;
    uint32_t prev = 0;  // last kept value so far (meaningful when c > 0)
    for (uint32_t base = 0; base < j.n; base += 64) {
        const uint32_t p = base + lane;
        uint32_t x = 0;
        const bool keep = p < j.n && small_value(j, lds, p, x);
        const uint64_t bal = __ballot(keep);
        if (!bal) continue;
        const uint64_t below = bal & lanes_below(lane);
        const uint32_t pv_lane = __shfl(x, below ? top_lane(below) : lane);
        const bool has_prev = below != 0 || c > 0;
        const uint32_t pv = below ? pv_lane : prev;
        const bool start = keep && !(has_prev && pv + 1u == x);
        r += (uint32_t)__popcll(__ballot(start));
        const uint32_t pos = c + (uint32_t)__popcll(below);
        if (keep && pos < room) d16[pos] = (uint16_t)x;
        c += (uint32_t)__popcll(bal);
        prev = uniform(__shfl(x, top_lane(bal)));
    }
    c = uniform(c);
    r = uniform(r);
    if (c == 0) return;
    const uint8_t type = p1_type(c, r);  // c <= SMALL_MAX: an array or runs
    const uint64_t nbytes = type == RG_ARRAY ? 2ull * c : 4ull * r;
    if (soff + nbytes > so.cap) {
        if (lane == 0 && so.err) atomicOr(so.err, 2u);
        return;
    }
    if (type == RG_RUN) {
        // the array writes of pass 1 complete before the runs overwrite them
        __builtin_amdgcn_s_waitcnt(0);
        // pass 2: run i is (start, length - 1) in 16-bit halves 2i, 2i + 1; a
        // run's length is written when the next run starts (and after the loop)
        uint32_t ri = 0, k = 0, last = 0, run_start = 0;
        for (uint32_t base = 0; base < j.n; base += 64) {
            const uint32_t p = base + lane;
            uint32_t x = 0;
            const bool keep = p < j.n && small_value(j, lds, p, x);
            const uint64_t bal = __ballot(keep);
            if (!bal) continue;
            const uint64_t below = bal & lanes_below(lane);
            const uint32_t pv_lane = __shfl(x, below ? top_lane(below) : lane);
            const bool has_prev = below != 0 || k > 0;
            const uint32_t pv = below ? pv_lane : last;
            const bool start = keep && !(has_prev && pv + 1u == x);
            const uint64_t sbal = __ballot(start);
            const uint64_t sbelow = sbal & lanes_below(lane);
            const uint32_t ps_lane = __shfl(x, sbelow ? top_lane(sbelow) : lane);
            const uint32_t prev_start = sbelow ? ps_lane : run_start;  // start of the run that pv ends
            if (start) {
                const uint32_t i = ri + (uint32_t)__popcll(sbelow);
                d16[2 * i] = (uint16_t)x;
                if (i > 0) d16[2 * i - 1] = (uint16_t)(pv - prev_start);
            }
            if (sbal) run_start = uniform(__shfl(x, top_lane(sbal)));
            ri += (uint32_t)__popcll(sbal);
            k += (uint32_t)__popcll(bal);
            last = uniform(__shfl(x, top_lane(bal)));
        }
        if (lane == 0) d16[2 * r - 1] = (uint16_t)(last - run_start);
    }
    if (lane == 0) {
        so.res_card[slot] = c;
        so.res_type[slot] = type;
        so.res_size[slot] = type == RG_ARRAY ? c : r;
    }
}

// The slots of one wave: SMALL_CHUNK consecutive slots (k-way) or list
// entries; lane i loads slot i's task and, when the slot is the kernel's, the
// op and both containers' type, size and payload offset, all in parallel. The
// wave then builds the results of its slots one after another, taking each
// slot's values from the lane that loaded them. (More slots per wave would
// leave too few waves to fill the chip on batches of 1e5 slots.)
constexpr uint32_t SMALL_CHUNK = 8;
struct SmallSlot {
    bool mine;
    uint32_t slot, op, ta, tb, sa, sb;
    uint64_t oa, ob;
};

__device__ __forceinline__ void small_load_side(const PoolView& P, uint32_t idx, uint32_t& ty, uint32_t& sz,
                                                uint64_t& off) {
    ty = 0;
    sz = 0;
    off = 0;
    if (idx != NONE) {
        ty = P.types[idx];
        sz = P.size[idx];
        off = P.off[idx];
    }
}

__device__ __forceinline__ void small_run_slots(const SmallSlot& v, const PoolView& PA, const PoolView& PB,
                                                const SlotOut& so, uint16_t* lds) {
    uint64_t m = __ballot(v.mine);
    while (m) {
        const uint32_t l = (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        SmallSide A, B;
        A.type = (uint8_t)__builtin_amdgcn_readlane(v.ta, l);
        A.size = __builtin_amdgcn_readlane(v.sa, l);
        A.pl = A.type ? PA.payload + readlane64(v.oa, l) : nullptr;
        B.type = (uint8_t)__builtin_amdgcn_readlane(v.tb, l);
        B.size = __builtin_amdgcn_readlane(v.sb, l);
        B.pl = B.type ? PB.payload + readlane64(v.ob, l) : nullptr;
        small_pair((int)__builtin_amdgcn_readlane(v.op, l), A, B, __builtin_amdgcn_readlane(v.slot, l), so, lds);
        __builtin_amdgcn_wave_barrier();  // the next slot restages this wave's LDS
    }
}

// k-way slots marked KW_TASK_SMALL by the bounds kernel (queries of one or two bitmaps)
__global__ void __launch_bounds__(256) k_kw_small(KwArgs a) {
    __shared__ __align__(16) uint16_t lds[4][SMALL_LDS];
    const uint32_t wid = threadIdx.x >> 6, lane = lane_id();
    const uint64_t step = (uint64_t)gridDim.x * 4 * SMALL_CHUNK;
    for (uint64_t c0 = (uint64_t)wave_index() * SMALL_CHUNK; c0 < a.n_slots; c0 += step) {
        SmallSlot v{};
        v.slot = (uint32_t)(c0 + lane);
        if (lane < SMALL_CHUNK && c0 + lane < a.n_slots) {
            const Task t = a.tasks[c0 + lane];
            v.mine = t.kind == KIND_MATCH && t.bin == KW_TASK_SMALL;
            if (v.mine) {
                v.op = a.queries[t.pair - a.pair_base].op;
                small_load_side(a.P0, t.ia, v.ta, v.sa, v.oa);
                small_load_side(a.P1, t.ib, v.tb, v.sb, v.ob);
            }
        }
        small_run_slots(v, a.P0, a.P1, a.so, lds[wid]);
    }
}

// slots of the binned intersection path (materialised), listed
__global__ void __launch_bounds__(256) k_small_list(ComputeArgs a) {
    __shared__ __align__(16) uint16_t lds[4][SMALL_LDS];
    const uint32_t wid = threadIdx.x >> 6, lane = lane_id();
    const uint32_t step = gridDim.x * 4 * SMALL_CHUNK;
    for (uint32_t i0 = wave_index() * SMALL_CHUNK; i0 < a.n; i0 += step) {
        SmallSlot v{};
        if (lane < SMALL_CHUNK && i0 + lane < a.n) {
            v.slot = a.list[i0 + lane];
            const Task t = a.tasks[v.slot];
            v.mine = true;
            v.op = (uint32_t)a.op;
            small_load_side(a.A, t.ia, v.ta, v.sa, v.oa);
            small_load_side(a.B, t.ib, v.tb, v.sb, v.ob);
        }
        small_run_slots(v, a.A, a.B, a.so, lds[wid]);
    }
}

void launch_kw_small(const KwArgs& a, hipStream_t st) {
    if (!a.n_slots || !a.small) return;
    const uint64_t g = (a.n_slots + 4 * SMALL_CHUNK - 1) / (4 * SMALL_CHUNK);
    hipLaunchKernelGGL(k_kw_small, dim3(g < 16384 ? (uint32_t)g : 16384u), dim3(256), 0, st, a);
}

void launch_small_list(const ComputeArgs& a, hipStream_t st) {
    if (!a.n) return;
    const uint32_t g = (a.n + 4 * SMALL_CHUNK - 1) / (4 * SMALL_CHUNK);
    hipLaunchKernelGGL(k_small_list, dim3(g < 16384 ? g : 16384u), dim3(256), 0, st, a);
}

}  // namespace rg
