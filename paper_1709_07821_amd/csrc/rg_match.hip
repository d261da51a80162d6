// rg_match.hip - per-pair preparation, key matching (the "high-level" merge of
// two sorted key lists, Section 1 / Appendix A), variant selection (bins),
// binning and the device prefix scan.
#include "rg_count_dev.h"

namespace rg {

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t* p, uint32_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static uint32_t grid_for(uint64_t n, uint32_t per_block, uint32_t cap = 65536) {
    uint64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
}
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
}

// ------------------------------------------------------------------ pairs
// Per pair: candidate count of the key match, payload bound of the result,
// bound on its container count, and the starting value of the count
// accumulator (Section 5.9 identities: unmatched containers contribute
// their stored cardinality).
__global__ void k_pair_prep(int op, int materialize, PoolView A, PoolView B, uint32_t nA, uint32_t nB,
                            const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs,
                            uint32_t* n_cand, uint64_t* bound, uint32_t* min_cont, long long* acc, uint32_t* err,
                            uint32_t* zero_word) {
    uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && zero_word) *zero_word = 0;
    if (p >= n_pairs) return;
    // without pair arrays, ia0 / ib0 name the bitmap of every pair, or (NONE)
    // pair p is bitmap p itself
    uint32_t a = ia ? ia[p] : ia0 == NONE ? (uint32_t)p : ia0;
    uint32_t b = ib ? ib[p] : ib0 == NONE ? (uint32_t)p : ib0;
    if (a >= nA || b >= nB) {  // bad index: report, and give the pair no work
        atomicOr(err, 1u);
        n_cand[p] = 0;
        if (bound) bound[p] = 0;
        if (min_cont) min_cont[p] = 0;
        acc[p] = 0;
        return;
    }
    uint32_t KA = (uint32_t)(A.bm_begin[a + 1] - A.bm_begin[a]);
    uint32_t KB = (uint32_t)(B.bm_begin[b + 1] - B.bm_begin[b]);
    if (materialize) {
        uint64_t WA = A.bm_wbytes[a], WB = B.bm_wbytes[b];
        uint32_t nc;
        uint64_t bd;
        uint32_t mc;
        if (op == RG_OR || op == RG_XOR) {
            nc = KA + KB;
            bd = WA + WB;
            mc = KA + KB;
        } else if (op == RG_AND) {
            nc = KA;
            bd = WA < WB ? WA : WB;
            mc = KA < KB ? KA : KB;
        } else {
            nc = KA;
            bd = WA;
            mc = KA;
        }
        n_cand[p] = nc;
        bound[p] = bd;
        min_cont[p] = mc;
    } else {
        n_cand[p] = KA < KB ? KA : KB;
        if (bound) bound[p] = 0;
        if (min_cont) min_cont[p] = 0;
        long long base = 0;
        if (op == RG_OR || op == RG_XOR) base = (long long)(A.bm_card[a] + B.bm_card[b]);
        else if (op == RG_ANDNOT) base = (long long)A.bm_card[a];
        acc[p] = base;
    }
}

void launch_pair_prep(int op, bool materialize, PoolView A, PoolView B, uint32_t nA, uint32_t nB,
                      const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs,
                      uint32_t* n_cand, uint64_t* bound, uint32_t* min_cont, long long* acc, uint32_t* err,
                      hipStream_t st, uint32_t* zero_word) {
    if (!n_pairs) return;
    hipLaunchKernelGGL(k_pair_prep, dim3((uint32_t)((n_pairs + 255) / 256)), dim3(256), 0, st, op, (int)materialize,
                       A, B, nA, nB, ia, ib, ia0, ib0, n_pairs, n_cand, bound, min_cont, acc, err, zero_word);
}

// ------------------------------------------------------------------ match

__device__ __forceinline__ uint32_t lower_bound_u16(const uint16_t* k, uint32_t n, uint16_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (k[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First index i in [0, n) for which pred(i) is false, pred being true on a
// prefix; n if it holds everywhere. The 64 lanes of a wave probe 64 evenly
// spaced positions per round, so a list of n entries takes about log64(n)
// dependent loads instead of log2(n). All lanes must call it together; the
// result is uniform.
template <class Pred>
__device__ __forceinline__ uint32_t wave_partition_point(uint32_t n, uint32_t lane, Pred pred) {
    uint32_t lo = 0, len = n;  // the answer lies in [lo, lo + len]
    while (len > 0) {
        const uint32_t step = (len + 63) >> 6;
        const uint32_t pos = lo + lane * step;
        const bool t = pos < lo + len && pred(pos);
        const uint32_t c = (uint32_t)__popcll(__ballot(t));  // lanes 0..c-1 hold
        if (c == 0) break;
        const uint32_t nlo = lo + (c - 1) * step + 1;
        const uint32_t nhi = lo + c * step < lo + len ? lo + c * step : lo + len;
        lo = uniform(nlo);
        len = uniform(nhi - nlo);
    }
    return lo;
}

// largest pl with off[pl] <= t (off has n_pairs + 1 entries, off[0] = 0 <= t < off[n_pairs])
__device__ __forceinline__ uint32_t wave_find_pair(const uint64_t* off, uint32_t n_pairs, uint64_t t, uint32_t lane) {
    return wave_partition_point(n_pairs + 1, lane, [&](uint32_t i) { return off[i] <= t; }) - 1;
}

// Variant selection (plain heuristic). It never changes results: every bin
// computes the same set; the bins differ only in how.

__device__ __forceinline__ uint8_t classify(int op, bool materialize, uint8_t kind, uint8_t ta, uint8_t tb,
                                            uint32_t ca, uint32_t cb, uint32_t ra, uint32_t rb, int mode,
                                            int fixed_bin, uint32_t gallop_ratio, uint32_t thread_max,
                                            const uint8_t* mlp_table) {
    if (ta == RG_BITSET && tb == RG_BITSET) return BIN_BB;
    // materialised: pairs with an array side are built by the one-wave array
    // kernel (listed in BIN_AA; forcing BIN_GEN turns that off), the rest by
    // the generic kernel
    if (materialize)
        return (mode != 2 || fixed_bin != BIN_GEN) && small_mat_ok(op, ta, tb, ca, cb) ? (uint8_t)BIN_AA
                                                                                        : (uint8_t)BIN_GEN;
    if (mode == 2) return variant_applies(fixed_bin, ta, tb, ca, cb) ? (uint8_t)fixed_bin : (uint8_t)BIN_GEN;
    if (mode == 1 && mlp_table) return mlp_table[mlp_cell(ta, tb, ca, cb, ra, rb)];  // learned
    // heuristic: a small array side is probed by one thread (each value
    // looked up in the other container); galloping when one array is much
    // smaller than the other (Section 2.2)
    if ((ta == RG_ARRAY && ca <= thread_max) || (tb == RG_ARRAY && cb <= thread_max)) return BIN_THREAD;
    if (ta == RG_ARRAY && tb == RG_ARRAY) {
        uint32_t mx = ca > cb ? ca : cb, mn = ca < cb ? ca : cb;
        return (uint64_t)mx >= (uint64_t)gallop_ratio * mn ? BIN_GALLOP : BIN_AA;
    }
    if (ta == RG_ARRAY || tb == RG_ARRAY) {
        if (ta == RG_BITSET || tb == RG_BITSET) return BIN_AB;
        return BIN_RR;  // array-run
    }
    return BIN_RR;      // run-run, run-bitset
}

constexpr uint32_t MATCH_LDS_KEYS = 4096;

// LDS of key matching when a block's candidates all belong to one pair: the
// searched side's keys in the candidates' range (window), or, with a key
// index, its presence words and ranks over that range.
union MatchLds {
    uint16_t lkeys[MATCH_LDS_KEYS];
    struct {
        uint64_t words[KIDX_WORDS];
        uint16_t rank[KIDX_WORDS];
    } kx;
};

// Looks `key` up in the key index of one bitmap (presence word x, rank of the
// word): its container's position among the bitmap's keys, or NONE.
__device__ __forceinline__ uint32_t kidx_lookup(uint64_t x, uint32_t rank, uint16_t key) {
    const uint32_t bit = key & 63u;
    if (!((x >> bit) & 1ull)) return NONE;
    return rank + (uint32_t)__popcll(x & ((1ull << bit) - 1ull));
}

// What matching decided for one candidate slot.
struct SlotOutcome {
    Task task;
    uint64_t slot;        // NONE: no slot
    uint32_t fused_pair;  // NONE: nothing counted in place
    uint32_t fused_inter;
};

// Variant choice (and, when fusing, the in-place count) of a candidate whose
// match is known; task.ia / task.ib / task.kind are set.
__device__ __forceinline__ void finish_slot(const MatchArgs& m, uint32_t* cnt, SlotOutcome& o) {
    Task& task = o.task;
    uint32_t ub = 0;
    if (task.kind != KIND_NOOP) {
        uint8_t ta, tb;
        uint32_t ca, cb, sa = 0, sb = 0, ra = 0, rb = 0;
        uint64_t da = 0, db = 0;
        bool ina = false, inb = false;
        const bool packed = m.A.meta && m.B.meta;
        if (packed) {
            // one record per side: type, card, size and the payload offset, or
            // the values themselves for the smallest arrays
            const u32x4 xa = m.A.meta[task.ia], xb = m.B.meta[task.ib];
            ta = (uint8_t)(xa.w >> 24);
            tb = (uint8_t)(xb.w >> 24);
            ca = xa.z;
            cb = xb.z;
            sa = xa.w & 0x1FFFFFu;
            sb = xb.w & 0x1FFFFFu;
            ina = (xa.w >> 21) & 1u;
            inb = (xb.w >> 21) & 1u;
            da = (uint64_t)xa.x | ((uint64_t)xa.y << 32);
            db = (uint64_t)xb.x | ((uint64_t)xb.y << 32);
            ra = ta == RG_RUN ? sa : 0;
            rb = tb == RG_RUN ? sb : 0;
        } else {
            ta = m.A.types[task.ia];
            tb = m.B.types[task.ib];
            ca = m.A.card[task.ia];
            cb = m.B.card[task.ib];
            const bool need_r = m.dispatch_mode == 1;
            ra = need_r && ta == RG_RUN ? m.A.size[task.ia] : 0;
            rb = need_r && tb == RG_RUN ? m.B.size[task.ib] : 0;
        }
        task.bin = classify(m.op, m.materialize, task.kind, ta, tb, ca, cb, ra, rb, m.dispatch_mode, m.fixed_bin,
                            m.gallop_ratio, m.thread_max, m.mlp_table);
        if (m.fuse_thread && task.bin == BIN_THREAD) {
            // the types are at hand: probe now instead of listing the pair
            o.fused_inter = packed ? thread_inter_rec(ta, tb, sa, sb, ina, inb, da, db, m.A.payload, m.B.payload)
                                   : thread_inter_typed(m.A, m.B, task.ia, task.ib, ta, tb);
            o.fused_pair = task.pair;
            task.kind = KIND_NOOP;
            task.bin = BIN_FUSED;
        }
        atomicAdd(&cnt[task.bin], 1u);
        if (m.materialize) ub = wbytes_of(ca < cb ? ca : cb);
    }
    if (m.materialize) {
        m.res_card[o.slot] = 0;
        m.ub[o.slot] = ub;
    }
}

// One candidate slot t of a block without a staged window: its pair is
// searched among the block's pairs [pl_lo, pl_hi], the other side's keys in
// global memory.
__device__ __forceinline__ void match_slot_global(const MatchArgs& m, uint64_t t, uint32_t pl_lo, uint32_t pl_hi,
                                                  uint32_t* cnt, SlotOutcome& o) {
    uint32_t lo = pl_lo, hi = pl_hi;  // largest pl in [lo, hi] with cand_off[pl] <= t
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (m.cand_off[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t pl = lo;
    const uint64_t p = m.pair0 + pl;
    const uint32_t a = m.ia ? m.ia[p] : m.ia0;
    const uint32_t b = m.ib ? m.ib[p] : m.ib0;
    const uint64_t a0 = m.A.bm_begin[a], b0 = m.B.bm_begin[b];
    const uint32_t KA = (uint32_t)(m.A.bm_begin[a + 1] - a0);
    const uint32_t KB = (uint32_t)(m.B.bm_begin[b + 1] - b0);
    const uint64_t u = t - m.cand_off[pl];
    Task& task = o.task;
    task.pair = (uint32_t)p;
    if (!m.materialize) {
        // count only: candidates from the side with fewer keys
        const bool a_small = KA <= KB;
        const uint16_t* sk = a_small ? m.A.keys + a0 : m.B.keys + b0;
        const uint16_t* lk = a_small ? m.B.keys + b0 : m.A.keys + a0;
        const uint32_t nl = a_small ? KB : KA;
        const uint8_t* lidx = a_small ? m.B.kidx : m.A.kidx;
        const uint16_t key = sk[u];
        uint32_t j;
        bool hit;
        if (lidx) {
            // key index of the searched bitmap: presence bit, then rank + popcount
            const uint8_t* ix = lidx + (uint64_t)(a_small ? b : a) * RG_KEY_INDEX_BYTES;
            const uint32_t wi = key >> 6;
            j = kidx_lookup(reinterpret_cast<const uint64_t*>(ix)[wi],
                            reinterpret_cast<const uint16_t*>(ix + 8 * KIDX_WORDS)[wi], key);
            hit = j != NONE;
        } else {
            j = lower_bound_u16(lk, nl, key);
            hit = j < nl && lk[j] == key;
        }
        task.key = key;
        if (hit) {
            task.kind = KIND_MATCH;
            task.ia = (uint32_t)(a_small ? a0 + u : a0 + j);
            task.ib = (uint32_t)(a_small ? b0 + j : b0 + u);
        }
    } else {
        // materialised intersection: one slot per key of A, in A's key order
        // (the other operations materialise through the k-way path)
        const uint16_t key = m.A.keys[a0 + u];
        const uint32_t j = lower_bound_u16(m.B.keys + b0, KB, key);
        task.key = key;
        task.ia = (uint32_t)(a0 + u);
        if (j < KB && m.B.keys[b0 + j] == key) {
            task.kind = KIND_MATCH;
            task.ib = (uint32_t)(b0 + j);
        }
    }
    o.slot = t;
    finish_slot(m, cnt, o);
}

// Key matching of one block of MATCH_SLOTS consecutive candidate slots from
// t0 (n_cand candidates in all): each thread carries MATCH_PER_THREAD of them
// (slots t0 + k * 256 + thread) through the same steps, so that their loads
// overlap. o[k] receives what was decided for slot t0 + k * 256 + thread; bin
// counts go to the LDS counters cnt[NBINS] (zeroed here). The LDS arrays are
// the caller's: pl_range[2], lwin[2], lkeys[MATCH_LDS_KEYS]. Contains barriers;
// the whole workgroup calls it.
__device__ __forceinline__ void match_block(const MatchArgs& m, uint64_t n_cand, uint64_t t0, uint32_t* cnt,
                                            uint32_t* pl_range, uint32_t* lwin, MatchLds& lds,
                                            SlotOutcome (&o)[MATCH_PER_THREAD]) {
    uint16_t* lkeys = lds.lkeys;
    if (threadIdx.x < NBINS) cnt[threadIdx.x] = 0;
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    // the pairs of this block's first and last candidate bound every thread's
    // search: wave 0 finds the first, wave 1 the last
    const uint64_t tl = t0 + MATCH_SLOTS - 1 < n_cand ? t0 + MATCH_SLOTS - 1 : n_cand - 1;
    if (wid < 2) {
        const uint32_t pl = wave_find_pair(m.cand_off, m.n_pairs, wid == 0 ? t0 : tl, lane);
        if (lane == 0) pl_range[wid] = pl;
    }
    __syncthreads();
    const uint32_t pl_lo = uniform(pl_range[0]), pl_hi = uniform(pl_range[1]);
    // Count-only block whose candidates all belong to one pair: its candidate
    // keys are consecutive keys of the pair's smaller side, so the matching keys
    // of the other side lie in one window; stage that window in LDS and search
    // there instead of in global memory. Wave 0 finds the window's first index
    // (first key >= the first candidate), wave 1 its end (first key > the last).
    bool staged = false, kstaged = false;
    uint64_t o_a0 = 0, o_b0 = 0, o_base = 0;
    uint32_t o_p = 0, win_lo = 0, win_n = 0, w0 = 0;
    bool o_a_small = true;
    const uint16_t* o_sk = nullptr;
    if (!m.materialize && pl_lo == pl_hi) {
        const uint64_t p = m.pair0 + pl_lo;
        const uint32_t a = uniform(m.ia ? m.ia[p] : m.ia0), b = uniform(m.ib ? m.ib[p] : m.ib0);
        const uint64_t a0 = uniform64(m.A.bm_begin[a]), b0 = uniform64(m.B.bm_begin[b]);
        const uint32_t KA = uniform((uint32_t)(m.A.bm_begin[a + 1] - a0));
        const uint32_t KB = uniform((uint32_t)(m.B.bm_begin[b + 1] - b0));
        const bool a_small = KA <= KB;
        const uint16_t* sk = a_small ? m.A.keys + a0 : m.B.keys + b0;
        const uint16_t* lk = a_small ? m.B.keys + b0 : m.A.keys + a0;
        const uint32_t nl = a_small ? KB : KA;
        const uint8_t* lidx = a_small ? m.B.kidx : m.A.kidx;
        const uint64_t base = uniform64(m.cand_off[pl_lo]);
        if (lidx) {
            // The candidates are consecutive keys of the smaller side: stage the
            // searched bitmap's presence words and ranks over their key range
            // (at most 1024 words); each candidate is then a bit test and a
            // popcount in LDS.
            const uint32_t kf = uniform(sk[t0 - base]), kl = uniform(sk[tl - base]);
            w0 = kf >> 6;
            const uint32_t nw = (kl >> 6) - w0 + 1;
            const uint8_t* ix = lidx + (uint64_t)(a_small ? b : a) * RG_KEY_INDEX_BYTES;
            const uint64_t* iw = reinterpret_cast<const uint64_t*>(ix) + w0;
            const uint16_t* ir = reinterpret_cast<const uint16_t*>(ix + 8 * KIDX_WORDS) + w0;
            for (uint32_t i = threadIdx.x; i < nw; i += blockDim.x) {
                lds.kx.words[i] = iw[i];
                lds.kx.rank[i] = ir[i];
            }
            kstaged = true;
        } else {
            if (wid < 2) {
                const uint16_t key = (uint16_t)uniform(sk[(wid == 0 ? t0 : tl) - base]);
                const uint32_t j = wid == 0 ? wave_partition_point(nl, lane, [&](uint32_t i) { return lk[i] < key; })
                                            : wave_partition_point(nl, lane, [&](uint32_t i) { return lk[i] <= key; });
                if (lane == 0) lwin[wid] = j;
            }
            __syncthreads();
            const uint32_t lo = uniform(lwin[0]), hi = uniform(lwin[1]);
            if (hi - lo <= MATCH_LDS_KEYS) {
                staged = true;
                for (uint32_t i = threadIdx.x; i < hi - lo; i += blockDim.x) lkeys[i] = lk[lo + i];
            }
            win_lo = lo;
            win_n = hi - lo;
        }
        __syncthreads();
        o_a0 = a0;
        o_b0 = b0;
        o_base = base;
        o_p = (uint32_t)p;
        o_a_small = a_small;
        o_sk = sk;
    }
#pragma unroll
    for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
        o[k].task = Task{};
        o[k].task.ia = NONE;
        o[k].task.ib = NONE;
        o[k].task.kind = KIND_NOOP;
        o[k].task.bin = 0xFF;
        o[k].slot = NONE;
        o[k].fused_pair = NONE;
        o[k].fused_inter = 0;
    }
    if (kstaged) {
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            const uint64_t t = t0 + (uint64_t)k * 256 + threadIdx.x;
            if (t >= n_cand) continue;
            const uint64_t u = t - o_base;
            const uint16_t key = o_sk[u];
            const uint32_t wi = (uint32_t)(key >> 6) - w0;
            const uint32_t j = kidx_lookup(lds.kx.words[wi], lds.kx.rank[wi], key);
            Task& task = o[k].task;
            task.pair = o_p;
            task.key = key;
            if (j != NONE) {
                task.kind = KIND_MATCH;
                task.ia = (uint32_t)(o_a_small ? o_a0 + u : o_a0 + j);
                task.ib = (uint32_t)(o_a_small ? o_b0 + j : o_b0 + u);
            }
            o[k].slot = t;
        }
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k)
            if (o[k].slot != NONE) finish_slot(m, cnt, o[k]);
    } else if (staged) {
        // every step for all of the thread's candidates before the next step
        uint32_t top = 0;
        if (win_n) top = 1u << (31 - __builtin_clz(win_n));
        uint16_t key[MATCH_PER_THREAD];
        uint32_t jl[MATCH_PER_THREAD];
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            const uint64_t t = t0 + (uint64_t)k * 256 + threadIdx.x;
            key[k] = t < n_cand ? o_sk[t - o_base] : (uint16_t)0;
            jl[k] = 0;
        }
        for (uint32_t step = top; step; step >>= 1) {
#pragma unroll
            for (int k = 0; k < (int)MATCH_PER_THREAD; ++k)
                if (jl[k] + step <= win_n && lkeys[jl[k] + step - 1] < key[k]) jl[k] += step;
        }
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            const uint64_t t = t0 + (uint64_t)k * 256 + threadIdx.x;
            if (t >= n_cand) continue;
            // a key past the window's end cannot match: the window ends at the
            // first key above the block's last candidate
            const uint64_t u = t - o_base;
            const uint32_t j = win_lo + jl[k];
            Task& task = o[k].task;
            task.pair = o_p;
            task.key = key[k];
            if (jl[k] < win_n && lkeys[jl[k]] == key[k]) {
                task.kind = KIND_MATCH;
                task.ia = (uint32_t)(o_a_small ? o_a0 + u : o_a0 + j);
                task.ib = (uint32_t)(o_a_small ? o_b0 + j : o_b0 + u);
            }
            o[k].slot = t;
        }
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k)
            if (o[k].slot != NONE) finish_slot(m, cnt, o[k]);
    } else if (!m.materialize && m.A.kidx && m.B.kidx && pl_hi - pl_lo < MATCH_LDS_KEYS / 2) {
        // Count-only block over several pairs with key indexes on both sides:
        // the pairs' candidate offsets (relative to the first pair's) are staged
        // in LDS, and each step - pair search, pair and bitmap records, the
        // candidate key, the presence word and rank - is issued for all of the
        // thread's candidates before the next, so that their loads overlap.
        uint32_t* rel = reinterpret_cast<uint32_t*>(lds.lkeys);
        const uint32_t nr = pl_hi - pl_lo + 1;
        const uint64_t base = uniform64(m.cand_off[pl_lo]);
        for (uint32_t i = threadIdx.x; i < nr; i += blockDim.x) rel[i] = (uint32_t)(m.cand_off[pl_lo + i] - base);
        __syncthreads();
        const uint32_t top = 1u << (31 - __builtin_clz(nr));
        bool live[MATCH_PER_THREAD];
        uint32_t tg[MATCH_PER_THREAD], pos[MATCH_PER_THREAD];
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            const uint64_t t = t0 + (uint64_t)k * 256 + threadIdx.x;
            live[k] = t < n_cand;
            tg[k] = live[k] ? (uint32_t)(t - base) : 0u;
            pos[k] = 0;
        }
        // largest pos with rel[pos] <= tg (rel[0] = 0)
        for (uint32_t step = top; step; step >>= 1) {
#pragma unroll
            for (int k = 0; k < (int)MATCH_PER_THREAD; ++k)
                if (pos[k] + step < nr && rel[pos[k] + step] <= tg[k]) pos[k] += step;
        }
        uint32_t av[MATCH_PER_THREAD], bv[MATCH_PER_THREAD];
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            const uint64_t p = m.pair0 + pl_lo + pos[k];
            av[k] = live[k] ? (m.ia ? m.ia[p] : m.ia0) : 0u;
            bv[k] = live[k] ? (m.ib ? m.ib[p] : m.ib0) : 0u;
        }
        // per candidate from here: the first container of its smaller side
        // (whose keys are the candidates) and of the searched side, the
        // searched bitmap, and which side is the smaller
        uint64_t sb[MATCH_PER_THREAD], lb[MATCH_PER_THREAD];
        uint32_t sid[MATCH_PER_THREAD];
        bool asm_[MATCH_PER_THREAD];
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            sb[k] = lb[k] = 0;
            sid[k] = 0;
            asm_[k] = true;
            if (live[k]) {
                const uint64_t a0 = m.A.bm_begin[av[k]], a1 = m.A.bm_begin[av[k] + 1];
                const uint64_t b0 = m.B.bm_begin[bv[k]], b1 = m.B.bm_begin[bv[k] + 1];
                asm_[k] = a1 - a0 <= b1 - b0;
                sb[k] = asm_[k] ? a0 : b0;
                lb[k] = asm_[k] ? b0 : a0;
                sid[k] = asm_[k] ? bv[k] : av[k];
            }
        }
        uint16_t key[MATCH_PER_THREAD];
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            tg[k] -= rel[pos[k]];  // the candidate's position in its pair
            key[k] = 0;
            if (live[k]) key[k] = asm_[k] ? m.A.keys[sb[k] + tg[k]] : m.B.keys[sb[k] + tg[k]];
        }
        uint64_t xw[MATCH_PER_THREAD];
        uint32_t xr[MATCH_PER_THREAD];
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            xw[k] = 0;
            xr[k] = 0;
            if (live[k]) {
                // the key index of the side with more keys (the searched one)
                const uint8_t* ix = (asm_[k] ? m.B.kidx : m.A.kidx) + (uint64_t)sid[k] * RG_KEY_INDEX_BYTES;
                const uint32_t wi = key[k] >> 6;
                xw[k] = reinterpret_cast<const uint64_t*>(ix)[wi];
                xr[k] = reinterpret_cast<const uint16_t*>(ix + 8 * KIDX_WORDS)[wi];
            }
        }
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            if (!live[k]) continue;
            const uint32_t j = kidx_lookup(xw[k], xr[k], key[k]);
            Task& task = o[k].task;
            task.pair = (uint32_t)(m.pair0 + pl_lo + pos[k]);
            task.key = key[k];
            if (j != NONE) {
                task.kind = KIND_MATCH;
                task.ia = (uint32_t)(asm_[k] ? sb[k] + tg[k] : lb[k] + j);
                task.ib = (uint32_t)(asm_[k] ? lb[k] + j : sb[k] + tg[k]);
            }
            o[k].slot = t0 + (uint64_t)k * 256 + threadIdx.x;
        }
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k)
            if (o[k].slot != NONE) finish_slot(m, cnt, o[k]);
    } else {
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            const uint64_t t = t0 + (uint64_t)k * 256 + threadIdx.x;
            if (t < n_cand) match_slot_global(m, t, pl_lo, pl_hi, cnt, o[k]);
        }
    }
}

// Key matching of a wave of candidate slots into task records and per-block
// bin counts (the binned path).
__global__ void __launch_bounds__(256) k_match(MatchArgs m) {
    __shared__ uint32_t cnt[NBINS];
    __shared__ uint32_t pl_range[2];
    __shared__ MatchLds lds;
    __shared__ uint32_t lwin[2];  // first index of the staged window in the searched list, and its end
    SlotOutcome o[MATCH_PER_THREAD];
    match_block(m, m.n_cand, (uint64_t)blockIdx.x * MATCH_SLOTS, cnt, pl_range, lwin, lds, o);
    if (m.fuse_thread) {
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) wave_aggregate_add(m.acc, o[k].fused_pair, o[k].fused_inter);
    }
    __syncthreads();
    if (threadIdx.x < NBINS) m.blk_cnt[(uint64_t)threadIdx.x * gridDim.x + blockIdx.x] = cnt[threadIdx.x];
    // With fusion, the tasks of a block that lists nothing are never read
    // (binning skips such blocks), so they are not written.
    uint32_t listed = 0;
    for (int b = 0; b < NBINS; ++b) listed += b == BIN_FUSED ? 0u : cnt[b];
    if (listed || !m.fuse_thread) {
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k)
            if (o[k].slot != NONE) m.tasks[o[k].slot] = o[k].task;
    }
}

void launch_match(const MatchArgs& m, hipStream_t st) {
    if (!m.n_cand) return;
    hipLaunchKernelGGL(k_match, dim3(match_blocks(m.n_cand)), dim3(256), 0, st, m);
}

// ------------------------------------------------------------------ fused count
// Count-only calls without a host round trip. One kernel matches the keys of
// every pair and counts every matched container pair, block by block, so no
// task list, binning or per-bin launch is needed and the number of candidate
// keys (device value cand_off[n_pairs]) never goes to the host. Each workgroup
// takes blocks of MATCH_SLOTS candidate slots from a work counter until none
// is left. In a block, key matching counts the small-array pairs in place (as
// in the binned path) and lists every other matched pair in LDS: workgroup
// items (generic LDS expansion, merge path) run one after the other on the
// whole workgroup; wave items (bitset pairs, galloping search, bitset probes,
// run merges) are taken by the four waves from an LDS counter. The kernel
// accumulates |A n B| per pair whatever operation was asked for (the other
// counts follow from the Section 5.9 identities).
// The listed container pairs of a block, as separate arrays (13 B per item
// instead of a 16-byte task), so that the kernel's shared block stays under
// 32 KiB and five workgroups fit on a compute unit
struct FusedItems {
    uint32_t pair[MATCH_SLOTS];
    uint32_t ia[MATCH_SLOTS];
    uint32_t ib[MATCH_SLOTS];
    uint8_t bin[MATCH_SLOTS];
    __device__ __forceinline__ void put(uint32_t i, const Task& t) {
        pair[i] = t.pair;
        ia[i] = t.ia;
        ib[i] = t.ib;
        bin[i] = t.bin;
    }
    // item i read by every lane of a wave, with all fields uniform
    __device__ __forceinline__ Task get(uint32_t i) const {
        Task t{};
        t.pair = uniform(pair[i]);
        t.ia = uniform(ia[i]);
        t.ib = uniform(ib[i]);
        t.bin = (uint8_t)uniform(bin[i]);
        t.kind = KIND_MATCH;
        return t;
    }
};

struct FusedShared {
    FusedItems items;  // workgroup items from the front, wave items from the back
    union {
        WgShared sh;    // processing
        MatchLds m;     // key matching's staged window or key-index words
    } u;
    uint32_t cnt[NBINS];
    uint32_t pl_range[2];
    uint32_t lwin[2];
    uint32_t blk, n_wg, n_wv, next_wv;
};

// Five waves per SIMD (the compiler keeps the kernel within 96 VGPRs): more
// candidate lookups in flight; measured 88.3 -> 79.1 ms on the 1e6-pair
// uneven batch against four waves per SIMD.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_count_fused(MatchArgs m, uint32_t* next_blk) {
    __shared__ FusedShared f;
    const uint32_t lane = lane_id();
    uint64_t matched = 0;  // m.matched: this thread's matched candidates
    const uint64_t n_cand = uniform64(m.cand_off[m.n_pairs]);
    const uint64_t nblk = (n_cand + MATCH_SLOTS - 1) / MATCH_SLOTS;
    for (;;) {
        if (threadIdx.x == 0) {
            f.blk = atomicAdd(next_blk, 1u);
            f.n_wg = 0;
            f.n_wv = 0;
            f.next_wv = 0;
        }
        __syncthreads();
        const uint32_t blk = uniform(f.blk);
        if (blk >= nblk) {  // the same value in every thread: the whole workgroup leaves
            if (m.matched) {
                const uint64_t t = wave_sum_u64(matched);
                if (lane == 0 && t) atomicAdd(m.matched, (unsigned long long)t);
            }
            break;
        }
        SlotOutcome o[MATCH_PER_THREAD];
        match_block(m, n_cand, (uint64_t)blk * MATCH_SLOTS, f.cnt, f.pl_range, f.lwin, f.u.m, o);
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) wave_aggregate_add(m.acc, o[k].fused_pair, o[k].fused_inter);
        if (m.matched) {
            // matched container pairs of the block (counted in place or listed
            // below), summed per thread; one atomic per wave when the kernel ends
#pragma unroll
            for (int k = 0; k < (int)MATCH_PER_THREAD; ++k)
                matched += (o[k].task.kind == KIND_MATCH || o[k].fused_pair != NONE) ? 1u : 0u;
        }
#pragma unroll
        for (int k = 0; k < (int)MATCH_PER_THREAD; ++k) {
            if (o[k].task.kind != KIND_MATCH) continue;
            const uint8_t b = o[k].task.bin;
            if (b == BIN_GEN || b == BIN_AA) f.items.put(atomicAdd(&f.n_wg, 1u), o[k].task);
            else f.items.put(MATCH_SLOTS - 1 - atomicAdd(&f.n_wv, 1u), o[k].task);
        }
        __syncthreads();  // the lists are complete; the staged key window is no longer needed
        const uint32_t n_wg = uniform(f.n_wg), n_wv = uniform(f.n_wv);
        for (uint32_t i = 0; i < n_wg; ++i) {
            const Task t = f.items.get(i);
            uint32_t c;
            if (t.bin == BIN_GEN) {
                c = generic_count_wg<RG_AND>(m.A, m.B, t, f.u.sh);
            } else {
                c = merge_inter_wg(m.A, m.B, t, reinterpret_cast<uint16_t*>(f.u.sh.sa),
                                   reinterpret_cast<uint16_t*>(f.u.sh.sb), f.u.sh.tmp64);
            }
            if (threadIdx.x == 0) acc_add(m.acc, t.pair, (long long)c);
            __syncthreads();
        }
        for (;;) {
            // lane 0 takes the next item; readlane makes the index a scalar, so
            // the loop exit is one branch for the whole wave
            uint32_t v = 0;
            if (lane == 0) v = atomicAdd(&f.next_wv, 1u);
            const uint32_t i = __builtin_amdgcn_readlane(v, 0);
            if (i >= n_wv) break;
            const Task t = f.items.get(MATCH_SLOTS - 1 - i);
            const uint32_t c = t.bin == BIN_BB ? bb_count_wave<RG_AND>(m.A, m.B, t, lane) : wave_inter(m.A, m.B, t, lane);
            if (lane == 0) acc_add(m.acc, t.pair, (long long)c);
        }
        __syncthreads();  // every wave is done with this block's lists
    }
}

// workgroups of the fused kernel that are resident on one compute unit at once
uint32_t count_fused_blocks_per_cu() {
    static int nb = 0;
    if (!nb && hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_count_fused, 256, 0) != hipSuccess) nb = 4;
    return nb > 0 ? (uint32_t)nb : 4u;
}

void launch_count_fused(const MatchArgs& m, uint32_t* next_blk, uint32_t grid, hipStream_t st) {
    if (!m.n_pairs || !grid) return;
    hipLaunchKernelGGL(k_count_fused, dim3(grid), dim3(256), 0, st, m, next_blk);
}

// ------------------------------------------------------------------ binning
// bin counts and offsets from the scanned per-block counts
__global__ void k_bin_totals(const uint64_t* blk_off, uint32_t nblk, const uint64_t* total, uint32_t* bin_info,
                             uint32_t* next) {
    const uint32_t b = threadIdx.x;
    if (b >= NBINS) return;
    const uint64_t o = blk_off[(uint64_t)b * nblk];
    const uint64_t e = b + 1 < NBINS ? blk_off[(uint64_t)(b + 1) * nblk] : *total;
    bin_info[b] = (uint32_t)(e - o);
    bin_info[NBINS + b] = (uint32_t)o;
    if (next) next[b] = 0;
}

void launch_bin_layout(const uint32_t* blk_cnt, uint32_t nblk, uint64_t* blk_off, uint64_t* partials, uint64_t* total,
                       uint32_t* bin_info, uint32_t* next, hipStream_t st) {
    launch_scan_u32_u64(blk_cnt, blk_off, (uint64_t)NBINS * nblk, 0, partials, total, st);
    hipLaunchKernelGGL(k_bin_totals, dim3(1), dim3(64), 0, st, (const uint64_t*)blk_off, nblk, (const uint64_t*)total,
                       bin_info, next);
}

// Slot ids into per-bin lists: the same MATCH_SLOTS-slot blocks as k_match, each
// block's slots of bin b go to blk_off[b][block] + rank (rank from LDS atomics).
// A block whose counts list nothing returns at once (its tasks may be unwritten).
__global__ void __launch_bounds__(256) k_bin_scatter(const Task* tasks, uint64_t n, const uint32_t* blk_cnt,
                                                     const uint64_t* blk_off, uint32_t* lists) {
    __shared__ uint32_t cnt[NBINS];
    __shared__ uint32_t listed;
    if (threadIdx.x < NBINS) cnt[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        uint32_t l = 0;
        for (int b = 0; b < NBINS; ++b)
            if (b != BIN_FUSED) l += blk_cnt[(uint64_t)b * gridDim.x + blockIdx.x];
        listed = l;
    }
    __syncthreads();
    if (uniform(listed) == 0) return;
#pragma unroll
    for (uint32_t k = 0; k < MATCH_PER_THREAD; ++k) {
        const uint64_t s = (uint64_t)blockIdx.x * MATCH_SLOTS + k * 256 + threadIdx.x;
        if (s < n) {
            const Task t = tasks[s];
            if (t.kind != KIND_NOOP) {
                const uint32_t rank = atomicAdd(&cnt[t.bin], 1u);
                lists[blk_off[(uint64_t)t.bin * gridDim.x + blockIdx.x] + rank] = (uint32_t)s;
            }
        }
    }
}

void launch_bin_scatter(const Task* tasks, uint64_t n, const uint32_t* blk_cnt, const uint64_t* blk_off,
                        uint32_t* bin_lists, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(k_bin_scatter, dim3(match_blocks(n)), dim3(256), 0, st, tasks, n, blk_cnt, blk_off, bin_lists);
}

// ------------------------------------------------------------------ scan
// Three-phase exclusive scan: per-tile sums, a single-block scan of the tile
// sums, then a per-tile rescan. Tile = 256 threads x 8 items.
constexpr uint32_t SCAN_PER_THREAD = 8;
constexpr uint32_t SCAN_TILE = 256 * SCAN_PER_THREAD;

size_t scan_partials_needed(uint64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

// NZ: the scanned value of element i is (in[i] != 0) rather than in[i]
template <bool NZ>
__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t* in, uint64_t n, uint64_t* partials) {
    __shared__ uint64_t tmp[4];
    uint64_t start = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_PER_THREAD; ++k)
        if (start + k < n) s += NZ ? (in[start + k] != 0u ? 1u : 0u) : in[start + k];
    s = block_sum_u64(s, tmp);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_scan_partials(uint64_t* partials, uint64_t nb, uint64_t base,
                                                       const uint64_t* base_dev, uint64_t* total_out) {
    __shared__ uint64_t tmp[256];
    // base_dev may be total_out itself: it is read here, before any barrier,
    // and written only at the end
    uint64_t carry = base + (base_dev ? *base_dev : 0);
    for (uint64_t c0 = 0; c0 < nb; c0 += 256) {
        uint64_t i = c0 + threadIdx.x;
        uint64_t v = i < nb ? partials[i] : 0;
        tmp[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan in LDS (256 entries)
        for (uint32_t o = 1; o < 256; o <<= 1) {
            uint64_t x = threadIdx.x >= o ? tmp[threadIdx.x - o] : 0;
            __syncthreads();
            tmp[threadIdx.x] += x;
            __syncthreads();
        }
        if (i < nb) partials[i] = carry + tmp[threadIdx.x] - v;
        uint64_t tot = tmp[255];
        __syncthreads();
        carry += tot;
    }
    __syncthreads();  // every thread has read base_dev before total_out is written
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <bool NZ>
__global__ void __launch_bounds__(256) k_scan_down(const uint32_t* in, uint64_t n, const uint64_t* partials,
                                                   uint64_t* out) {
    __shared__ uint64_t tmp[4];
    uint64_t start = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_PER_THREAD; ++k) {
        v[k] = start + k < n ? (NZ ? (in[start + k] != 0u ? 1u : 0u) : in[start + k]) : 0;
        s += v[k];
    }
    // block exclusive scan of per-thread sums (64-bit)
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    uint64_t inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t x = __shfl_up(inc, o);
        if (lane >= (uint32_t)o) inc += x;
    }
    if (lane == 63) tmp[wid] = inc;
    __syncthreads();
    uint64_t wbase = 0;
    for (uint32_t w = 0; w < wid; ++w) wbase += tmp[w];
    uint64_t run = partials[blockIdx.x] + wbase + inc - s;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_PER_THREAD; ++k) {
        if (start + k < n) out[start + k] = run;
        run += v[k];
    }
}

// one tile: the whole scan in one workgroup (small inputs: one launch, not three)
template <bool NZ>
__global__ void __launch_bounds__(256) k_scan_single(const uint32_t* in, uint64_t n, uint64_t base,
                                                     const uint64_t* base_dev, uint64_t* out, uint64_t* total_out) {
    __shared__ uint64_t tmp[4];
    base += base_dev ? *base_dev : 0;  // read before the barrier; total_out (maybe the same word) after it
    const uint64_t start = (uint64_t)threadIdx.x * SCAN_PER_THREAD;
    uint32_t v[SCAN_PER_THREAD];
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_PER_THREAD; ++k) {
        v[k] = start + k < n ? (NZ ? (in[start + k] != 0u ? 1u : 0u) : in[start + k]) : 0;
        s += v[k];
    }
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    uint64_t inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t x = __shfl_up(inc, o);
        if (lane >= (uint32_t)o) inc += x;
    }
    if (lane == 63) tmp[wid] = inc;
    __syncthreads();
    uint64_t wbase = 0;
    for (uint32_t w = 0; w < wid; ++w) wbase += tmp[w];
    uint64_t run = base + wbase + inc - s;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_PER_THREAD; ++k) {
        if (start + k < n) out[start + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255 && total_out) *total_out = base + wbase + inc;
}

// total_out = base + *base_dev (an empty scan)
__global__ void k_scan_empty(uint64_t base, const uint64_t* base_dev, uint64_t* total_out) {
    *total_out = base + (base_dev ? *base_dev : 0);
}

template <bool NZ>
static void launch_scan(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t base, uint64_t* partials,
                        uint64_t* total_out, hipStream_t st, const uint64_t* base_dev) {
    uint64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 0) {
        if (total_out) hipLaunchKernelGGL(k_scan_empty, dim3(1), dim3(1), 0, st, base, base_dev, total_out);
        return;
    }
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_single<NZ>, dim3(1), dim3(256), 0, st, in, n, base, base_dev, out, total_out);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce<NZ>, dim3((uint32_t)nb), dim3(256), 0, st, in, n, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(256), 0, st, partials, nb, base, base_dev, total_out);
    hipLaunchKernelGGL(k_scan_down<NZ>, dim3((uint32_t)nb), dim3(256), 0, st, in, n, partials, out);
}

void launch_scan_u32_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t base, uint64_t* partials,
                         uint64_t* total_out, hipStream_t st, const uint64_t* base_dev) {
    launch_scan<false>(in, out, n, base, partials, total_out, st, base_dev);
}

void launch_scan_nonzero_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t base, uint64_t* partials,
                             uint64_t* total_out, hipStream_t st, const uint64_t* base_dev) {
    launch_scan<true>(in, out, n, base, partials, total_out, st, base_dev);
}

}  // namespace rg
