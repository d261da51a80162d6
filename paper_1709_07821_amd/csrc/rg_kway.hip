// rg_kway.hip - k-way intersection and union of bitmaps of one pool, for many
// queries at once (the building block of the serving loop).
//
// The paper folds many bitmaps pairwise or aggregates lazily (Section 5.9,
// wide unions; lazy aggregation, Section 2.2). Here a query's result is built
// key by key, each key by one workgroup, so no intermediate bitmap is ever
// written:
//   1. k_kw_keys: one workgroup per query builds the query's result key set as
//      a 65536-bit LDS mask (AND of the bitmaps' key masks, or OR), writes the
//      keys in ascending order as one task per result key, and marks the rest
//      of the query's slot range empty (k_kw_keys_small: the same for queries
//      of one or two bitmaps with few keys, one wave each).
//   2. k_kw_bounds: one wave per slot looks the key up in the k bitmaps (one
//      lane per bitmap) and bounds the result payload (AND: the smallest
//      container, OR: the sum, both capped at a bitset) - the slot sizes of
//      step 3. Materialised slots of one or two bitmaps with an array side
//      (small_mat_ok) are marked for the one-wave array kernel (rg_small.hip).
//   3. k_kw_eval: one workgroup per remaining result key. Intersection: every container
//      is expanded into an LDS bitset and combined word by word, stopping once
//      the running result is empty. Union, symmetric difference, difference:
//      bitset containers are combined in registers (each thread owns four
//      result words), then all array and run containers fold into the LDS
//      bitset at once (an LDS atomic per value or run). Then the common output
//      step (P1 type, payload into the slot) or, count-only, the population
//      count.
// Compaction of non-empty results into per-query bitmaps uses the pairwise
// path's kernels (flags, scan, compact, bitmap starts).
#include "rg_count_dev.h"

namespace rg {

constexpr int KW_UNROLL = 4;  // independent loads in flight per thread in the key and fold passes
constexpr uint32_t KW_BS_BATCH = 8;    // bitset containers whose words a fold loads at once
constexpr uint64_t KW_EVAL_FEW = 8192;  // slots up to which each gets its own evaluation workgroup
// KwArgs.eval_chunk: slots whose tasks an evaluation workgroup reads at once
// (at most 64; 0: chosen by the launcher). A chunk's keys are built one after
// another, so chunks add their latencies: with few slots (at most
// KW_EVAL_FEW, about what the GPU holds at once) every slot gets its own
// workgroup; with many, chunks of 4 save workgroup starts and task reads
// (measured on pairwise calls: 1, 4, 16; on k-way steps of 1e3 to 2.5e5 slots).

// The pool of a query's j-th bitmap, selected field by field (plain pointer
// selects; no address arithmetic on the kernel-argument block).
__device__ __forceinline__ PoolView kw_side(const KwArgs& a, bool second) {
    PoolView v;
    v.bm_begin = second ? a.P1.bm_begin : a.P0.bm_begin;
    v.keys = second ? a.P1.keys : a.P0.keys;
    v.types = second ? a.P1.types : a.P0.types;
    v.card = second ? a.P1.card : a.P0.card;
    v.size = second ? a.P1.size : a.P0.size;
    v.off = second ? a.P1.off : a.P0.off;
    v.payload = second ? a.P1.payload : a.P0.payload;
    v.bm_card = second ? a.P1.bm_card : a.P0.bm_card;
    v.bm_wbytes = second ? a.P1.bm_wbytes : a.P0.bm_wbytes;
    v.meta = second ? a.P1.meta : a.P0.meta;
    v.kidx = second ? a.P1.kidx : a.P0.kidx;
    return v;
}

// ---------------------------------------------------------------- 1. keys
// Queries of one or two bitmaps with at most KW_KEYS_SMALL keys together are
// built by k_kw_keys_small, one wave per query: the two sorted key lists,
// staged in LDS, are walked in merged order (union and symmetric difference)
// or the first list is filtered (intersection: keys the second list holds;
// difference: all of them), 64 keys per round; a ballot gives each result key
// its slot. The workgroup kernel below takes the other queries.
constexpr uint32_t KW_KEYS_SMALL = 1024;
constexpr uint32_t KW_KEYS_CHUNK = 8;  // most queries whose sizes the workgroup kernel reads at once

__global__ void __launch_bounds__(256) k_kw_keys_small(KwArgs a) {
    __shared__ uint16_t lk[4][KW_KEYS_SMALL + 8];
    const uint32_t wid = threadIdx.x >> 6, lane = lane_id();
    const uint32_t q = wave_index();
    if (q >= a.n_queries) return;
    const KwQuery Q = a.queries[q];
    const uint32_t op = uniform(Q.op), k = uniform(Q.k), ids0 = uniform(Q.ids_off);
    if (k > 2) return;
    const uint64_t slot0 = uniform64(Q.slot0);
    const uint32_t kbound = uniform(Q.kbound);
    const uint32_t b0 = uniform(a.ids[ids0]);
    const uint64_t s0 = uniform64(a.P0.bm_begin[b0]);
    const uint32_t n0 = uniform((uint32_t)(a.P0.bm_begin[b0 + 1] - s0));
    uint64_t s1 = 0;
    uint32_t n1 = 0;
    if (k == 2) {
        const uint32_t b1 = uniform(a.ids[ids0 + 1]);
        s1 = uniform64(a.P1.bm_begin[b1]);
        n1 = uniform((uint32_t)(a.P1.bm_begin[b1 + 1] - s1));
    }
    if (n0 + n1 > KW_KEYS_SMALL) return;  // the workgroup kernel's
    uint16_t* A = lk[wid];
    uint16_t* B = lk[wid] + ((n0 + 7u) & ~7u);
    for (uint32_t i = lane; i < n0; i += 64) A[i] = a.P0.keys[s0 + i];
    for (uint32_t i = lane; i < n1; i += 64) B[i] = a.P1.keys[s1 + i];
    __builtin_amdgcn_wave_barrier();
    const bool merge = op == RG_OR || op == RG_XOR;
    const uint32_t n = merge ? n0 + n1 : n0;
    uint32_t pos = 0;
    for (uint32_t base = 0; base < n; base += 64) {
        const uint32_t p = base + lane;
        bool keep = false;
        uint32_t key = 0, ia = NONE, ib = NONE;
        if (p < n) {
            if (merge) {
                // merge path: i = keys of the first list among the first p
                uint32_t lo = p > n1 ? p - n1 : 0u, hi = p < n0 ? p : n0;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (A[mid] <= B[p - 1 - mid]) lo = mid + 1;
                    else hi = mid;
                }
                const uint32_t i = lo, j = p - lo;
                if (i < n0 && (j >= n1 || A[i] <= B[j])) {
                    key = A[i];
                    ia = (uint32_t)(s0 + i);
                    if (j < n1 && B[j] == key) ib = (uint32_t)(s1 + j);
                    keep = true;
                } else {
                    key = B[j];
                    ib = (uint32_t)(s1 + j);
                    keep = !(i > 0 && A[i - 1] == key);  // else listed with the first list's copy
                }
            } else {
                key = A[p];
                ia = (uint32_t)(s0 + p);
                uint32_t lo = 0, hi = n1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (B[mid] < key) lo = mid + 1;
                    else hi = mid;
                }
                const bool in_b = lo < n1 && B[lo] == key;
                if (in_b) ib = (uint32_t)(s1 + lo);
                keep = op == RG_AND && k == 2 ? in_b : true;  // one bitmap: its own keys
            }
        }
        const uint64_t bal = __ballot(keep);
        const uint32_t at = pos + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        if (keep && at < kbound) {
            Task t;
            t.pair = a.pair_base + q;
            t.ia = ia;
            t.ib = ib;
            t.key = (uint16_t)key;
            t.kind = KIND_MATCH;
            t.bin = KW_TASK_INDEXED;
            a.tasks[slot0 + at] = t;
        }
        pos += (uint32_t)__popcll(bal);
    }
    pos = uniform(pos);
    for (uint32_t i = (pos < kbound ? pos : kbound) + lane; i < kbound; i += 64) {
        Task t;
        t.pair = a.pair_base + q;
        t.ia = NONE;
        t.ib = NONE;
        t.key = 0;
        t.kind = KIND_NOOP;
        t.bin = 0;
        a.tasks[slot0 + i] = t;
    }
    if (lane == 0 && pos > kbound) atomicOr(a.err, 1u);
}

constexpr uint32_t KW_KEY_UNROLL = 16;  // keys per thread per round of a multi-bitmap key pass

// Sets the key bits of the query's bitmaps j0 .. j1-1 (key lists at rs[j],
// rn[j]) in one pass over their concatenated lists: into masks[j - j0] when
// per_bitmap, else all into masks[0]. Each thread takes KW_KEY_UNROLL
// consecutive keys per round (their loads issued together); sorted lists put
// most of them in one or two 64-key words, so the thread ORs their bits
// together and issues one LDS atomic per word it touches (the keys of many
// bitmaps over a small universe otherwise pile onto a few words). roff gets
// the exclusive prefix of the lengths. Ends with a barrier.
__device__ void kw_fill_keys(const KwArgs& a, const uint64_t* rs, const uint32_t* rn, uint32_t* roff, uint32_t j0,
                             uint32_t j1, uint64_t (*masks)[1024], bool per_bitmap) {
    const uint32_t tid = threadIdx.x, m = j1 - j0;
    if (tid == 0) {
        uint32_t o = 0;
        for (uint32_t j = 0; j < m; ++j) {
            roff[j] = o;
            o += rn[j0 + j];
        }
        roff[m] = o;
    }
    __syncthreads();
    const uint32_t total = uniform(roff[m]);
    // the bitmap holding the thread's current position and its range in the
    // concatenated order, kept in registers: positions only grow, so the
    // bitmap only moves forward (a few LDS reads per round, not one per key)
    uint32_t jj = 0, lo_off = 0, hi_off = roff[1];
    const uint16_t* src = nullptr;  // the bitmap's key list
    auto enter = [&](uint32_t i) {
        while (hi_off <= i) {
            ++jj;
            lo_off = hi_off;
            hi_off = roff[jj + 1];
        }
        const uint32_t j = j0 + jj;
        src = (j ? a.P1.keys : a.P0.keys) + rs[j];
    };
    for (uint32_t base = 0; base < total; base += 256 * KW_KEY_UNROLL) {
        const uint32_t i0 = base + tid * KW_KEY_UNROLL;
        if (i0 < total) enter(i0);
        uint32_t key[KW_KEY_UNROLL], mi[KW_KEY_UNROLL];
#pragma unroll
        for (uint32_t r = 0; r < KW_KEY_UNROLL; ++r) {
            const uint32_t i = i0 + r;
            key[r] = 0xFFFFFFFFu;
            mi[r] = 0;
            if (i < total) {
                if (i >= hi_off) enter(i);
                key[r] = src[i - lo_off];
                mi[r] = per_bitmap ? jj : 0u;
            }
        }
        // runs of keys in the same word of the same mask: one atomic each
        uint32_t cw = 0xFFFFFFFFu, cm = 0;
        uint64_t bits = 0;
#pragma unroll
        for (uint32_t r = 0; r < KW_KEY_UNROLL; ++r) {
            if (key[r] == 0xFFFFFFFFu) continue;
            const uint32_t w = key[r] >> 6;
            if (w != cw || mi[r] != cm) {
                if (bits) atomicOr(reinterpret_cast<unsigned long long*>(&masks[cm][cw]), bits);
                cw = w;
                cm = mi[r];
                bits = 0;
            }
            bits |= 1ull << (key[r] & 63);
        }
        if (bits) atomicOr(reinterpret_cast<unsigned long long*>(&masks[cm][cw]), bits);
    }
    __syncthreads();
}

// Key masks straight from the pools' key-presence indexes (1024 presence
// words per bitmap, the key set as a bitset): thread t gets words 4t..4t+3 of
// the AND (and_) or the OR of the presence words of the query's bitmaps
// j0 .. j1-1, KW_BS_BATCH bitmaps' words in flight at a time.
__device__ void kw_pres_words(const KwArgs& a, uint32_t ids0, uint32_t j0, uint32_t j1, bool and_,
                              uint64_t (&r)[4]) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = and_ ? ~0ull : 0ull;
    for (uint32_t b0 = j0; b0 < j1; b0 += KW_BS_BATCH) {
        u32x4 v0[KW_BS_BATCH], v1[KW_BS_BATCH];
#pragma unroll
        for (uint32_t u = 0; u < KW_BS_BATCH; ++u) {
            const uint32_t j = b0 + u;
            if (j < j1) {
                const uint8_t* ix = (j ? a.P1.kidx : a.P0.kidx) + (uint64_t)a.ids[ids0 + j] * RG_KEY_INDEX_BYTES;
                const u32x4* src = reinterpret_cast<const u32x4*>(ix) + 2 * tid;
                v0[u] = src[0];
                v1[u] = src[1];
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < KW_BS_BATCH; ++u) {
            if (b0 + u < j1) {
                const uint64_t x[4] = {(uint64_t)v0[u].x | ((uint64_t)v0[u].y << 32),
                                       (uint64_t)v0[u].z | ((uint64_t)v0[u].w << 32),
                                       (uint64_t)v1[u].x | ((uint64_t)v1[u].y << 32),
                                       (uint64_t)v1[u].z | ((uint64_t)v1[u].w << 32)};
#pragma unroll
                for (int q = 0; q < 4; ++q) r[q] = and_ ? (r[q] & x[q]) : (r[q] | x[q]);
            }
        }
    }
}

// Position of the r-th set bit (r < popcount) of x.
__device__ __forceinline__ uint32_t kw_select_bit(uint64_t x, uint32_t r) {
    uint32_t bit = 0;
#pragma unroll
    for (uint32_t w = 32; w >= 1; w >>= 1) {
        const uint32_t c = (uint32_t)__popcll(x & ((1ull << w) - 1ull));
        if (r >= c) {
            r -= c;
            x >>= w;
            bit += w;
        }
    }
    return bit;
}

// Writes query q's result keys (the set bits of the result words, ascending)
// as one task per key into its slot range, and no-op tasks into the rest of the
// range. The result words: acc, or with at most two bitmaps (indexed) the
// combination of the two bitmaps' key masks acc and cur, and then each task
// also records the positions of its containers. Keys are handed out by rank,
// not by word: the per-word prefix counts go to LDS (wp: 3 x 1024 entries),
// and thread t builds the tasks of ranks t, t + 256, ... (a binary search of
// the prefixes, then the rank's bit in its word), so a key set packed into a
// few words is spread over the whole workgroup.
__device__ void kw_emit_tasks(const KwArgs& a, uint32_t q, uint32_t op, uint32_t k, uint64_t slot0, uint32_t kbound,
                              const uint64_t* acc, const uint64_t* cur, const uint64_t* rs, bool indexed,
                              uint32_t* tmp, uint16_t* wp) {
    const uint32_t tid = threadIdx.x;
    const bool two = indexed && k == 2;
    auto result_word = [&](uint64_t m0, uint64_t m1) {
        return !indexed || k == 1 ? m0 : op == RG_AND ? (m0 & m1) : op == RG_ANDNOT ? m0 : (m0 | m1);
    };
    uint64_t w[4], m0[4], m1[4];
    uint32_t c = 0, c0 = 0, c1 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        m0[j] = acc[4 * tid + j];
        m1[j] = two ? cur[4 * tid + j] : 0ull;
        w[j] = result_word(m0[j], m1[j]);
        c += __popcll(w[j]);
        c0 += __popcll(m0[j]);
        c1 += __popcll(m1[j]);
    }
    uint32_t total;
    uint32_t pos = block_excl_scan_u32(c, tmp, &total);
    // with recorded positions: ranks of this thread's first word in each key mask
    uint32_t r0 = 0, r1 = 0, unused;
    if (indexed) {
        r0 = block_excl_scan_u32(c0, tmp, &unused);
        r1 = block_excl_scan_u32(c1, tmp, &unused);
    }
    // per-word exclusive prefixes (at most 65 472: the prefix of the last word)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        wp[4 * tid + j] = (uint16_t)pos;
        pos += __popcll(w[j]);
        if (indexed) {
            wp[1024 + 4 * tid + j] = (uint16_t)r0;
            wp[2048 + 4 * tid + j] = (uint16_t)r1;
            r0 += __popcll(m0[j]);
            r1 += __popcll(m1[j]);
        }
    }
    __syncthreads();
    // total <= kbound holds by construction of the host bound; guard anyway
    const uint32_t used = total < kbound ? total : kbound;
    for (uint32_t p = tid; p < used; p += 256) {
        // the last word whose prefix is <= p holds rank p
        uint32_t lo = 0, hi = 1024;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (wp[mid] <= p) lo = mid;
            else hi = mid;
        }
        const uint64_t x0 = acc[lo], x1 = two ? cur[lo] : 0ull;
        const uint32_t b = kw_select_bit(result_word(x0, x1), p - wp[lo]);
        Task t;
        t.pair = a.pair_base + q;
        t.ia = NONE;
        t.ib = NONE;
        t.key = (uint16_t)(lo * 64 + b);
        t.kind = KIND_MATCH;
        t.bin = 0;
        if (indexed) {
            // container index = list start + number of the bitmap's keys below this one
            const uint64_t below = (1ull << b) - 1ull;
            if ((x0 >> b) & 1ull) t.ia = (uint32_t)(rs[0] + wp[1024 + lo] + __popcll(x0 & below));
            if ((x1 >> b) & 1ull) t.ib = (uint32_t)(rs[1] + wp[2048 + lo] + __popcll(x1 & below));
            t.bin = KW_TASK_INDEXED;
        }
        a.tasks[slot0 + p] = t;
    }
    for (uint32_t i = used + tid; i < kbound; i += 256) {
        Task t;
        t.pair = a.pair_base + q;
        t.ia = NONE;
        t.ib = NONE;
        t.key = 0;
        t.kind = KIND_NOOP;
        t.bin = 0;
        a.tasks[slot0 + i] = t;
    }
    if (tid == 0 && total > kbound) atomicOr(a.err, 1u);
}

__global__ void __launch_bounds__(256) k_kw_keys(KwArgs a, uint32_t chunk) {
    __shared__ uint64_t accm[1][1024];
    __shared__ uint64_t grp[KW_AND_GROUP][1024];  // key masks of a group of bitmaps (intersection)
    uint64_t* acc = accm[0];
    uint64_t* cur = grp[0];
    __shared__ uint32_t tmp[8];
    __shared__ uint64_t rs[KW_MAX_K];  // key-list start of each of the query's bitmaps
    __shared__ uint32_t rn[KW_MAX_K];  // and its length
    __shared__ uint32_t roff[KW_MAX_K + 1];  // exclusive prefix of the lengths (union pass)
    __shared__ uint16_t wpre[3 * 1024];      // per-word key prefixes (task output)
    __shared__ uint32_t chunk_mask;
    // chunks of `chunk` queries: whether each is the workgroup kernel's (more
    // than two bitmaps, or more than KW_KEYS_SMALL keys) is read for the whole
    // chunk at once, then those queries are built one after another
    for (uint32_t c0 = blockIdx.x * chunk; c0 < a.n_queries; c0 += gridDim.x * chunk) {
    bool big = false;
    if (threadIdx.x < chunk && c0 + threadIdx.x < a.n_queries) {
        const KwQuery Q = a.queries[c0 + threadIdx.x];
        if (Q.flags & KW_SPLIT) {
            big = false;  // built by k_kw_keys_part
        } else if (Q.k > 2) {
            big = true;
        } else {
            const uint32_t b0 = a.ids[Q.ids_off];
            uint64_t n = a.P0.bm_begin[b0 + 1] - a.P0.bm_begin[b0];
            if (Q.k == 2) {
                const uint32_t b1 = a.ids[Q.ids_off + 1];
                n += a.P1.bm_begin[b1 + 1] - a.P1.bm_begin[b1];
            }
            big = n > KW_KEYS_SMALL;
        }
    }
    const uint64_t bm = __ballot(big);  // wave 0 holds the chunk
    if (threadIdx.x == 0) chunk_mask = (uint32_t)bm;
    __syncthreads();
    uint32_t todo = uniform(chunk_mask);
    __syncthreads();  // read before the next chunk writes it
    while (todo) {
    const uint32_t q = c0 + (uint32_t)__builtin_ctz(todo);
    todo &= todo - 1;
    const KwQuery Q = a.queries[q];
    const uint32_t op = uniform(Q.op), k = uniform(Q.k), ids0 = uniform(Q.ids_off);
    const uint64_t slot0 = uniform64(Q.slot0);
    const uint32_t kbound = uniform(Q.kbound);
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < 1024; i += 256) acc[i] = 0;
    // all key ranges at once (one load level instead of one per bitmap)
    const uint32_t kk = op == RG_ANDNOT ? 1u : k;  // bitmaps that decide the result keys
    // With at most two bitmaps each result key's containers are recorded in its
    // task (positions from the two key masks), so the later kernels need no search.
    const bool indexed = k <= 2;
    const bool pres = a.P0.kidx != nullptr && a.P1.kidx != nullptr;  // key masks from presence indexes
    for (uint32_t j = tid; (indexed || !pres) && j < (indexed ? k : kk); j += 256) {
        const uint64_t* bmb = j ? a.P1.bm_begin : a.P0.bm_begin;
        const uint32_t b = a.ids[ids0 + j];
        const uint64_t s0 = bmb[b];
        rs[j] = s0;
        rn[j] = (uint32_t)(bmb[b + 1] - s0);
    }
    __syncthreads();
    // result keys: AND - in every bitmap; OR, XOR - in any; ANDNOT - the first bitmap's
    if (pres) {
        // the key masks are the presence words: acc = bitmap 0 and cur =
        // bitmap 1 (at most two bitmaps), else the combination of the deciding ones
        uint64_t r[4];
        kw_pres_words(a, ids0, 0, indexed ? 1u : kk, op == RG_AND, r);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[4 * tid + q] = r[q];
        if (indexed && k == 2) {
            kw_pres_words(a, ids0, 1, 2, false, r);
#pragma unroll
            for (int q = 0; q < 4; ++q) cur[4 * tid + q] = r[q];
        }
        __syncthreads();
    } else if (indexed) {
        // the key masks of both bitmaps, side by side: acc = bitmap 0, cur = bitmap 1
        for (uint32_t i = tid; i < 1024; i += 256) cur[i] = 0;
        __syncthreads();
        for (uint32_t j = 0; j < k; ++j) {
            const uint16_t* pkeys = j ? a.P1.keys : a.P0.keys;
            const uint64_t s0 = rs[j];
            const uint32_t n = uniform(rn[j]);
            uint64_t* dst = j == 0 ? acc : cur;
            for (uint32_t base = 0; base < n; base += 256 * KW_UNROLL) {
                uint32_t key[KW_UNROLL];
#pragma unroll
                for (int r = 0; r < KW_UNROLL; ++r) {
                    const uint32_t i = base + r * 256 + tid;
                    key[r] = i < n ? pkeys[s0 + i] : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int r = 0; r < KW_UNROLL; ++r)
                    if (key[r] != 0xFFFFFFFFu)
                        atomicOr(reinterpret_cast<unsigned long long*>(&dst[key[r] >> 6]), 1ull << (key[r] & 63));
            }
        }
        __syncthreads();
    } else if (op != RG_AND) {
        // a union of key sets: every key of every deciding bitmap sets its bit,
        // in one pass over the concatenated lists
        kw_fill_keys(a, rs, rn, roff, 0, kk, accm, false);
    } else {
        // intersection: the first bitmap's keys, then groups of KW_AND_GROUP
        // bitmaps, each into its own mask in one pass, ANDed into the result
        kw_fill_keys(a, rs, rn, roff, 0, 1, accm, false);
        for (uint32_t j0 = 1; j0 < k; j0 += KW_AND_GROUP) {
            const uint32_t j1 = j0 + KW_AND_GROUP < k ? j0 + KW_AND_GROUP : k;
            for (uint32_t i = tid; i < (j1 - j0) * 1024; i += 256) grp[i >> 10][i & 1023] = 0;
            __syncthreads();
            kw_fill_keys(a, rs, rn, roff, j0, j1, grp, true);
            for (uint32_t i = tid; i < 1024; i += 256) {
                uint64_t x = acc[i];
                for (uint32_t g = 0; g < j1 - j0; ++g) x &= grp[g][i];
                acc[i] = x;
            }
            __syncthreads();
        }
    }
    kw_emit_tasks(a, q, op, k, slot0, kbound, acc, cur, rs, indexed, tmp, wpre);
    __syncthreads();  // LDS read before the next query's pass
    }
    }
}


// Split key passes (queries of many bitmaps, parts from the host): each
// workgroup builds the key set of its part's bitmaps in LDS (union: every key;
// intersection: keys of all of them) and ORs it into the query's key mask in
// device memory (an intersection ORs the complement, so that a zeroed mask
// serves both). The last part of a query to arrive (counted after a fence)
// reads the mask back and writes the query's tasks, as k_kw_keys does.
__global__ void __launch_bounds__(256) k_kw_keys_part(KwArgs a) {
    __shared__ uint64_t accm[1][1024];
    __shared__ uint64_t grp[KW_AND_GROUP][1024];
    uint64_t* acc = accm[0];
    __shared__ uint32_t tmp[8];
    __shared__ uint64_t rs[KW_MAX_K];
    __shared__ uint32_t rn[KW_MAX_K];
    __shared__ uint32_t roff[KW_MAX_K + 1];
    __shared__ uint16_t wpre[3 * 1024];
    __shared__ uint32_t last;
    const uint32_t tid = threadIdx.x;
    for (uint32_t p = blockIdx.x; p < a.n_parts; p += gridDim.x) {
        const KwPart P = a.parts[p];
        const uint32_t q = uniform(P.q), j0 = uniform(P.j01 & 0xFFFFu);
        const uint32_t mi = uniform(P.mi), n = uniform(P.n);
        const KwQuery Q = a.queries[q];
        const uint32_t op = uniform(Q.op), k = uniform(Q.k), ids0 = uniform(Q.ids_off);
        uint32_t j1 = uniform(P.j01 >> 16);
        const bool pres = a.P0.kidx != nullptr && a.P1.kidx != nullptr;
        // parts come from the host within these limits (an intersection part
        // without presence indexes: one LDS mask per bitmap); a part outside
        // them is cut to them (memory-safe) and reported
        if (j1 > k || j0 >= j1 || (!pres && op == RG_AND && j1 - j0 > KW_AND_GROUP)) {
            if (tid == 0) atomicOr(a.err, 1u);
            j1 = j1 > k ? k : j1;
            j1 = !pres && op == RG_AND && j1 > j0 + KW_AND_GROUP ? j0 + KW_AND_GROUP : j1;
        }
        for (uint32_t j = j0 + tid; !pres && j < j1; j += 256) {
            const uint64_t* bmb = j ? a.P1.bm_begin : a.P0.bm_begin;
            const uint32_t b = a.ids[ids0 + j];
            const uint64_t s0 = bmb[b];
            rs[j] = s0;
            rn[j] = (uint32_t)(bmb[b + 1] - s0);
        }
        for (uint32_t i = tid; i < 1024; i += 256) acc[i] = 0;
        __syncthreads();
        if (j0 >= j1) {
            // an empty part (only after a cut): adds no key, removes none
            for (uint32_t i = tid; i < 1024; i += 256) acc[i] = op == RG_AND ? ~0ull : 0ull;
            __syncthreads();
        } else if (pres) {
            uint64_t r[4];
            kw_pres_words(a, ids0, j0, j1, op == RG_AND, r);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[4 * tid + q] = r[q];
            __syncthreads();
        } else if (op != RG_AND) {
            kw_fill_keys(a, rs, rn, roff, j0, j1, accm, false);
        } else {
            // at most KW_AND_GROUP bitmaps: one mask each, then their AND
            for (uint32_t i = tid; i < (j1 - j0) * 1024; i += 256) grp[i >> 10][i & 1023] = 0;
            __syncthreads();
            kw_fill_keys(a, rs, rn, roff, j0, j1, grp, true);
            for (uint32_t i = tid; i < 1024; i += 256) {
                uint64_t x = ~0ull;
                for (uint32_t g = 0; g < j1 - j0; ++g) x &= grp[g][i];
                acc[i] = x;
            }
            __syncthreads();
        }
        uint64_t* gm = a.kmask + (uint64_t)mi * 1024;
        for (uint32_t i = tid; i < 1024; i += 256) {
            const uint64_t x = op == RG_AND ? ~acc[i] : acc[i];
            if (x) atomicOr(reinterpret_cast<unsigned long long*>(&gm[i]), (unsigned long long)x);
        }
        __threadfence();
        __syncthreads();
        if (tid == 0) last = atomicAdd(&a.kdone[mi], 1u) == n - 1 ? 1u : 0u;
        __syncthreads();
        if (uniform(last)) {
            __threadfence();
            for (uint32_t i = tid; i < 1024; i += 256) {
                const uint64_t x = __hip_atomic_load(&gm[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                acc[i] = op == RG_AND ? ~x : x;
            }
            __syncthreads();
            kw_emit_tasks(a, q, op, k, uniform64(Q.slot0), uniform(Q.kbound), acc, nullptr, rs, false, tmp, wpre);
        }
        __syncthreads();  // LDS read before the next part
    }
}

// ---------------------------------------------------------------- 2. bounds
// One wave per slot: lane j looks the key up in the query's j-th bitmap (64
// bitmaps per round), so the k searches run side by side.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t x = __shfl_xor(v, o);
        v = x < v ? x : v;
    }
    return v;
}

__global__ void __launch_bounds__(256) k_kw_bounds(KwArgs a) {
    const uint32_t lane = lane_id();
    const uint64_t s = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= a.n_slots) return;  // wave-uniform
    const Task t = uniform_task(a.tasks, (uint32_t)s);
    uint32_t ub = 0;
    uint8_t mark = 0;  // KW_TASK_SMALL / KW_TASK_BB / KW_TASK_WAVE: the slot's one-wave kernel
    if (t.kind == KIND_MATCH) {
        const KwQuery* Qp = a.queries + (t.pair - a.pair_base);
        const uint32_t flags = uniform(Qp->flags);
        {
            // unions and symmetric differences of more than two bitmaps (tasks
            // without recorded containers), at most KW_WAVE_MAX_K of them:
            // folded by one wave, materialised or counted
            const uint32_t op = uniform(Qp->op), k = uniform(Qp->k);
            if (a.wave && t.bin != KW_TASK_INDEXED && (op == RG_OR || op == RG_XOR) && k <= KW_WAVE_MAX_K)
                mark = KW_TASK_WAVE;
        }
        if (flags & KW_MATERIALIZE) {
            const uint32_t op = uniform(Qp->op), k = uniform(Qp->k), ids0 = uniform(Qp->ids_off);
            // AND: the smallest container; OR, XOR: the sum; ANDNOT: the first
            uint64_t sum = 0;
            uint32_t mn = 0xFFFFFFFFu, first = 0;
            uint32_t ty = 0, sz = 0;  // type and size of lane j's container (0: absent)
            for (uint32_t j0 = 0; j0 < k; j0 += 64) {
                const uint32_t j = j0 + lane;
                uint32_t cj = 0;
                if (j < k) {
                    const PoolView pv = kw_side(a, j != 0);
                    const uint32_t ci = t.bin == KW_TASK_INDEXED ? (j == 0 ? t.ia : t.ib)
                                                                 : kw_find_key(pv.bm_begin, pv.keys, pv.kidx,
                                                                               a.ids[ids0 + j], t.key);
                    cj = ci == NONE ? 0u : pv.card[ci];
                    if (ci != NONE && j0 == 0) {
                        ty = pv.types[ci];
                        sz = pv.size[ci];
                    }
                }
                if (j0 == 0) first = __builtin_amdgcn_readlane(cj, 0);
                sum += wave_sum_u64(cj);
                const uint32_t m = wave_min_u32(j < k ? cj : 0xFFFFFFFFu);
                mn = m < mn ? m : mn;
            }
            const uint64_t bc = op == RG_AND ? (uint64_t)mn : op == RG_ANDNOT ? (uint64_t)first : sum;
            ub = wbytes_of(bc);
            if (a.small && t.bin == KW_TASK_INDEXED) {
                const uint32_t ta = __builtin_amdgcn_readlane(ty, 0), sa = __builtin_amdgcn_readlane(sz, 0);
                const uint32_t tb = k > 1 ? __builtin_amdgcn_readlane(ty, 1) : 0u;
                const uint32_t sb = k > 1 ? __builtin_amdgcn_readlane(sz, 1) : 0u;
                mark = small_mat_ok((int)op, (uint8_t)ta, (uint8_t)tb, sa, sb) ? KW_TASK_SMALL
                       : bb_mat_ok((int)op, (uint8_t)ta, (uint8_t)tb)       ? KW_TASK_BB
                                                                            : 0;
            }
        }
    }
    if (lane == 0) {
        a.ub[s] = ub;
        a.res_card[s] = 0;
        if (mark) a.tasks[s].bin = mark;
    }
}

// The same for calls whose queries all have at most two bitmaps (pairwise
// materialisation): every task records its containers, so a slot needs no
// search and one thread per slot does (a wave per slot would leave 62 of its
// lanes idle).
__global__ void __launch_bounds__(256) k_kw_bounds_pairs(KwArgs a) {
    const uint64_t s = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= a.n_slots) return;
    const Task t = a.tasks[s];
    uint32_t ub = 0;
    uint8_t mark = 0;
    if (t.kind == KIND_MATCH && t.bin != KW_TASK_INDEXED) {
        atomicOr(a.err, 1u);  // cannot happen: the key kernels index every pairwise task
    } else if (t.kind == KIND_MATCH) {
        const KwQuery& Q = a.queries[t.pair - a.pair_base];
        if (Q.flags & KW_MATERIALIZE) {
            const uint32_t op = Q.op, k = Q.k;
            uint32_t ca = 0, cb = 0, sa = 0, sb = 0;
            uint8_t ta = 0, tb = 0;
            if (t.ia != NONE) {
                ca = a.P0.card[t.ia];
                ta = a.P0.types[t.ia];
                sa = a.P0.size[t.ia];
            }
            if (k > 1 && t.ib != NONE) {
                cb = a.P1.card[t.ib];
                tb = a.P1.types[t.ib];
                sb = a.P1.size[t.ib];
            }
            const uint64_t bc = op == RG_AND ? (uint64_t)(k > 1 ? (ca < cb ? ca : cb) : ca)
                                : op == RG_ANDNOT ? (uint64_t)ca : (uint64_t)ca + cb;
            ub = wbytes_of(bc);
            if (a.small)
                mark = small_mat_ok((int)op, ta, tb, sa, sb) ? KW_TASK_SMALL
                       : bb_mat_ok((int)op, ta, tb)          ? KW_TASK_BB
                                                             : 0;
        }
    }
    a.ub[s] = ub;
    a.res_card[s] = 0;
    if (mark) a.tasks[s].bin = mark;
}

// ---------------------------------------------------------------- 3. evaluate
// Folds a set of containers into the LDS bitset r with one read-modify-write
// per unit: OP 0 sets bits (union), 1 flips them (symmetric difference: each
// container flips its own values, so a bit ends up set when an odd number of
// containers hold it), 2 clears them (difference). Units: array value, bitset
// word, run.
template <int OP>
__device__ __forceinline__ void kw_apply(uint64_t* r, uint32_t wi, uint64_t m) {
    unsigned long long* dst = reinterpret_cast<unsigned long long*>(&r[wi]);
    if (OP == 0) atomicOr(dst, m);
    else if (OP == 1) atomicXor(dst, m);
    else atomicAnd(dst, ~m);
}

template <int OP>
__device__ __forceinline__ void kw_fold_units(uint64_t* r, const uint32_t* cunits, const uint8_t* ctype,
                                              const uint64_t* cpl, uint32_t total) {
    uint32_t j = 0;
    for (uint32_t base = 0; base < total; base += 256 * KW_UNROLL) {
        // the round's units are read first, so that their loads overlap
        uint64_t raw[KW_UNROLL];
        uint32_t loc[KW_UNROLL];
        uint8_t type[KW_UNROLL];
#pragma unroll
        for (int q = 0; q < KW_UNROLL; ++q) {
            const uint32_t u = base + q * 256 + threadIdx.x;
            type[q] = 0;
            loc[q] = 0;
            raw[q] = 0;
            if (u < total) {
                while (cunits[j + 1] <= u) ++j;  // u only grows, so j only moves forward
                loc[q] = u - cunits[j];
                type[q] = ctype[j];
                const uint8_t* pl = reinterpret_cast<const uint8_t*>(cpl[j]);
                if (type[q] == RG_ARRAY) raw[q] = reinterpret_cast<const uint16_t*>(pl)[loc[q]];
                else if (type[q] == RG_BITSET) raw[q] = reinterpret_cast<const uint64_t*>(pl)[loc[q]];
                else raw[q] = reinterpret_cast<const uint32_t*>(pl)[loc[q]];
            }
        }
#pragma unroll
        for (int q = 0; q < KW_UNROLL; ++q) {
            if (type[q] == RG_ARRAY) {
                kw_apply<OP>(r, (uint32_t)raw[q] >> 6, 1ull << (raw[q] & 63));
            } else if (type[q] == RG_BITSET) {
                if (raw[q]) kw_apply<OP>(r, loc[q], raw[q]);
            } else if (type[q] == RG_RUN) {
                const uint32_t first = (uint32_t)raw[q] & 0xFFFFu, last = first + ((uint32_t)raw[q] >> 16);
                for (uint32_t wi = first >> 6; wi <= last >> 6; ++wi) {
                    const uint32_t lo = wi == first >> 6 ? first & 63 : 0;
                    const uint32_t hi = wi == last >> 6 ? last & 63 : 63;
                    kw_apply<OP>(r, wi, (~0ull << lo) & (~0ull >> (63 - hi)));
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_kw_eval(KwArgs a) {
    __shared__ WgShared sh;
    __shared__ uint32_t cidx[KW_MAX_K];
    __shared__ uint32_t cunits[KW_MAX_K + 1];  // exclusive prefix of the containers' unit counts
    __shared__ uint8_t ctype[KW_MAX_K];
    __shared__ uint64_t cpl[KW_MAX_K];         // payload address of each container
    __shared__ uint8_t bsl[KW_MAX_K];          // the bitset containers (union, symmetric difference, difference)
    __shared__ uint32_t chunk_mask;
    const uint32_t tid = threadIdx.x;
    // chunks of eval_chunk slots: their tasks are read at once, then the
    // workgroup evaluates those that are its own (not empty, not the one-wave
    // kernel's) one after another
    const uint32_t chunk = a.eval_chunk;
    for (uint64_t c0 = (uint64_t)blockIdx.x * chunk; c0 < a.n_slots; c0 += (uint64_t)gridDim.x * chunk) {
    bool own = false;
    if (tid < chunk && c0 + tid < a.n_slots) {
        const Task t = a.tasks[c0 + tid];
        own = t.kind == KIND_MATCH && t.bin != KW_TASK_SMALL && t.bin != KW_TASK_DONE;
    }
    const uint64_t ob = __ballot(own);  // wave 0 holds the chunk
    if (tid == 0) chunk_mask = (uint32_t)ob;
    __syncthreads();
    uint32_t todo = uniform(chunk_mask);
    __syncthreads();  // read before the next chunk writes it
    while (todo) {
        const uint64_t s = c0 + (uint32_t)__builtin_ctz(todo);
        todo &= todo - 1;
        const Task t = uniform_task(a.tasks, (uint32_t)s);
        const uint32_t q = t.pair - a.pair_base;
        const KwQuery Q = a.queries[q];
        const uint32_t op = uniform(Q.op), k = uniform(Q.k), flags = uniform(Q.flags);
        const uint32_t ids0 = uniform(Q.ids_off);
        if (tid < k) {
            if (t.bin == KW_TASK_INDEXED || t.bin == KW_TASK_BB) {
                cidx[tid] = tid == 0 ? t.ia : t.ib;
            } else {
                const uint64_t* bmb = tid ? a.P1.bm_begin : a.P0.bm_begin;
                const uint16_t* pkeys = tid ? a.P1.keys : a.P0.keys;
                const uint8_t* pidx = tid ? a.P1.kidx : a.P0.kidx;
                cidx[tid] = kw_find_key(bmb, pkeys, pidx, a.ids[ids0 + tid], t.key);
            }
        }
        __syncthreads();
        bool empty = false;
        bool first = true;
        bool direct = false;  // the result words are already in w (registers)
        uint64_t w[4] = {0, 0, 0, 0};
        if (op != RG_AND) {
            // Union, symmetric difference, difference. Every thread owns words
            // 4t..4t+3 of the result: it combines the matching words of each
            // bitset container in registers (no atomics), starting from zero or,
            // for a difference, from the expanded first container. Array and
            // run containers then fold into the LDS bitset all at once with one
            // LDS atomic per value or run. No container waits for another.
            const uint32_t j0 = op == RG_ANDNOT ? 1u : 0u;
            // per container: its unit count (values or runs; 0 for a bitset),
            // and for the bitsets their place in a list
            uint32_t units = 0, isbs = 0;
            if (tid < k) {
                ctype[tid] = 0;  // absent (or the first container of a difference)
                const uint32_t ci = cidx[tid];
                if (ci != NONE && tid >= j0) {
                    const PoolView pv = kw_side(a, tid != 0);
                    const uint8_t ty = pv.types[ci];
                    isbs = ty == RG_BITSET ? 1u : 0u;
                    units = isbs ? 0u : pv.size[ci];
                    ctype[tid] = ty;
                    cpl[tid] = reinterpret_cast<uint64_t>(pv.payload + pv.off[ci]);
                }
            }
            uint32_t total, nbs;
            const uint32_t pos = block_excl_scan_u32(units, sh.tmp, &total);
            const uint32_t bpos = block_excl_scan_u32(isbs, sh.tmp, &nbs);
            if (tid < k) cunits[tid] = pos;
            if (tid == 0) cunits[k] = total;
            if (isbs) bsl[bpos] = (uint8_t)tid;
            if (op == RG_ANDNOT) expand_container(sh.sa, a.P0, uniform(cidx[0]), sh);  // ends with a barrier
            else __syncthreads();
            uint64_t r[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) r[q] = op == RG_ANDNOT ? sh.sa[4 * tid + q] : 0ull;
            // the bitsets, KW_BS_BATCH at a time with all their loads in flight
            // (each operation is order-free across the containers it folds)
            const uint32_t nb = uniform(nbs);
            for (uint32_t b0 = 0; b0 < nb; b0 += KW_BS_BATCH) {
                u32x4 v0[KW_BS_BATCH], v1[KW_BS_BATCH];
#pragma unroll
                for (uint32_t u = 0; u < KW_BS_BATCH; ++u) {
                    if (b0 + u < nb) {
                        const u32x4* src = reinterpret_cast<const u32x4*>(cpl[bsl[b0 + u]]) + 2 * tid;
                        v0[u] = src[0];
                        v1[u] = src[1];
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < KW_BS_BATCH; ++u) {
                    if (b0 + u < nb) {
                        const uint64_t x[4] = {(uint64_t)v0[u].x | ((uint64_t)v0[u].y << 32),
                                               (uint64_t)v0[u].z | ((uint64_t)v0[u].w << 32),
                                               (uint64_t)v1[u].x | ((uint64_t)v1[u].y << 32),
                                               (uint64_t)v1[u].z | ((uint64_t)v1[u].w << 32)};
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            r[q] = op == RG_OR ? (r[q] | x[q]) : op == RG_XOR ? (r[q] ^ x[q]) : (r[q] & ~x[q]);
                    }
                }
            }
            const uint32_t tu = uniform(total);
            if (tu == 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) w[q] = r[q];
                direct = true;
            } else {
                __syncthreads();  // every thread has read its start words from sh.sa
#pragma unroll
                for (int q = 0; q < 4; ++q) sh.sa[4 * tid + q] = r[q];
                __syncthreads();
                if (op == RG_ANDNOT) kw_fold_units<2>(sh.sa, cunits, ctype, cpl, tu);
                else if (op == RG_XOR) kw_fold_units<1>(sh.sa, cunits, ctype, cpl, tu);
                else kw_fold_units<0>(sh.sa, cunits, ctype, cpl, tu);
                __syncthreads();
            }
            first = false;
        }
        // intersection: running result in sh.sa, starting from the container
        // with the fewest values (ties: the lowest index); each other one is
        // expanded into sh.sb and combined, stopping once the result is empty
        uint32_t jmin = 0;
        if (op == RG_AND) {
            uint32_t key = 0xFFFFFFFFu;  // cardinality << 8 | index; a missing container counts as empty
            if (tid < k) {
                const uint32_t ci = cidx[tid];
                const PoolView pv = kw_side(a, tid != 0);
                key = ((ci == NONE ? 0u : pv.card[ci]) << 8) | tid;
            }
            key = wave_min_u32(key);
            if ((tid & 63) == 0) sh.xchg[tid >> 6] = key;
            __syncthreads();
            uint32_t m = sh.xchg[0];
            for (int w = 1; w < 4; ++w) m = sh.xchg[w] < m ? sh.xchg[w] : m;
            jmin = uniform(m & 0xFFu);
            __syncthreads();
        }
        for (uint32_t step = 0; op == RG_AND && step < k && !empty; ++step) {
            const uint32_t j = step == 0 ? jmin : (step - 1 < jmin ? step - 1 : step);
            const uint32_t ci = uniform(cidx[j]);
            if (ci == NONE) {  // cannot happen: the key is in every bitmap
                empty = true;
                continue;
            }
            const PoolView pv = kw_side(a, j != 0);
            expand_container(first ? sh.sa : sh.sb, pv, ci, sh);
            if (!first) {
                uint32_t any = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t wi = 4 * tid + i;
                    const uint64_t v = sh.sa[wi] & sh.sb[wi];
                    sh.sa[wi] = v;
                    any |= v != 0 ? 1u : 0u;
                }
                empty = block_sum_u64(any, sh.tmp64) == 0;
            }
            first = false;
        }
        if (!direct) {
#pragma unroll
            for (int i = 0; i < 4; ++i) w[i] = (empty || first) ? 0ull : sh.sa[4 * tid + i];
        }
        __syncthreads();
        if (flags & KW_MATERIALIZE) {
            finalize_words(w, (uint32_t)s, a.so, sh.sa, sh.sb, sh);
        } else {
            const uint32_t c = count_words(w, sh);
            if (tid == 0 && c) atomicAdd(reinterpret_cast<unsigned long long*>(&a.acc[q]), (unsigned long long)c);
        }
        __syncthreads();
    }
    }
}

// per-query cardinality of count-only and materialised queries alike
__global__ void k_kw_cards(KwArgs a, const uint64_t* bm_card, uint64_t* cards) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.n_queries) return;
    cards[q] = (a.queries[q].flags & KW_MATERIALIZE) ? bm_card[q] : (uint64_t)a.acc[q];
}

// Zeroes what a step accumulates into, in one launch: two scan totals, the
// error flag, and per query its count accumulator, cardinality and payload bound.
__global__ void k_kw_step_init(uint64_t* totals, uint32_t* err, long long* acc, uint64_t* bm_card,
                               uint64_t* bm_wbytes, uint32_t nq, uint64_t* kmask, uint32_t* kdone, uint32_t n_masks) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2) totals[i] = 0;
    if (i == 0) *err = 0;
    if (i < nq) {
        acc[i] = 0;
        bm_card[i] = 0;
        bm_wbytes[i] = 0;
    }
    if (i < n_masks * 1024u) kmask[i] = 0;
    if (i < n_masks) kdone[i] = 0;
}

void launch_kw_step_init(uint64_t* totals, uint32_t* err, long long* acc, uint64_t* bm_card, uint64_t* bm_wbytes,
                         uint32_t nq, uint64_t* kmask, uint32_t* kdone, uint32_t n_masks, hipStream_t st) {
    uint32_t n = nq > 2 ? nq : 2;
    n = n > n_masks * 1024u ? n : n_masks * 1024u;
    hipLaunchKernelGGL(k_kw_step_init, dim3((n + 255) / 256), dim3(256), 0, st, totals, err, acc, bm_card, bm_wbytes,
                       nq, kmask, kdone, n_masks);
}

void launch_kw_keys(const KwArgs& a, hipStream_t st, bool pairs, bool whole) {
    if (!a.n_queries) return;
    if (a.n_parts)
        hipLaunchKernelGGL(k_kw_keys_part, dim3(a.n_parts < 16384 ? a.n_parts : 16384u), dim3(256), 0, st, a);
    if (pairs) hipLaunchKernelGGL(k_kw_keys_small, dim3((a.n_queries + 3) / 4), dim3(256), 0, st, a);
    if (!pairs && !whole) return;
    // a query per workgroup for small batches (each may be large); up to
    // KW_KEYS_CHUNK for large ones, where most are the one-wave kernel's
    uint32_t chunk = a.n_queries / 2048;
    chunk = chunk < 1 ? 1u : chunk > KW_KEYS_CHUNK ? KW_KEYS_CHUNK : chunk;
    const uint32_t g = (a.n_queries + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_kw_keys, dim3(g < 16384 ? g : 16384u), dim3(256), 0, st, a, chunk);
}
void launch_kw_bounds(const KwArgs& a, hipStream_t st, bool pairs_only) {
    if (!a.n_slots) return;
    if (pairs_only) hipLaunchKernelGGL(k_kw_bounds_pairs, dim3((uint32_t)((a.n_slots + 255) / 256)), dim3(256), 0, st, a);
    else hipLaunchKernelGGL(k_kw_bounds, dim3((uint32_t)((a.n_slots + 3) / 4)), dim3(256), 0, st, a);
}
void launch_kw_eval(const KwArgs& a, hipStream_t st) {
    if (!a.n_slots) return;
    const uint32_t chunk = a.eval_chunk == 0 ? (a.n_slots <= KW_EVAL_FEW ? 1u : 4u)
                           : a.eval_chunk > 64 ? 64u : a.eval_chunk;
    KwArgs b = a;
    b.eval_chunk = chunk;
    const uint64_t nc = (a.n_slots + chunk - 1) / chunk;
    const uint32_t g = nc < 65536 ? (uint32_t)nc : 65536u;
    hipLaunchKernelGGL(k_kw_eval, dim3(g), dim3(256), 0, st, b);
}
void launch_kw_cards(const KwArgs& a, const uint64_t* bm_card, uint64_t* cards, hipStream_t st) {
    if (a.n_queries)
        hipLaunchKernelGGL(k_kw_cards, dim3((a.n_queries + 255) / 256), dim3(256), 0, st, a, bm_card, cards);
}

}  // namespace rg

namespace rg {

// pairwise materialisation through the k-way path: query q is pair pair0 + q.
// single: the query is the union of the pair's first bitmap alone (k = 1),
// which rebuilds that bitmap's containers in P1 form (canonicalisation).
// Without pair arrays, ia0 / ib0 == NONE make pair p bitmap p.
__global__ void k_kw_pair_queries(int op, const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0,
                                  uint64_t pair0, uint32_t n_pairs, const uint64_t* cand_off, KwQuery* queries,
                                  uint32_t* ids, int single) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    const uint64_t p = pair0 + q;
    ids[2 * q] = ia ? ia[p] : ia0 == NONE ? (uint32_t)p : ia0;
    ids[2 * q + 1] = ib ? ib[p] : ib0 == NONE ? (uint32_t)p : ib0;
    KwQuery Q;
    Q.op = single ? (uint32_t)RG_OR : (uint32_t)op;
    Q.k = single ? 1u : 2u;
    Q.ids_off = 2 * q;
    Q.flags = KW_MATERIALIZE;
    Q.slot0 = cand_off[q];
    Q.kbound = (uint32_t)(cand_off[q + 1] - cand_off[q]);
    Q.pad = 0;
    queries[q] = Q;
}

void launch_kw_pair_queries(int op, const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0,
                            uint64_t pair0, uint32_t n_pairs, const uint64_t* cand_off, KwQuery* queries,
                            uint32_t* ids, hipStream_t st, bool single) {
    if (n_pairs)
        hipLaunchKernelGGL(k_kw_pair_queries, dim3((n_pairs + 255) / 256), dim3(256), 0, st, op, ia, ib, ia0, ib0,
                           pair0, n_pairs, cand_off, queries, ids, (int)single);
}

// first key | last key << 16 of a bitmap with keys (0 for one without)
__device__ __forceinline__ uint32_t kw_span(const uint64_t* bm_begin, const uint16_t* keys, uint32_t b) {
    const uint64_t s = bm_begin[b], e = bm_begin[b + 1];
    return s < e ? (uint32_t)keys[s] | (uint32_t)keys[e - 1] << 16 : 0u;
}

// per id: key count, payload bound (bm_wbytes), validity and key span, for host-side bounds
__global__ void k_kw_gather_meta(const uint64_t* bm_begin, const uint16_t* keys, const uint64_t* bm_wbytes,
                                 uint32_t n_bitmaps, const uint32_t* ids, uint32_t k, uint64_t* out) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= k) return;
    const uint32_t b = ids[j];
    if (b >= n_bitmaps) {
        out[4 * j] = 0;
        out[4 * j + 1] = 0;
        out[4 * j + 2] = 0;
        out[4 * j + 3] = 0;
        return;
    }
    out[4 * j] = bm_begin[b + 1] - bm_begin[b];
    out[4 * j + 1] = bm_wbytes[b];
    out[4 * j + 2] = 1;
    out[4 * j + 3] = kw_span(bm_begin, keys, b);
}

void launch_kw_gather_meta(const uint64_t* bm_begin, const uint16_t* keys, const uint64_t* bm_wbytes,
                           uint32_t n_bitmaps, const uint32_t* ids, uint32_t k, uint64_t* out, hipStream_t st) {
    if (k) hipLaunchKernelGGL(k_kw_gather_meta, dim3((k + 255) / 256), dim3(256), 0, st, bm_begin, keys, bm_wbytes,
                              n_bitmaps, ids, k, out);
}

__global__ void k_kw_key_span(const uint64_t* bm_begin, const uint16_t* keys, uint32_t n, uint32_t* out) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n) out[b] = kw_span(bm_begin, keys, b);
}

void launch_kw_key_span(const uint64_t* bm_begin, const uint16_t* keys, uint32_t n, uint32_t* out, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_kw_key_span, dim3((n + 255) / 256), dim3(256), 0, st, bm_begin, keys, n, out);
}

}  // namespace rg
