// rg_serve.cpp - k-way queries (roaring_multi) and the serving loop.
//
// Both run "steps": a batch of k-way AND/OR queries over one pool, enqueued
// on a stream without host synchronisation (rg_kway.hip kernels, then the
// pairwise path's compaction and the per-bitmap fingerprint). The host sizes a
// step from per-bitmap key counts and payload bounds alone:
//   AND:     at most min_i K_i result containers and min_i W_i payload bytes,
//   OR, XOR: at most min(65536, sum_i K_i) containers and sum_i W_i bytes,
//   ANDNOT:  at most K_0 containers and W_0 bytes,
// (W_i = sum over bitmap i's containers of min(8192, 2c), rounded to 16 B,
// which bounds every container's P1 form), so a step never needs a readback
// before its results.
//
// The server admits queries in arrival order into steps as step slots and
// arena memory allow (continuous batching: queries that arrive while steps
// are on the GPU join the next step; up to `max_inflight` steps are enqueued
// at once, on alternating streams, so their kernels overlap), retires steps
// whose completion event has fired, and reports per-query latency from
// arrival to result-ready.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "rg_host.h"

namespace {

using Clock = std::chrono::steady_clock;

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now().time_since_epoch()).count();
}

struct Bounds {
    uint64_t kbound = 0;  // result containers
    uint64_t pbound = 0;  // result payload bytes (0 for count-only)
};

// meta[4j..4j+3] = key count, payload bound, valid flag and key span (first
// key | last key << 16, when the count is not zero) of the query's j-th bitmap.
// Result keys lie in the bitmaps' key lists (Section 1: a bitmap is its sorted
// keys and their containers): a union or symmetric difference holds at most
// every key between the smallest first key and the largest last key, an
// intersection only keys between the largest first key and the smallest last
// key, a difference only keys of its first bitmap. Each result container takes
// at most 8 KiB, so the payload bound is also capped by the key bound.
Bounds query_bounds(int op, uint32_t k, const uint64_t* meta, bool mat) {
    uint64_t kmin = ~0ull, ksum = 0, wmin = ~0ull, wsum = 0;
    uint32_t lo_min = 65535, lo_max = 0, hi_min = 65535, hi_max = 0;  // over bitmaps with keys
    for (uint32_t j = 0; j < k; ++j) {
        const uint64_t n = meta[4 * j];
        kmin = std::min(kmin, n);
        ksum += n;
        wmin = std::min(wmin, meta[4 * j + 1]);
        wsum += meta[4 * j + 1];
        if (n) {
            const uint32_t lo = (uint32_t)(meta[4 * j + 3] & 0xFFFF), hi = (uint32_t)(meta[4 * j + 3] >> 16 & 0xFFFF);
            lo_min = std::min(lo_min, lo);
            lo_max = std::max(lo_max, lo);
            hi_min = std::min(hi_min, hi);
            hi_max = std::max(hi_max, hi);
        }
    }
    Bounds b;
    if (op == RG_AND) {
        b.kbound = kmin && hi_min >= lo_max ? std::min<uint64_t>(kmin, hi_min - lo_max + 1) : 0;
        b.pbound = wmin;
    } else if (op == RG_ANDNOT) {
        b.kbound = meta[0];
        b.pbound = meta[1];
    } else {
        b.kbound = ksum ? std::min<uint64_t>(ksum, hi_max - lo_min + 1) : 0;
        b.pbound = wsum;
    }
    b.pbound = std::min<uint64_t>(b.pbound, b.kbound * 8192);
    if (!mat) b.pbound = 0;
    return b;
}

// Splits the key pass of query q (record Q, key count of its j-th bitmap at
// nkeys[j * stride]) into parts of whole bitmaps for k_kw_keys_part. With the
// pool's key-presence index (pres) a part combines the presence words of up to
// KW_PART_BITMAPS bitmaps; without it a union or symmetric difference is cut
// into parts of about KW_PART_KEYS keys and an intersection into groups of
// KW_AND_GROUP bitmaps. With two parts or more the query is marked KW_SPLIT
// with key mask *n_masks (then counted) and its parts are appended; otherwise
// nothing changes. A difference's keys are its first bitmap's: never split.
void split_query(KwQuery* Q, uint32_t q, const uint64_t* nkeys, size_t stride, bool pres, std::vector<KwPart>* parts,
                 uint32_t* n_masks) {
    const uint32_t k = Q->k;
    if (k <= 2 || Q->op == RG_ANDNOT) return;
    std::vector<uint32_t> cut{0};
    uint64_t acc = 0;
    for (uint32_t j = 0; j < k; ++j) {
        const uint64_t n = nkeys[j * stride];
        const bool full = pres              ? j - cut.back() == KW_PART_BITMAPS
                          : Q->op == RG_AND ? j - cut.back() == KW_AND_GROUP
                                            : acc > 0 && acc + n > KW_PART_KEYS;
        if (full) {
            cut.push_back(j);
            acc = 0;
        }
        acc += n;
    }
    cut.push_back(k);
    const uint32_t n_parts = (uint32_t)cut.size() - 1;
    if (n_parts < 2) return;
    const uint32_t mi = (*n_masks)++;
    for (uint32_t i = 0; i < n_parts; ++i) parts->push_back(KwPart{q, cut[i] | cut[i + 1] << 16, mi, n_parts});
    Q->flags |= KW_SPLIT;
    Q->pad = mi;
}

// Device layout of one step (each piece 256-byte aligned):
//   upload   : queries, ids, cand_off            (mirrored in pinned host memory)
//   download : cards, digest, bm_begin, totals, err
//   work     : tasks, ub, slot_off, res_card, res_type, res_size, out_idx, partials, acc
//   out      : keys, types, card, size, off, payload, bm_card, bm_wbytes (unless the caller's)
struct StepLayout {
    uint32_t nq = 0;
    uint64_t nids = 0, S = 0, P = 0;
    uint32_t n_parts = 0, n_masks = 0;  // split key passes of the step (set when staged)
    bool pairs = true, whole = true;    // some query of <= 2 bitmaps / some unsplit one of more
    bool big = true;                    // some query of more than 2 bitmaps
    bool own_out = true;
    size_t up_bytes = 0, down_off = 0, down_bytes = 0, total = 0;
    // offsets
    size_t o_queries, o_ids, o_cand, o_parts, o_kmask, o_kdone, o_cards, o_digest, o_bm_begin, o_totals, o_err, o_tasks, o_ub, o_slot_off,
        o_res_card, o_res_type, o_res_size, o_out_idx, o_partials, o_acc, o_keys, o_types, o_card,
        o_size, o_off, o_payload, o_bm_card, o_bm_wbytes;

    void plan(uint32_t nq_, uint64_t nids_, uint64_t S_, uint64_t P_, bool own) {
        nq = nq_;
        nids = nids_;
        S = S_;
        P = P_;
        own_out = own;
        size_t u = 0;
        auto take = [&](size_t bytes) {
            size_t o = u;
            u += align256(bytes ? bytes : 1);
            return o;
        };
        o_queries = take(sizeof(KwQuery) * nq);
        o_ids = take(4 * nids);
        o_cand = take(8 * (nq + 1));
        o_parts = take(sizeof(KwPart) * nids);  // a part holds one bitmap or more
        up_bytes = u;
        down_off = u;
        o_cards = take(8 * nq);
        o_digest = take(8 * nq);
        o_bm_begin = take(8 * (nq + 1));
        o_totals = take(16);
        o_err = take(4);
        down_bytes = u - down_off;
        o_tasks = take(sizeof(Task) * S);
        o_ub = take(4 * S);
        o_slot_off = take(8 * S);
        o_res_card = take(4 * S);
        o_res_type = take(S);
        o_res_size = take(4 * S);
        o_out_idx = take(8 * S);
        o_partials = take(8 * scan_partials_needed(S));
        o_acc = take(8 * nq);
        o_kmask = take(8192 * (size_t)nq);  // a split query's key mask
        o_kdone = take(4 * nq);
        if (own) {
            o_keys = take(2 * S);
            o_types = take(S);
            o_card = take(4 * S);
            o_size = take(4 * S);
            o_off = take(8 * S);
            o_payload = take(P);
            o_bm_card = take(8 * nq);
            o_bm_wbytes = take(8 * nq);
        }
        total = u;
    }
};

// Output arrays of a step: its own (serving) or the caller's rg_out (roaring_multi).
struct StepOut {
    uint64_t* bm_begin;
    uint16_t* keys;
    uint8_t* types;
    uint32_t* card;
    uint32_t* size;
    uint64_t* off;
    uint8_t* payload;
    uint64_t* bm_card;
    uint64_t* bm_wbytes;
};

StepOut own_out(const StepLayout& L, uint8_t* d) {
    return StepOut{reinterpret_cast<uint64_t*>(d + L.o_bm_begin), reinterpret_cast<uint16_t*>(d + L.o_keys),
                   d + L.o_types, reinterpret_cast<uint32_t*>(d + L.o_card),
                   reinterpret_cast<uint32_t*>(d + L.o_size), reinterpret_cast<uint64_t*>(d + L.o_off),
                   d + L.o_payload, reinterpret_cast<uint64_t*>(d + L.o_bm_card),
                   reinterpret_cast<uint64_t*>(d + L.o_bm_wbytes)};
}

// A failed HIP call in step_enqueue: the message goes to *err (the caller's
// context, or the server's own record: the server thread never writes the
// context, which its owner may be using meanwhile).
#define STEPCHK(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            *err_out = std::string(#call) + ": " + hipGetErrorString(e_);              \
            return RG_EDEVICE;                                                         \
        }                                                                              \
    } while (0)

// Enqueues one step. h_stage: pinned host memory of L.down_off + L.down_bytes
// bytes whose upload section is filled; the download section receives the
// results once the stream reaches the end of the step.
// prof: the context whose kernel timing brackets the evaluation kernel
// (roaring_multi), or null (the server, which never touches the context).
// digest: the step's results get their fingerprints (some query asked).
rg_status step_enqueue(std::string* err_out, const rg_pool& pool, const StepLayout& L, uint8_t* d, const StepOut& o,
                       uint8_t* h_stage, hipStream_t st, bool digest, rg_ctx* prof = nullptr) {
    auto* queries = reinterpret_cast<KwQuery*>(d + L.o_queries);
    auto* ids = reinterpret_cast<uint32_t*>(d + L.o_ids);
    auto* cand = reinterpret_cast<uint64_t*>(d + L.o_cand);
    auto* cards = reinterpret_cast<uint64_t*>(d + L.o_cards);
    auto* d_digest = reinterpret_cast<uint64_t*>(d + L.o_digest);
    auto* totals = reinterpret_cast<uint64_t*>(d + L.o_totals);
    auto* err = reinterpret_cast<uint32_t*>(d + L.o_err);
    auto* tasks = reinterpret_cast<Task*>(d + L.o_tasks);
    auto* ub = reinterpret_cast<uint32_t*>(d + L.o_ub);
    auto* slot_off = reinterpret_cast<uint64_t*>(d + L.o_slot_off);
    auto* res_card = reinterpret_cast<uint32_t*>(d + L.o_res_card);
    auto* res_type = d + L.o_res_type;
    auto* res_size = reinterpret_cast<uint32_t*>(d + L.o_res_size);
    auto* out_idx = reinterpret_cast<uint64_t*>(d + L.o_out_idx);
    auto* partials = reinterpret_cast<uint64_t*>(d + L.o_partials);
    auto* acc = reinterpret_cast<long long*>(d + L.o_acc);
    auto* step_bm_begin = reinterpret_cast<uint64_t*>(d + L.o_bm_begin);

    STEPCHK(hipMemcpyAsync(d, h_stage, L.up_bytes, hipMemcpyHostToDevice, st));
    auto* kmask = reinterpret_cast<uint64_t*>(d + L.o_kmask);
    auto* kdone = reinterpret_cast<uint32_t*>(d + L.o_kdone);
    launch_kw_step_init(totals, err, acc, o.bm_card, o.bm_wbytes, L.nq, kmask, kdone, L.n_masks, st);
    KwArgs a;
    a.P0 = view(pool);
    a.P1 = a.P0;
    a.pair_base = 0;
    a.queries = queries;
    a.n_queries = L.nq;
    a.ids = ids;
    a.tasks = tasks;
    a.n_slots = L.S;
    a.ub = ub;
    a.res_card = res_card;
    a.so = SlotOut{slot_off, o.payload, res_card, res_type, res_size};
    a.acc = acc;
    a.err = err;
    a.parts = reinterpret_cast<const KwPart*>(d + L.o_parts);
    a.n_parts = L.n_parts;
    a.kmask = kmask;
    a.kdone = kdone;
    // Steps of many slots fold unions and symmetric differences of up to 64
    // bitmaps by one wave per result key (more keys in flight: throughput);
    // smaller steps keep one workgroup per key (four times the lanes per key:
    // latency)
    a.wave = L.big && L.S > KW_WAVE_MIN_SLOTS;
    // the one-wave array and bitset kernels take only queries of at most two
    // bitmaps; skip their launches when the step has none (L.pairs), and the
    // workgroup key kernel when every query of more bitmaps is split (L.whole)
    launch_kw_keys(a, st, L.pairs, L.whole);
    launch_kw_bounds(a, st, !L.big);
    if (L.S) launch_scan_u32_u64(ub, slot_off, L.S, 0, partials, totals, st);
    if (prof) {
        if (L.pairs) {
            timed(prof, PROF_KWSMALL, true, L.S, st, [&] { launch_kw_small(a, st); });
            timed(prof, PROF_KWBB, true, L.S, st, [&] { launch_kw_bb(a, st); });
        }
        if (a.wave) timed(prof, PROF_KWWAVE, true, L.S, st, [&] { launch_kw_wave(a, st); });
        timed(prof, PROF_KWEVAL, true, L.S, st, [&] { launch_kw_eval(a, st); });
    } else {
        if (L.pairs) {
            launch_kw_small(a, st);
            launch_kw_bb(a, st);
        }
        if (a.wave) launch_kw_wave(a, st);
        launch_kw_eval(a, st);
    }
    if (L.S) {
        launch_scan_nonzero_u64(res_card, out_idx, L.S, 0, partials, totals + 1, st);
        CompactArgs cp;
        cp.tasks = tasks;
        cp.n_slots = L.S;
        cp.res_card = res_card;
        cp.res_type = res_type;
        cp.res_size = res_size;
        cp.slot_off = slot_off;
        cp.out_idx = out_idx;
        cp.keys = o.keys;
        cp.types = o.types;
        cp.card = o.card;
        cp.size = o.size;
        cp.off = o.off;
        cp.bm_card = o.bm_card;
        cp.bm_wbytes = o.bm_wbytes;
        cp.pair0 = 0;
        launch_compact(cp, st);
    }
    launch_bm_begin(cand, out_idx, L.S, totals + 1, L.nq, 0, step_bm_begin, true, st);
    if (o.bm_begin != step_bm_begin)
        STEPCHK(hipMemcpyAsync(o.bm_begin, step_bm_begin, 8 * (L.nq + 1), hipMemcpyDeviceToDevice, st));
    launch_kw_cards(a, o.bm_card, cards, st);
    rg_pool outp{L.nq, L.S, L.P, step_bm_begin, o.keys, o.types, o.card, o.size, o.off, o.payload, o.bm_card,
                 o.bm_wbytes};
    if (digest) launch_pool_digest_n(outp, totals + 1, d_digest, st);
    STEPCHK(hipMemcpyAsync(h_stage + L.down_off, d + L.down_off, L.down_bytes, hipMemcpyDeviceToHost, st));
    STEPCHK(hipGetLastError());
    return RG_OK;
}

// Fills the upload section of h_stage for queries q (host ids), slot ranges in query order.
void stage_upload(const StepLayout& L, uint8_t* h_stage, const std::vector<KwQuery>& qs,
                  const std::vector<uint32_t>& ids, const std::vector<KwPart>& parts) {
    memcpy(h_stage + L.o_queries, qs.data(), sizeof(KwQuery) * qs.size());
    memcpy(h_stage + L.o_ids, ids.data(), 4 * ids.size());
    if (!parts.empty()) memcpy(h_stage + L.o_parts, parts.data(), sizeof(KwPart) * parts.size());
    auto* cand = reinterpret_cast<uint64_t*>(h_stage + L.o_cand);
    for (size_t q = 0; q < qs.size(); ++q) cand[q] = qs[q].slot0;
    cand[qs.size()] = L.S;
}

}  // namespace

// ---------------------------------------------------------------- roaring_multi

extern "C" rg_status roaring_multi(rg_ctx* c, int op, const rg_pool* pool, const uint32_t* d_ids, uint32_t k,
                                   uint32_t flags, rg_out* out, uint64_t* d_card, void* stream) {
    if (!c) return RG_EINVAL;
    if (op < RG_AND || op > RG_ANDNOT) return fail(c, RG_EINVAL, "roaring_multi: op must be RG_AND..RG_ANDNOT");
    if (k < 1 || k > KW_MAX_K || !d_ids) return fail(c, RG_EINVAL, "roaring_multi: 1 <= k <= 256 device ids");
    if (!pool_ok(pool)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    const bool mat = flags & RG_FLAG_MATERIALIZE;
    if (!(flags & (RG_FLAG_MATERIALIZE | RG_FLAG_CARD))) return fail(c, RG_EINVAL, "flags select no output");
    if ((flags & RG_FLAG_CARD) && !d_card) return fail(c, RG_EINVAL, "RG_FLAG_CARD needs d_card");
    if (mat && (!out || !out->bm_begin || !out->keys || !out->types || !out->card || !out->size || !out->off ||
                !out->payload || !out->bm_card || !out->bm_wbytes))
        return fail(c, RG_EINVAL, "materialisation needs a complete rg_out (with bm_wbytes)");
    HIPCHK(c, hipSetDevice(c->device));
    WorkspaceOrder order(c, (hipStream_t)stream);
    hipStream_t st = (hipStream_t)stream;
    // per-id metadata -> host bounds (one small readback)
    Scratch sc(c);
    void* mbase = nullptr;
    if (rg_status s = sc.take(WS_PAIRS, align256(32 * k) + 256, &mbase)) return s;
    auto* d_meta = reinterpret_cast<uint64_t*>(mbase);
    // the pinned staging: 32 k <= 8 KiB of metadata, then the ids (both in one readback)
    auto* h_meta = reinterpret_cast<uint64_t*>(c->host);
    auto* h_ids = reinterpret_cast<uint32_t*>(h_meta + 4 * k);
    launch_kw_gather_meta(pool->bm_begin, pool->keys, pool->bm_wbytes, pool->n_bitmaps, d_ids, k, d_meta, st);
    HIPCHK(c, hipMemcpyAsync(h_meta, d_meta, 32 * k, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(h_ids, d_ids, 4ull * k, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const std::vector<uint32_t> ids(h_ids, h_ids + k);  // the staging is reused below
    for (uint32_t j = 0; j < k; ++j)
        if (!h_meta[4 * j + 2]) return fail(c, RG_EINVAL, "roaring_multi: bitmap id out of range of the pool");
    const Bounds b = query_bounds(op, k, h_meta, mat);
    if (mat) {
        out->needed_containers = b.kbound;
        out->needed_payload_bytes = b.pbound;
        out->n_containers = 0;
        out->payload_used = 0;
        if (out->cap_containers < b.kbound || out->cap_payload_bytes < b.pbound)
            return fail(c, RG_ECAPACITY, "output arena too small");
    }
    std::vector<KwQuery> qs(1);
    qs[0] = KwQuery{(uint32_t)op, k, 0, mat ? KW_MATERIALIZE : 0u, 0, (uint32_t)b.kbound, 0};
    std::vector<KwPart> parts;
    uint32_t n_masks = 0;
    split_query(&qs[0], 0, h_meta, 4, pool->key_index != nullptr, &parts, &n_masks);  // before h_meta's staging is reused
    StepLayout L;
    L.plan(1, k, b.kbound, mat ? b.pbound : 0, !mat);
    L.n_parts = (uint32_t)parts.size();
    L.n_masks = n_masks;
    L.pairs = k <= 2;
    L.whole = k > 2 && !(qs[0].flags & KW_SPLIT);
    L.big = k > 2;
    void* wbase = nullptr;
    if (rg_status s = sc.take(WS_WAVE, L.total, &wbase)) return s;
    uint8_t* h = nullptr;
    if (rg_status s = host_buffer(c, L.down_off + L.down_bytes + 256, &h)) return s;
    auto* d = reinterpret_cast<uint8_t*>(wbase);
    // the ids into the staging copy (the step uploads the whole section)
    memcpy(h + L.o_ids, ids.data(), 4ull * k);
    memcpy(h + L.o_queries, qs.data(), sizeof(KwQuery));
    if (!parts.empty()) memcpy(h + L.o_parts, parts.data(), sizeof(KwPart) * parts.size());
    reinterpret_cast<uint64_t*>(h + L.o_cand)[0] = 0;
    reinterpret_cast<uint64_t*>(h + L.o_cand)[1] = L.S;
    StepOut o = mat ? StepOut{out->bm_begin, out->keys, out->types, out->card, out->size, out->off, out->payload,
                              out->bm_card, out->bm_wbytes}
                    : own_out(L, d);
    if (rg_status s = step_enqueue(&c->err, *pool, L, d, o, h, st, false, c)) return s;
    HIPCHK(c, hipStreamSynchronize(st));
    const uint64_t* totals = reinterpret_cast<const uint64_t*>(h + L.o_totals);
    const uint32_t err = *reinterpret_cast<const uint32_t*>(h + L.o_err);
    if (err) return fail(c, RG_EDEVICE, "roaring_multi: result key set exceeded its bound (internal error)");
    if (mat) {
        out->n_containers = totals[1];
        out->payload_used = totals[0];
    }
    if (flags & RG_FLAG_CARD)
        HIPCHK(c, hipMemcpyAsync(d_card, d + L.o_cards, 8, hipMemcpyDeviceToDevice, st));
    return RG_OK;
}

// ---------------------------------------------------------------- server

namespace {

// first-fit allocator over [0, cap) of the device arena, 256-byte units
class ArenaAlloc {
public:
    void reset(uint64_t cap) {
        free_.clear();
        if (cap) free_[0] = cap;
        cap_ = cap;
        used_ = peak_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = align256(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align256(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t peak() const { return peak_; }
    uint64_t cap() const { return cap_; }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t cap_ = 0, used_ = 0, peak_ = 0;
};

struct Entry {
    rg_query q;  // copy; its ids live in `ids`
    std::vector<uint32_t> ids;
    Bounds b;
    uint64_t arrival_ns = 0;
    uint64_t done_ns = 0;
    bool done = false;
    bool released = false;
    rg_status status = RG_OK;
    uint64_t card = 0, digest = 0, n_containers = 0, c_end = 0;
    struct Step* step = nullptr;
    uint32_t q_in_step = 0;
};

struct Step {
    StepLayout L;
    uint64_t arena_off = 0;
    uint8_t* d = nullptr;
    uint8_t* h = nullptr;  // pinned staging
    hipEvent_t done = nullptr;
    hipStream_t st = nullptr;
    std::vector<uint64_t> tickets;
    uint32_t live = 0;  // queries not yet released
};

}  // namespace

struct rg_server {
    rg_ctx* c = nullptr;
    rg_pool pool{};
    std::vector<uint64_t> h_bm_begin, h_wbytes;
    std::vector<uint32_t> h_span;  // first key | last key << 16 of every bitmap (with keys)
    uint8_t* arena = nullptr;
    ArenaAlloc alloc;
    uint32_t max_batch = 64, max_inflight = 2;
    uint64_t max_step_slots = 1ull << 22;
    hipStream_t streams[2] = {nullptr, nullptr};
    uint32_t next_stream = 0;
    std::vector<uint8_t*> pinned_free;  // staging buffers of pinned_bytes
    size_t pinned_bytes = 0;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    bool auto_release = false;
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, std::unique_ptr<Entry>> entries;
    std::deque<Step*> inflight;
    uint64_t next_ticket = 1;
    // stats
    uint64_t n_done = 0, n_steps = 0, n_deferred = 0, sum_batch = 0;
    std::string fatal;
    void run();
    bool admit_locked(std::vector<uint64_t>* take, uint64_t* S, uint64_t* P, uint64_t* nids);
    void retire_locked(Step* s);
    void free_step_locked(Step* s);
};

namespace {

bool query_host_ok(const rg_server* s, const rg_query* q) {
    if (!q || q->op < RG_AND || q->op > RG_ANDNOT || q->k < 1 || q->k > KW_MAX_K || !q->ids) return false;
    for (uint32_t j = 0; j < q->k; ++j)
        if (q->ids[j] >= s->pool.n_bitmaps) return false;
    return (q->flags & (RG_FLAG_MATERIALIZE | RG_FLAG_CARD)) != 0;
}

}  // namespace

// Called with mu held: picks queries from the front of the queue for one step.
bool rg_server::admit_locked(std::vector<uint64_t>* take, uint64_t* S, uint64_t* P, uint64_t* nids) {
    *S = *P = *nids = 0;
    for (uint64_t t : pending) {
        if (take->size() >= max_batch) break;
        Entry& e = *entries[t];
        if (*S + e.b.kbound > max_step_slots && !take->empty()) break;
        StepLayout L;
        L.plan((uint32_t)take->size() + 1, *nids + e.q.k, *S + e.b.kbound, *P + e.b.pbound, true);
        uint64_t off;
        if (!alloc.alloc(L.total, &off)) {
            if (take->empty()) ++n_deferred;
            break;
        }
        alloc.release(off, L.total);  // probe only; the step allocates once below
        take->push_back(t);
        *S += e.b.kbound;
        *P += e.b.pbound;
        *nids += e.q.k;
    }
    return !take->empty();
}

void rg_server::free_step_locked(Step* s) {
    alloc.release(s->arena_off, s->L.total);
    if (s->h) pinned_free.push_back(s->h);
    (void)hipEventDestroy(s->done);
    delete s;
}

void rg_server::retire_locked(Step* s) {
    const uint64_t t_done = now_ns();
    const uint64_t* cards = reinterpret_cast<const uint64_t*>(s->h + s->L.o_cards);
    const uint64_t* dig = reinterpret_cast<const uint64_t*>(s->h + s->L.o_digest);
    const uint64_t* bmb = reinterpret_cast<const uint64_t*>(s->h + s->L.o_bm_begin);
    const uint32_t err = *reinterpret_cast<const uint32_t*>(s->h + s->L.o_err);
    for (uint32_t i = 0; i < s->tickets.size(); ++i) {
        Entry& e = *entries[s->tickets[i]];
        e.done = true;
        e.done_ns = t_done;
        e.status = err ? RG_EDEVICE : RG_OK;
        e.card = cards[i];
        e.digest = (e.q.flags & RG_FLAG_DIGEST) ? dig[i] : 0;
        e.n_containers = bmb[i + 1] - bmb[i];
        e.c_end = bmb[i + 1];
        ++n_done;
        if (auto_release) {
            e.released = true;
            --s->live;
        }
    }
    // results are copied out: the staging buffer serves the next step; the
    // arena region stays until every query of the step is released
    pinned_free.push_back(s->h);
    s->h = nullptr;
    if (s->live == 0) free_step_locked(s);
}

void rg_server::run() {
    (void)hipSetDevice(c->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = false;
        // retire finished steps in order
        while (!inflight.empty()) {
            Step* s = inflight.front();
            const hipError_t q = hipEventQuery(s->done);
            if (q == hipErrorNotReady) break;
            inflight.pop_front();
            if (q != hipSuccess) fatal = std::string("step failed: ") + hipGetErrorString(q);
            retire_locked(s);
            progressed = true;
        }
        if (progressed) cv_done.notify_all();
        if (stop && pending.empty() && inflight.empty()) break;
        // admit the next step
        if (inflight.size() < max_inflight && !pending.empty() && fatal.empty()) {
            std::vector<uint64_t> take;
            uint64_t S, P, nids;
            if (admit_locked(&take, &S, &P, &nids)) {
                auto* s = new Step();
                s->L.plan((uint32_t)take.size(), nids, S, P, true);
                if (!alloc.alloc(s->L.total, &s->arena_off) || pinned_free.empty() ||
                    s->L.down_off + s->L.down_bytes > pinned_bytes) {
                    // cannot happen after admit_locked unless the staging buffer is too small
                    fatal = "step staging exceeds its pinned buffer";
                    delete s;
                } else {
                    s->d = arena + s->arena_off;
                    s->h = pinned_free.back();
                    pinned_free.pop_back();
                    s->st = streams[next_stream++ % 2];
                    s->tickets = take;
                    s->live = (uint32_t)take.size();
                    std::vector<KwQuery> qs;
                    std::vector<uint32_t> ids;
                    std::vector<KwPart> parts;
                    std::vector<uint64_t> nk;
                    uint32_t n_masks = 0;
                    uint64_t slot = 0;
                    bool digest = false;
                    for (uint32_t i = 0; i < take.size(); ++i) {
                        Entry& e = *entries[take[i]];
                        digest |= (e.q.flags & RG_FLAG_DIGEST) != 0;
                        e.step = s;
                        e.q_in_step = i;
                        qs.push_back(KwQuery{(uint32_t)e.q.op, e.q.k, (uint32_t)ids.size(),
                                             (e.q.flags & RG_FLAG_MATERIALIZE) ? KW_MATERIALIZE : 0u, slot,
                                             (uint32_t)e.b.kbound, 0});
                        nk.resize(e.q.k);
                        for (uint32_t j = 0; j < e.q.k; ++j) nk[j] = h_bm_begin[e.ids[j] + 1] - h_bm_begin[e.ids[j]];
                        split_query(&qs.back(), i, nk.data(), 1, pool.key_index != nullptr, &parts, &n_masks);
                        ids.insert(ids.end(), e.ids.begin(), e.ids.end());
                        slot += e.b.kbound;
                    }
                    pending.erase(pending.begin(), pending.begin() + take.size());
                    s->L.n_parts = (uint32_t)parts.size();
                    s->L.n_masks = n_masks;
                    s->L.pairs = false;
                    s->L.whole = false;
                    s->L.big = false;
                    for (const KwQuery& Q : qs) {
                        s->L.pairs |= Q.k <= 2;
                        s->L.whole |= Q.k > 2 && !(Q.flags & KW_SPLIT);
                        s->L.big |= Q.k > 2;
                    }
                    stage_upload(s->L, s->h, qs, ids, parts);
                    ++n_steps;
                    sum_batch += take.size();
                    lk.unlock();
                    std::string step_err;
                    rg_status st = step_enqueue(&step_err, pool, s->L, s->d, own_out(s->L, s->d), s->h, s->st, digest);
                    if (st == RG_OK && hipEventCreateWithFlags(&s->done, hipEventDisableTiming) != hipSuccess)
                        st = RG_EDEVICE;
                    if (st == RG_OK && hipEventRecord(s->done, s->st) != hipSuccess) st = RG_EDEVICE;
                    lk.lock();
                    if (st != RG_OK) fatal = step_err.empty() ? "step enqueue failed" : step_err;
                    inflight.push_back(s);
                    progressed = true;
                }
            }
        }
        if (!progressed) {
            if (inflight.empty())
                cv_work.wait_for(lk, std::chrono::microseconds(200));
            else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(5));
                lk.lock();
            }
        }
    }
}

extern "C" {

rg_status rg_serve_start(rg_ctx* c, const rg_pool* pool, uint64_t arena_bytes, uint32_t max_batch,
                         uint32_t max_inflight, rg_server** out) {
    if (!c) return RG_EINVAL;
    if (!out) return fail(c, RG_EINVAL, "null server pointer");
    *out = nullptr;
    if (!pool_ok(pool)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    if (max_batch < 1 || max_batch > 4096 || max_inflight < 1 || max_inflight > 2 || arena_bytes < (1u << 20))
        return fail(c, RG_EINVAL, "rg_serve_start: 1 <= max_batch <= 4096, 1 <= max_inflight <= 2, arena >= 1 MiB");
    HIPCHK(c, hipSetDevice(c->device));
    auto* s = new rg_server();
    s->c = c;
    s->pool = *pool;
    s->max_batch = max_batch;
    s->max_inflight = max_inflight;
    s->h_bm_begin.resize(pool->n_bitmaps + 1);
    s->h_wbytes.resize(std::max<uint32_t>(pool->n_bitmaps, 1));
    s->h_span.resize(std::max<uint32_t>(pool->n_bitmaps, 1));
    auto cleanup = [&](rg_status st, const char* m) {
        for (uint8_t* p : s->pinned_free) (void)hipHostFree(p);
        if (s->arena) (void)hipFree(s->arena);
        for (auto& x : s->streams)
            if (x) (void)hipStreamDestroy(x);
        delete s;
        return fail(c, st, m);
    };
    if (hipMemcpy(s->h_bm_begin.data(), pool->bm_begin, 8ull * (pool->n_bitmaps + 1), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        (pool->n_bitmaps && hipMemcpy(s->h_wbytes.data(), pool->bm_wbytes, 8ull * pool->n_bitmaps,
                                      hipMemcpyDeviceToHost) != hipSuccess))
        return cleanup(RG_EDEVICE, "rg_serve_start: pool metadata readback failed");
    if (pool->n_bitmaps) {
        void* d_span = nullptr;
        if (hipMalloc(&d_span, 4ull * pool->n_bitmaps) != hipSuccess)
            return cleanup(RG_EDEVICE, "rg_serve_start: key span buffer");
        launch_kw_key_span(pool->bm_begin, pool->keys, pool->n_bitmaps, reinterpret_cast<uint32_t*>(d_span), nullptr);
        const bool ok = hipMemcpy(s->h_span.data(), d_span, 4ull * pool->n_bitmaps, hipMemcpyDeviceToHost) ==
                        hipSuccess;
        (void)hipFree(d_span);
        if (!ok) return cleanup(RG_EDEVICE, "rg_serve_start: key span readback failed");
    }
    if (hipMalloc(&s->arena, arena_bytes) != hipSuccess) return cleanup(RG_EDEVICE, "rg_serve_start: arena");
    s->alloc.reset(arena_bytes);
    for (auto& x : s->streams)
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess)
            return cleanup(RG_EDEVICE, "rg_serve_start: stream");
    // staging per in-flight step, sized for max_batch queries of up to KW_MAX_K ids
    StepLayout L;
    L.plan(max_batch, (uint64_t)max_batch * KW_MAX_K, 0, 0, true);
    s->pinned_bytes = L.down_off + L.down_bytes;
    for (uint32_t i = 0; i < max_inflight; ++i) {
        void* p = nullptr;
        if (hipHostMalloc(&p, s->pinned_bytes, hipHostMallocDefault) != hipSuccess)
            return cleanup(RG_EDEVICE, "rg_serve_start: pinned staging");
        s->pinned_free.push_back(reinterpret_cast<uint8_t*>(p));
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return RG_OK;
}

rg_status rg_serve_submit(rg_server* s, const rg_query* q, uint64_t arrival_ns, uint64_t* ticket) {
    if (!s || !ticket) return RG_EINVAL;
    if (!query_host_ok(s, q)) return fail(s->c, RG_EINVAL, "rg_serve_submit: bad query (op, k, ids or flags)");
    auto e = std::make_unique<Entry>();
    e->q = *q;
    e->ids.assign(q->ids, q->ids + q->k);
    e->q.ids = nullptr;
    std::vector<uint64_t> meta(4 * q->k);
    for (uint32_t j = 0; j < q->k; ++j) {
        const uint32_t b = e->ids[j];
        meta[4 * j] = s->h_bm_begin[b + 1] - s->h_bm_begin[b];
        meta[4 * j + 1] = s->h_wbytes[b];
        meta[4 * j + 2] = 1;
        meta[4 * j + 3] = s->h_span[b];
    }
    e->b = query_bounds(q->op, q->k, meta.data(), q->flags & RG_FLAG_MATERIALIZE);
    e->arrival_ns = arrival_ns ? arrival_ns : now_ns();
    {
        StepLayout L;
        L.plan(1, q->k, e->b.kbound, e->b.pbound, true);
        if (L.total > s->alloc.cap())
            return fail(s->c, RG_ECAPACITY, "rg_serve_submit: the query's result bound exceeds the arena");
    }
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->fatal.empty()) return fail(s->c, RG_EDEVICE, s->fatal);
    const uint64_t t = s->next_ticket++;
    s->entries[t] = std::move(e);
    s->pending.push_back(t);
    *ticket = t;
    s->cv_work.notify_one();
    return RG_OK;
}

rg_status rg_serve_poll(rg_server* s, uint64_t ticket, int wait, rg_result* r) {
    if (!s || !r) return RG_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return fail(s->c, RG_EINVAL, "rg_serve_poll: unknown ticket");
    Entry& e = *it->second;
    if (wait)
        s->cv_done.wait(lk, [&] { return e.done || !s->fatal.empty(); });
    memset(r, 0, sizeof(*r));
    r->done = e.done ? 1 : 0;
    if (!e.done) return s->fatal.empty() ? RG_OK : fail(s->c, RG_EDEVICE, s->fatal);
    r->status = e.status;
    r->card = e.card;
    r->digest = e.digest;
    r->n_containers = e.n_containers;
    r->latency_ns = e.done_ns - e.arrival_ns;
    if (!e.released && e.step) {
        const Step* st = e.step;
        const StepLayout& L = st->L;
        uint8_t* d = st->d;
        r->view = rg_pool{1, e.c_end, L.P, reinterpret_cast<const uint64_t*>(d + L.o_bm_begin) + e.q_in_step,
                          reinterpret_cast<const uint16_t*>(d + L.o_keys), d + L.o_types,
                          reinterpret_cast<const uint32_t*>(d + L.o_card),
                          reinterpret_cast<const uint32_t*>(d + L.o_size),
                          reinterpret_cast<const uint64_t*>(d + L.o_off), d + L.o_payload,
                          reinterpret_cast<const uint64_t*>(d + L.o_bm_card) + e.q_in_step,
                          reinterpret_cast<const uint64_t*>(d + L.o_bm_wbytes) + e.q_in_step};
    }
    return RG_OK;
}

rg_status rg_serve_release(rg_server* s, uint64_t ticket) {
    if (!s) return RG_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return fail(s->c, RG_EINVAL, "rg_serve_release: unknown ticket");
    Entry& e = *it->second;
    if (!e.done) return fail(s->c, RG_EINVAL, "rg_serve_release: query not finished");
    if (!e.released && e.step) {
        e.released = true;
        if (--e.step->live == 0) s->free_step_locked(e.step);
    }
    s->entries.erase(it);
    return RG_OK;
}

rg_status rg_serve_replay(rg_server* s, uint64_t n, const rg_query* qs, const uint64_t* arrival_ns,
                          uint64_t* latency_ns, uint64_t* cards, uint64_t* digests) {
    if (!s || (n && (!qs || !arrival_ns))) return RG_EINVAL;
    std::vector<uint64_t> tickets(n);
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->auto_release = true;
    }
    const uint64_t t0 = now_ns();
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t due = t0 + arrival_ns[i];
        while (now_ns() < due) std::this_thread::yield();
        if (rg_status st = rg_serve_submit(s, &qs[i], due, &tickets[i])) return st;
    }
    for (uint64_t i = 0; i < n; ++i) {
        rg_result r;
        if (rg_status st = rg_serve_poll(s, tickets[i], 1, &r)) return st;
        if (r.status != RG_OK) return fail(s->c, (rg_status)r.status, "rg_serve_replay: a query failed");
        if (latency_ns) latency_ns[i] = r.latency_ns;
        if (cards) cards[i] = r.card;
        if (digests) digests[i] = r.digest;
        std::lock_guard<std::mutex> g(s->mu);
        s->entries.erase(tickets[i]);
    }
    std::lock_guard<std::mutex> g(s->mu);
    s->auto_release = false;
    return RG_OK;
}

rg_status rg_serve_stop(rg_server* s, rg_serve_stats* stats) {
    if (!s) return RG_EINVAL;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->c->device);
    (void)hipDeviceSynchronize();
    if (stats) {
        stats->queries = s->n_done;
        stats->steps = s->n_steps;
        stats->mean_batch = s->n_steps ? (double)s->sum_batch / (double)s->n_steps : 0.0;
        stats->arena_peak_bytes = s->alloc.peak();
        stats->deferred = s->n_deferred;
    }
    const bool ok = s->fatal.empty();
    const std::string msg = s->fatal;
    // steps whose queries were never released
    std::vector<Step*> steps;
    for (auto& kv : s->entries)
        if (kv.second->step && !kv.second->released) {
            Step* st = kv.second->step;
            if (std::find(steps.begin(), steps.end(), st) == steps.end()) steps.push_back(st);
        }
    for (Step* st : steps) {
        if (st->h) s->pinned_free.push_back(st->h);
        (void)hipEventDestroy(st->done);
        delete st;
    }
    for (uint8_t* p : s->pinned_free) (void)hipHostFree(p);
    (void)hipFree(s->arena);
    for (auto& x : s->streams) (void)hipStreamDestroy(x);
    rg_ctx* c = s->c;
    delete s;
    return ok ? RG_OK : fail(c, RG_EDEVICE, msg);
}

}  // extern "C"
