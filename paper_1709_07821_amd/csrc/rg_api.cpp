// rg_api.cpp - the C ABI: context, workspace, and the orchestration of one
// batched call (pair preparation -> key matching in waves -> binned compute
// kernels -> output assembly or count finishing).
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include <mutex>

#include "rg_host.h"

// Scratch of roaring_batch_static, for callers that cannot allocate: a fixed
// array in the library's device code. Each GPU the library runs on holds its
// own copy, at its own address, until the process ends. Host code never uses
// this name as an address: rg_create looks the address up once per device
// (hipGetSymbolAddress) and keeps it in static_scratch_ptr.
static __device__ __align__(256) uint8_t scratch[RG_STATIC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex static_scratch_mu;
void* static_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device`, which must be the current device.
rg_status static_scratch_init(int device, void** out) {
    if (device < 0 || device >= MAX_DEVICES) return RG_ENOTSUP;
    std::lock_guard<std::mutex> lk(static_scratch_mu);
    if (!static_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RG_EDEVICE;
        static_scratch_ptr[device] = p;
    }
    *out = static_scratch_ptr[device];
    return RG_OK;
}

rg_status drain_profile(rg_ctx* c) {
    if (c->prof_fused_pending) {
        // matched container pairs counted by timed fused launches (the context's
        // device block; ordered after them on the device by the wait below)
        uint64_t* h = static_cast<uint64_t*>(c->host);
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipMemcpy(h, fused_matched_word(c), 8, hipMemcpyDeviceToHost));
        c->prof_items[PROF_FUSED][0] += *h;
        HIPCHK(c, hipMemset(fused_matched_word(c), 0, 8));
        c->prof_fused_pending = false;
    }
    for (auto& p : c->pend) {
        float ms = 0;
        HIPCHK(c, hipEventSynchronize(p.b));
        HIPCHK(c, hipEventElapsedTime(&ms, p.a, p.b));
        c->prof_ms[p.cls][p.mat] += ms;
        c->prof_launches[p.cls][p.mat] += 1;
        c->prof_items[p.cls][p.mat] += p.items;
        c->evpool.push_back(p.a);
        c->evpool.push_back(p.b);
    }
    c->pend.clear();
    return RG_OK;
}

}  // namespace

// ---- workspace sizing (shared by the calls and rg_workspace_size)

// per-pair scratch of an asynchronous count-only call
size_t count_pair_bytes(uint64_t n_pairs) {
    return align256(4 * n_pairs) + align256(8 * n_pairs) + align256(8 * (n_pairs + 1)) +
           align256(8 * scan_partials_needed(n_pairs)) + align256(4);
}

// Whether packing the pools' metadata pays for a count-only call: when it is
// expected to visit at least META_PACK_FACTOR candidate keys per container
// (estimate: pairs x the smaller mean key count per bitmap).
bool count_pack_pays(const rg_pool* A, const rg_pool* B, uint64_t n_pairs, uint64_t* n_records, bool* same_pool) {
    const bool same = A->keys == B->keys && A->off == B->off && A->n_containers == B->n_containers;
    *same_pool = same;
    const uint64_t nA = A->n_containers, nB = same ? 0 : B->n_containers;
    *n_records = nA + nB;
    if (!*n_records || (A->meta && B->meta)) return false;
    const double kA = A->n_bitmaps ? (double)A->n_containers / A->n_bitmaps : 0.0;
    const double kB = B->n_bitmaps ? (double)B->n_containers / B->n_bitmaps : 0.0;
    const double est = (double)n_pairs * std::min(kA, kB);
    return est >= (double)META_PACK_FACTOR * (double)(nA + nB);
}

// per-pair scratch of the materialising (binned) path
size_t mat_pair_bytes(uint64_t n_pairs) {
    return align256(4 * n_pairs) + align256(8 * n_pairs) + align256(4 * n_pairs) + align256(8 * n_pairs);
}

// scratch of one wave of S candidate slots over at most P pairs
size_t wave_bytes(uint64_t S, uint64_t P, bool kw) {
    const uint64_t nb = (uint64_t)NBINS * match_blocks(S);
    size_t b = 0;
    for (size_t x : {sizeof(Task) * S, 4 * S, 8 * S, 4 * S, 1 * S, 4 * S, 8 * S, 4 * S})
        b += align256(x);  // tasks, ub, slot_off, res_card, res_type, res_size, out_idx, lists
    // scan partials serve the slot scans (S) and the pair-offset scan (P)
    b += align256(8 * (P + 1)) + align256(8 * scan_partials_needed(std::max(S, P))) + align256(4 * nb) +
         align256(8 * nb) + align256(8 * scan_partials_needed(nb));
    if (kw) b += align256(sizeof(KwQuery) * P) + align256(8 * P);
    return b;
}

// most candidate slots one pair can need (a wave holds whole pairs)
uint64_t max_pair_slots(int op, bool mat) {
    if (!mat) return 65536;
    return (op == RG_OR || op == RG_XOR) ? 131072 : 65536;
}

// Persistent grid of the fused count kernel: as many workgroups as are
// resident at once, never more blocks than there can be candidate blocks
// (65536 keys per pair at most).
uint32_t fused_grid(rg_ctx* c, uint64_t n_pairs) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    const uint64_t cap = (uint64_t)cus * count_fused_blocks_per_cu();
    const uint64_t most = n_pairs * (65536 / MATCH_SLOTS);
    return (uint32_t)std::max<uint64_t>(1, std::min(cap, most));
}

// Count-only batched call with no host round trip: per-pair preparation,
// device scan of the candidate counts, the fused match-and-count kernel, and
// the conversion to the requested count (Section 5.9 identities). Pair indices
// outside their pool give count 0 and set the context's asynchronous error
// flag (rg_sync reports it).
// `fixed`, when given, is the device region all scratch comes from (the
// static scratch of roaring_batch_static); kernel timing is then skipped, so
// the call creates no events either.
rg_status run_count_async(rg_ctx* c, int op, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia,
                          const uint32_t* d_ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs, uint32_t flags,
                          uint64_t* d_cards, double* d_jacc, hipStream_t st, void* fixed = nullptr,
                          size_t fixed_bytes = 0) {
    Scratch sc = fixed ? Scratch(c, fixed, fixed_bytes) : Scratch(c);
    void* base = nullptr;
    if (rg_status s = sc.take(WS_PAIRS, count_pair_bytes(n_pairs), &base)) return s;
    Bump bp{(uint8_t*)base};
    uint32_t* n_cand = bp.take<uint32_t>(n_pairs);
    long long* acc = bp.take<long long>(n_pairs);
    uint64_t* cand_off = bp.take<uint64_t>(n_pairs + 1);
    uint64_t* partials = bp.take<uint64_t>(scan_partials_needed(n_pairs));
    uint32_t* next_blk = bp.take<uint32_t>(1);
    PoolView pa = view(*A), pb = view(*B);
    // Packed metadata records: the pools' own, or packed here when the call is
    // expected to visit many candidate keys per container (one pass, 16 B per
    // container). Without the memory for it the call reads the arrays.
    uint64_t nrec = 0;
    bool same = false;
    if (count_pack_pays(A, B, n_pairs, &nrec, &same)) {
        void* mm = nullptr;
        bool ok = false;
        if (sc.caller()) {
            ok = align256(16 * nrec) <= sc.left() && sc.take(WS_META, 16 * nrec, &mm) == RG_OK;
        } else {
            ok = grow_device(c, &c->ws_meta, &c->ws_meta_bytes, 16 * nrec) == RG_OK;
            mm = c->ws_meta;
            if (!ok) (void)hipGetLastError();  // not an error of the call: it runs unpacked
        }
        if (ok) {
            u32x4* ma = reinterpret_cast<u32x4*>(mm);
            launch_pack_meta(view(*A), A->n_containers, ma, st);
            if (!same) launch_pack_meta(view(*B), B->n_containers, ma + A->n_containers, st);
            pa.meta = ma;
            pb.meta = same ? ma : ma + A->n_containers;
        }
    }
    // Key-presence indexes (10 KiB per bitmap) of pools with many keys per
    // bitmap: key matching then finds each candidate key with a bit test and a
    // popcount instead of a binary search. Without the memory the call searches.
    {
        const bool same = A->keys == B->keys && A->bm_begin == B->bm_begin;
        const uint64_t nA = kidx_pays(A, n_pairs) ? A->n_bitmaps : 0, nB = (!same && kidx_pays(B, n_pairs)) ? B->n_bitmaps : 0;
        if (nA + nB) {
            void* km = nullptr;
            bool ok = false;
            const size_t need = (size_t)RG_KEY_INDEX_BYTES * (nA + nB);
            if (sc.caller()) {
                ok = align256(need) <= sc.left() && sc.take(WS_KIDX, need, &km) == RG_OK;
            } else {
                ok = grow_device(c, &c->ws_kidx, &c->ws_kidx_bytes, need) == RG_OK;
                km = c->ws_kidx;
                if (!ok) (void)hipGetLastError();
            }
            if (ok) {
                uint8_t* kb = static_cast<uint8_t*>(km);
                if (nA) {
                    launch_key_index(view(*A), A->n_bitmaps, kb, st);
                    pa.kidx = kb;
                    if (same) pb.kidx = kb;
                }
                if (nB) {
                    launch_key_index(view(*B), B->n_bitmaps, kb + (size_t)RG_KEY_INDEX_BYTES * nA, st);
                    pb.kidx = kb + (size_t)RG_KEY_INDEX_BYTES * nA;
                }
            }
        }
    }
    launch_pair_prep(RG_AND, false, pa, pb, A->n_bitmaps, B->n_bitmaps, d_ia, d_ib, ia0, ib0, n_pairs, n_cand,
                     nullptr, nullptr, acc, async_err_word(c), st, next_blk);
    launch_scan_u32_u64(n_cand, cand_off, n_pairs, 0, partials, cand_off + n_pairs, st);
    MatchArgs m{};
    m.op = RG_AND;
    m.materialize = false;
    m.A = pa;
    m.B = pb;
    m.ia = d_ia;
    m.ib = d_ib;
    m.ia0 = ia0;
    m.ib0 = ib0;
    m.pair0 = 0;
    m.n_pairs = (uint32_t)n_pairs;
    m.cand_off = cand_off;
    m.n_cand = 0;  // read on the device
    m.dispatch_mode = c->dispatch_mode;
    m.fixed_bin = c->fixed_bin;
    m.gallop_ratio = c->gallop_ratio;
    m.thread_max = c->thread_max;
    m.mlp_table = c->mlp_table;
    m.fuse_thread = true;
    m.acc = acc;
    const uint32_t grid = fused_grid(c, n_pairs);
    if (fixed || !c->prof) {
        launch_count_fused(m, next_blk, grid, st);
    } else {
        // timed: the kernel also counts the matched container pairs (the
        // class's items, read when the timings are drained)
        m.matched = fused_matched_word(c);
        timed(c, PROF_FUSED, false, 0, st, [&] { launch_count_fused(m, next_blk, grid, st); });
        c->prof_fused_pending = true;
    }
    launch_finish_counts(RG_AND, op, acc, pa, pb, A->n_bitmaps, B->n_bitmaps, d_ia, d_ib, ia0, ib0, 0,
                         (uint32_t)n_pairs, (flags & RG_FLAG_CARD) ? d_cards : nullptr,
                         (flags & RG_FLAG_JACCARD) ? d_jacc : nullptr, st);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

// one batched call (also used by the dispatcher's cost sampling)
// single (materialising, op RG_ANDNOT): every pair is the union of its A
// bitmap alone, i.e. that bitmap rebuilt in P1 form (rg_pool_canonicalize)
rg_status run_batch(rg_ctx* c, int op, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia,
                    const uint32_t* d_ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs, uint32_t flags, rg_out* out,
                    uint64_t* d_cards, double* d_jacc, hipStream_t st, bool single) {
    if (!c) return RG_EINVAL;
    if (op < RG_AND || op > RG_ANDNOT) return fail(c, RG_EINVAL, "op must be RG_AND..RG_ANDNOT");
    if (!pool_ok(A) || !pool_ok(B)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    const bool mat = flags & RG_FLAG_MATERIALIZE;
    if (!(flags & (RG_FLAG_MATERIALIZE | RG_FLAG_CARD | RG_FLAG_JACCARD)))
        return fail(c, RG_EINVAL, "flags select no output");
    if ((flags & RG_FLAG_CARD) && !d_cards) return fail(c, RG_EINVAL, "RG_FLAG_CARD needs d_cards");
    if ((flags & RG_FLAG_JACCARD) && !d_jacc) return fail(c, RG_EINVAL, "RG_FLAG_JACCARD needs d_jacc");
    if (mat && (!out || !out->bm_begin || !out->keys || !out->types || !out->card || !out->size || !out->off ||
                !out->payload || !out->bm_card))
        return fail(c, RG_EINVAL, "materialisation needs a complete rg_out");
    if (n_pairs > 0xFFFFFFFFull) return fail(c, RG_EINVAL, "at most 2^32-1 pairs per call");
    if ((d_ia == nullptr) != (d_ib == nullptr)) return fail(c, RG_EINVAL, "d_ia and d_ib go together");
    HIPCHK(c, hipSetDevice(c->device));
    WorkspaceOrder order(c, st);
    if (mat) {
        out->n_containers = 0;
        out->payload_used = 0;
        out->needed_containers = 0;
        out->needed_payload_bytes = 0;
    }
    if (n_pairs == 0) {
        if (mat) launch_fill_u64(out->bm_begin, 0, 1, st);
        return RG_OK;
    }
    // count-only calls (other than the dispatcher's cost sampling) run without
    // a host round trip
    if (!mat && !c->cost_out)
        return run_count_async(c, op, A, B, d_ia, d_ib, ia0, ib0, n_pairs, flags, d_cards, d_jacc, st);
    PoolView pa = view(*A), pb = view(*B);
    Scratch sc(c);

    // ---- per-pair preparation
    Bump bp{nullptr};
    void* pbase = nullptr;
    if (rg_status s = sc.take(WS_PAIRS, mat_pair_bytes(n_pairs), &pbase)) return s;
    bp.base = (uint8_t*)pbase;
    uint32_t* n_cand = bp.take<uint32_t>(n_pairs);
    uint64_t* bound = bp.take<uint64_t>(n_pairs);
    uint32_t* min_cont = bp.take<uint32_t>(n_pairs);
    long long* acc = bp.take<long long>(n_pairs);
    uint32_t* d_err = reinterpret_cast<uint32_t*>(c->small);
    uint32_t* bin_info = d_err + 128;                              // [2 NBINS] counts, offsets
    uint64_t* bin_total = reinterpret_cast<uint64_t*>(d_err + 160);
    uint64_t* totals = reinterpret_cast<uint64_t*>(d_err + 64);  // [0] payload end, [1] container end
    uint64_t* pair_totals = reinterpret_cast<uint64_t*>(d_err + 256);  // launch_pair_totals' four sums

    // Count-only calls accumulate |A n B| for every operation and convert at
    // the end (Section 5.9 identities): the kernels then depend on the
    // operation only when they materialise.
    const int kop = mat ? op : RG_AND;
    launch_fill_u32(d_err, 0, 1, st);
    launch_pair_prep(kop, mat, pa, pb, A->n_bitmaps, B->n_bitmaps, d_ia, d_ib, ia0, ib0, n_pairs, n_cand, bound,
                     min_cont, acc, d_err, st);
    const size_t host_pairs = align256(4 * n_pairs);
    uint8_t* hbase = nullptr;
    if (rg_status s = host_buffer(c, host_pairs + 4096 + align256(8 * (n_pairs + 1)) + 512, &hbase)) return s;
    Bump hb{hbase};
    uint32_t* h_cand = hb.take<uint32_t>(n_pairs);  // per-pair slots, read back only for waves of pairs
    uint32_t* h_small = hb.take<uint32_t>(1024);
    uint64_t* h_coff = hb.take<uint64_t>(n_pairs + 1);
    // sizing from device-side sums (a few words back, not the per-pair arrays)
    launch_pair_totals(n_cand, mat ? bound : nullptr, mat ? min_cont : nullptr, n_pairs, pair_totals, st);
    HIPCHK(c, hipMemcpyAsync(h_small + 256, pair_totals, 32, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(h_small, d_err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (h_small[0]) return fail(c, RG_EINVAL, "pair index out of range of its pool");
    const uint64_t* h_tot = reinterpret_cast<const uint64_t*>(h_small + 256);
    const uint64_t total_cand = h_tot[0], most_cand = h_tot[3];

    if (mat) {
        const uint64_t tb = h_tot[1], tcont = h_tot[2];
        out->needed_payload_bytes = tb;
        out->needed_containers = tcont;
        if (out->cap_payload_bytes < tb || out->cap_containers < tcont)
            return fail(c, RG_ECAPACITY, "output arena too small");
        launch_fill_u64(out->bm_card, 0, n_pairs, st);
        if (out->bm_wbytes) launch_fill_u64(out->bm_wbytes, 0, n_pairs, st);
    }

    // ---- plan waves of at most S_cap candidate slots (a caller workspace
    // bounds S_cap by what is left of it; a wave holds whole pairs)
    const bool kw = mat && op != RG_AND;
    uint64_t S_cap = c->max_wave_slots;
    if (sc.caller()) {
        uint64_t lo = 0, hi = S_cap;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) / 2;
            if (wave_bytes(mid, n_pairs, kw) <= sc.left()) lo = mid;
            else hi = mid - 1;
        }
        S_cap = lo;
        if (most_cand > S_cap)
            return fail(c, RG_ECAPACITY,
                        "workspace too small for one pair's candidate slots (rg_workspace_size gives enough)");
    }
    // one wave when every candidate slot fits (its pair offsets scanned on the
    // device); otherwise waves of whole pairs planned from the per-pair counts
    const bool one_wave = total_cand <= S_cap;
    std::vector<uint64_t> wstart{0};
    uint64_t S_max = 0, P_max = 0;
    if (one_wave) {
        S_max = total_cand;
        P_max = n_pairs;
        wstart.push_back(n_pairs);
    } else {
        HIPCHK(c, hipMemcpyAsync(h_cand, n_cand, 4 * n_pairs, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        uint64_t accs = 0;
        for (uint64_t p = 0; p < n_pairs; ++p) {
            if (accs + h_cand[p] > S_cap && accs > 0) {
                S_max = std::max(S_max, accs);
                P_max = std::max(P_max, p - wstart.back());
                wstart.push_back(p);
                accs = 0;
            }
            accs += h_cand[p];
        }
        S_max = std::max(S_max, accs);
        P_max = std::max(P_max, n_pairs - wstart.back());
        wstart.push_back(n_pairs);
    }

    // materialised OR / XOR / ANDNOT run through the k-way path (two bitmaps
    // per query): key set per pair, then one workgroup per result key
    void* wbase = nullptr;
    if (rg_status s = sc.take(WS_WAVE, wave_bytes(S_max, P_max, kw), &wbase)) return s;
    Bump wb{(uint8_t*)wbase};
    Task* tasks = wb.take<Task>(S_max);
    uint32_t* ub = wb.take<uint32_t>(S_max);
    uint64_t* slot_off = wb.take<uint64_t>(S_max);
    uint32_t* res_card = wb.take<uint32_t>(S_max);
    uint8_t* res_type = wb.take<uint8_t>(S_max);
    uint32_t* res_size = wb.take<uint32_t>(S_max);
    uint64_t* out_idx = wb.take<uint64_t>(S_max);
    uint32_t* bin_lists = wb.take<uint32_t>(S_max);
    uint64_t* cand_off = wb.take<uint64_t>(P_max + 1);
    uint64_t* partials = wb.take<uint64_t>(scan_partials_needed(std::max(S_max, P_max)));
    uint32_t* blk_cnt = wb.take<uint32_t>((size_t)NBINS * match_blocks(S_max));
    uint64_t* blk_off = wb.take<uint64_t>((size_t)NBINS * match_blocks(S_max));
    uint64_t* bpart = wb.take<uint64_t>(scan_partials_needed((uint64_t)NBINS * match_blocks(S_max)));
    KwQuery* kw_queries = kw ? wb.take<KwQuery>(P_max) : nullptr;
    uint32_t* kw_ids = kw ? wb.take<uint32_t>(2 * P_max) : nullptr;

    uint64_t out_base = 0, pay_base = 0;
    const size_t nw = wstart.size() - 1;
    for (size_t w = 0; w < nw; ++w) {
        const uint64_t p0 = wstart[w], p1 = wstart[w + 1];
        const uint32_t np = (uint32_t)(p1 - p0);
        uint64_t C;
        if (one_wave) {
            C = total_cand;
            launch_scan_u32_u64(n_cand, cand_off, np, 0, partials, cand_off + np, st);
        } else {
            h_coff[0] = 0;
            for (uint32_t q = 0; q < np; ++q) h_coff[q + 1] = h_coff[q] + h_cand[p0 + q];
            C = h_coff[np];
            HIPCHK(c, hipMemcpyAsync(cand_off, h_coff, 8 * (np + 1), hipMemcpyHostToDevice, st));
        }
        const bool last = w + 1 == nw;
        if (C == 0) {
            if (mat) {
                launch_fill_u64(totals + 1, out_base, 1, st);
                launch_bm_begin(cand_off, out_idx, 0, totals + 1, np, p0, out->bm_begin, last, st);
            }
            continue;
        }
        uint64_t pay_end = 0;
        if (kw) {
            launch_kw_pair_queries(op, d_ia, d_ib, ia0, ib0, p0, np, cand_off, kw_queries, kw_ids, st, single);
            KwArgs ka;
            ka.P0 = pa;
            ka.P1 = pb;
            ka.pair_base = (uint32_t)p0;
            ka.queries = kw_queries;
            ka.n_queries = np;
            ka.ids = kw_ids;
            ka.tasks = tasks;
            ka.n_slots = C;
            ka.ub = ub;
            ka.res_card = res_card;
            ka.so = SlotOut{slot_off, out->payload, res_card, res_type, res_size};
            ka.so.cap = out->cap_payload_bytes;
            ka.so.err = d_err;
            ka.acc = nullptr;
            ka.err = d_err;
            ka.small = !(c->dispatch_mode == 2 && c->fixed_bin == BIN_GEN);
            launch_kw_keys(ka, st);
            launch_kw_bounds(ka, st, true);  // pairwise queries only
            launch_scan_u32_u64(ub, slot_off, C, pay_base, partials, totals, st);
            timed(c, PROF_KWSMALL, true, C, st, [&] { launch_kw_small(ka, st); });
            timed(c, PROF_KWBB, true, C, st, [&] { launch_kw_bb(ka, st); });
            timed(c, PROF_KWEVAL, true, C, st, [&] { launch_kw_eval(ka, st); });
        } else {
            MatchArgs m;
            m.op = kop;
            m.materialize = mat;
            m.A = pa;
            m.B = pb;
            m.ia = d_ia;
            m.ib = d_ib;
            m.ia0 = ia0;
            m.ib0 = ib0;
            m.pair0 = p0;
            m.n_pairs = np;
            m.cand_off = cand_off;
            m.n_cand = C;
            m.tasks = tasks;
            m.ub = ub;
            m.res_card = res_card;
            m.blk_cnt = blk_cnt;
            m.dispatch_mode = c->dispatch_mode;
            m.fixed_bin = c->fixed_bin;
            m.gallop_ratio = c->gallop_ratio;
            m.thread_max = c->thread_max;
            m.mlp_table = c->mlp_table;
            // cost sampling times the thread kernel itself, so nothing is fused then
            m.fuse_thread = !mat && !c->cost_out;
            m.acc = acc;
            launch_match(m, st);
            if (mat) launch_scan_u32_u64(ub, slot_off, C, pay_base, partials, totals, st);
            launch_bin_layout(blk_cnt, match_blocks(C), blk_off, bpart, bin_total, bin_info, nullptr, st);
            launch_bin_scatter(tasks, C, blk_cnt, blk_off, bin_lists, st);
            HIPCHK(c, hipMemcpyAsync(h_small, bin_info, 8 * NBINS, hipMemcpyDeviceToHost, st));
            if (mat) HIPCHK(c, hipMemcpyAsync(h_small + 64, totals, 8, hipMemcpyDeviceToHost, st));
            HIPCHK(c, hipStreamSynchronize(st));
            uint32_t cnt[NBINS], boff[NBINS];
            for (int b = 0; b < NBINS; ++b) {
                cnt[b] = h_small[b];
                boff[b] = h_small[NBINS + b];
            }
            pay_end = mat ? *reinterpret_cast<uint64_t*>(h_small + 64) : 0;
            // the slots' payload bounds come from the containers' cardinalities,
            // the arena check above from bm_wbytes: a pool whose two disagree
            // fails here, before any kernel writes past the arena
            if (mat && pay_end > out->cap_payload_bytes)
                return fail(c, RG_ECAPACITY, "result payload exceeds the arena (pool bm_wbytes inconsistent with card)");

            ComputeArgs ca;
            ca.cost = nullptr;
            if (c->cost_out) {  // dispatcher training: per-slot costs of a single wave
                if (nw != 1) return fail(c, RG_EINVAL, "cost sampling needs all pairs in one wave");
                c->cost_slots = C;
                c->cost_tasks = tasks;
                if (C <= c->cost_cap) {
                    launch_fill_u32(reinterpret_cast<uint32_t*>(c->cost_out), 0, C, st);
                    ca.cost = c->cost_out;
                }
            }
            ca.op = kop;
            ca.materialize = mat;
            ca.A = pa;
            ca.B = pb;
            ca.tasks = tasks;
            ca.acc = acc;
            ca.pair0 = p0;
            ca.so = SlotOut{slot_off, mat ? out->payload : nullptr, res_card, res_type, res_size};
            ca.so.cap = out ? out->cap_payload_bytes : ~0ull;
            for (int b = 0; b < NBINS; ++b) {
                if (!cnt[b]) continue;
                if (b == BIN_FUSED) {  // already counted by key matching
                    if (c->prof) c->prof_items[BIN_FUSED][mat ? 1 : 0] += cnt[b];
                    continue;
                }
                ca.list = bin_lists + boff[b];
                ca.n = cnt[b];
                timed(c, b, mat, cnt[b], st, [&] {
                    switch (b) {
                    case BIN_BB: launch_bb(ca, st); break;
                    case BIN_AA: mat ? launch_small_list(ca, st) : launch_aa(ca, st); break;
                    case BIN_GALLOP: launch_gallop(ca, st); break;
                    case BIN_AB: launch_ab(ca, st); break;
                    case BIN_RR: launch_rr(ca, st); break;
                    case BIN_THREAD: launch_thread(ca, st); break;
                    default: launch_generic(ca, st); break;
                    }
                });
            }
        }
        HIPCHK(c, hipGetLastError());
        if (mat) {
            launch_scan_nonzero_u64(res_card, out_idx, C, out_base, partials, totals + 1, st);
            CompactArgs cp;
            cp.tasks = tasks;
            cp.n_slots = C;
            cp.res_card = res_card;
            cp.res_type = res_type;
            cp.res_size = res_size;
            cp.slot_off = slot_off;
            cp.out_idx = out_idx;
            cp.keys = out->keys;
            cp.types = out->types;
            cp.card = out->card;
            cp.size = out->size;
            cp.off = out->off;
            cp.bm_card = out->bm_card;
            cp.bm_wbytes = out->bm_wbytes;
            cp.pair0 = p0;
            launch_compact(cp, st);
            launch_bm_begin(cand_off, out_idx, C, totals + 1, np, p0, out->bm_begin, last, st);
            HIPCHK(c, hipMemcpyAsync(h_small + 66, totals + 1, 8, hipMemcpyDeviceToHost, st));
            if (kw) {
                HIPCHK(c, hipMemcpyAsync(h_small + 64, totals, 8, hipMemcpyDeviceToHost, st));
                HIPCHK(c, hipMemcpyAsync(h_small + 68, d_err, 4, hipMemcpyDeviceToHost, st));
            }
            HIPCHK(c, hipStreamSynchronize(st));
            out_base = *reinterpret_cast<uint64_t*>(h_small + 66);
            pay_base = kw ? *reinterpret_cast<uint64_t*>(h_small + 64) : pay_end;
            if (kw && (h_small[68] & 2u))
                return fail(c, RG_ECAPACITY,
                            "result payload exceeds the arena (pool cardinalities inconsistent with the payload)");
            if (kw && h_small[68]) return fail(c, RG_EDEVICE, "result key set exceeded its bound (internal error)");
        }
    }
    if (mat) {
        out->n_containers = out_base;
        out->payload_used = pay_base;
        if (flags & (RG_FLAG_CARD | RG_FLAG_JACCARD))
            launch_mat_counts(op, out->bm_card, pa, pb, d_ia, d_ib, ia0, ib0, n_pairs,
                              (flags & RG_FLAG_CARD) ? d_cards : nullptr, (flags & RG_FLAG_JACCARD) ? d_jacc : nullptr,
                              st);
    } else {
        launch_finish_counts(kop, op, acc, pa, pb, A->n_bitmaps, B->n_bitmaps, d_ia, d_ib, ia0, ib0, 0,
                             (uint32_t)n_pairs,
                             (flags & RG_FLAG_CARD) ? d_cards : nullptr, (flags & RG_FLAG_JACCARD) ? d_jacc : nullptr,
                             st);
    }
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status single(rg_ctx* c, int op, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib, uint32_t flags,
                 rg_out* out, uint64_t* d_card, double* d_j, void* stream) {
    if (!c) return RG_EINVAL;
    if (!A || !B) return fail(c, RG_EINVAL, "null pool");
    if (ia >= A->n_bitmaps || ib >= B->n_bitmaps) return fail(c, RG_EINVAL, "bitmap index out of range");
    return run_batch(c, op, A, B, nullptr, nullptr, ia, ib, 1, flags, out, d_card, d_j, (hipStream_t)stream);
}


extern "C" {

rg_status rg_create(rg_ctx** ctx, int device) {
    if (!ctx) return RG_EINVAL;
    *ctx = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return RG_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return RG_EDEVICE;
    rg_ctx* c = new rg_ctx();
    c->device = device;
    if (hipMalloc(&c->small, 4096) != hipSuccess) {
        delete c;
        return RG_EDEVICE;
    }
    if (hipMemset(c->small, 0, 4096) != hipSuccess ||
        hipHostMalloc(&c->host, HOST_STAGING_BYTES, hipHostMallocDefault) != hipSuccess) {
        (void)hipFree(c->small);
        delete c;
        return RG_EDEVICE;
    }
    c->host_bytes = HOST_STAGING_BYTES;
    // made here so that no call has to create it (roaring_batch_static creates
    // nothing), and the static scratch's address on this device
    if (hipEventCreateWithFlags(&c->ws_event, hipEventDisableTiming) != hipSuccess ||
        static_scratch_init(device, &c->static_ws) != RG_OK) {
        if (c->ws_event) (void)hipEventDestroy(c->ws_event);
        (void)hipHostFree(c->host);
        (void)hipFree(c->small);
        delete c;
        return RG_EDEVICE;
    }
    *ctx = c;
    return RG_OK;
}

rg_status rg_set_workspace(rg_ctx* c, void* d_ws, uint64_t bytes) {
    if (!c) return RG_EINVAL;
    if (d_ws && (reinterpret_cast<uintptr_t>(d_ws) & 255))
        return fail(c, RG_EINVAL, "rg_set_workspace: the workspace must be 256-byte aligned");
    if (d_ws && bytes == 0) return fail(c, RG_EINVAL, "rg_set_workspace: empty workspace");
    HIPCHK(c, hipSetDevice(c->device));
    // calls still running on the previous workspace must finish before the
    // caller reuses or frees it: wait for the last one
    if (c->ws_event_live) HIPCHK(c, hipEventSynchronize(c->ws_event));
    c->user_ws = d_ws;
    c->user_ws_bytes = d_ws ? (size_t)bytes : 0;
    return RG_OK;
}

rg_status rg_workspace_size(rg_ctx* c, int op, uint32_t flags, const rg_pool* A, const rg_pool* B,
                            uint64_t n_pairs, uint64_t* bytes) {
    if (!c) return RG_EINVAL;
    if (!bytes || !A || !B) return fail(c, RG_EINVAL, "rg_workspace_size: null argument");
    if (op < RG_AND || op > RG_ANDNOT) return fail(c, RG_EINVAL, "op must be RG_AND..RG_ANDNOT");
    if (!(flags & (RG_FLAG_MATERIALIZE | RG_FLAG_CARD | RG_FLAG_JACCARD)))
        return fail(c, RG_EINVAL, "flags select no output");
    const bool mat = flags & RG_FLAG_MATERIALIZE;
    if (!mat) {
        size_t b = count_pair_bytes(n_pairs);
        uint64_t nrec = 0;
        bool same = false;
        if (count_pack_pays(A, B, n_pairs, &nrec, &same)) b += align256(16 * nrec);
        const bool same_k = A->keys == B->keys && A->bm_begin == B->bm_begin;
        const uint64_t nk = (kidx_pays(A, n_pairs) ? A->n_bitmaps : 0) + ((!same_k && kidx_pays(B, n_pairs)) ? B->n_bitmaps : 0);
        if (nk) b += align256((size_t)RG_KEY_INDEX_BYTES * nk);
        *bytes = b;
        return RG_OK;
    }
    // the per-pair arrays and one wave that holds the largest possible pair;
    // more lets a call run in fewer waves
    const bool kw = op != RG_AND;
    *bytes = mat_pair_bytes(n_pairs) + wave_bytes(max_pair_slots(op, true), n_pairs, kw);
    return RG_OK;
}

rg_status rg_sync(rg_ctx* c, void* stream) {
    if (!c) return RG_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    uint32_t* h = reinterpret_cast<uint32_t*>(c->host);
    HIPCHK(c, hipMemcpyAsync(h, async_err_word(c), 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (*h) {
        launch_fill_u32(async_err_word(c), 0, 1, st);
        HIPCHK(c, hipStreamSynchronize(st));
        return fail(c, RG_EINVAL, "an asynchronous call had a pair index out of range of its pool");
    }
    return RG_OK;
}

void rg_destroy(rg_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->ws_pairs) (void)hipFree(c->ws_pairs);
    if (c->ws_wave) (void)hipFree(c->ws_wave);
    if (c->ws_meta) (void)hipFree(c->ws_meta);
    if (c->ws_kidx) (void)hipFree(c->ws_kidx);
    if (c->ws_event) (void)hipEventDestroy(c->ws_event);
    if (c->small) (void)hipFree(c->small);
    if (c->host) (void)hipHostFree(c->host);
    if (c->mlp_table) (void)hipFree(c->mlp_table);
    for (auto& p : c->pend) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    delete c;
}

const char* rg_last_error(const rg_ctx* c) { return c ? c->err.c_str() : "null context"; }

rg_status rg_profile_enable(rg_ctx* c, int on) {
    if (!c) return RG_EINVAL;
    if (!on) {
        if (rg_status s = drain_profile(c)) return s;
    }
    c->prof = on != 0;
    return RG_OK;
}

rg_status rg_profile_reset(rg_ctx* c) {
    if (!c) return RG_EINVAL;
    if (rg_status s = drain_profile(c)) return s;
    memset(c->prof_ms, 0, sizeof(c->prof_ms));
    memset(c->prof_launches, 0, sizeof(c->prof_launches));
    memset(c->prof_items, 0, sizeof(c->prof_items));
    return RG_OK;
}

rg_status rg_profile_read(rg_ctx* c, int variant, int materialize, double* total_ms, uint64_t* launches,
                          uint64_t* items) {
    if (!c) return RG_EINVAL;
    if (variant < 0 || variant >= NPROF || !total_ms || !launches || !items)
        return fail(c, RG_EINVAL, "bad profile query");
    if (rg_status s = drain_profile(c)) return s;
    const int m = materialize ? 1 : 0;
    *total_ms = c->prof_ms[variant][m];
    *launches = c->prof_launches[variant][m];
    *items = c->prof_items[variant][m];
    return RG_OK;
}

rg_status rg_set_dispatch(rg_ctx* c, int mode, int variant) {
    if (!c) return RG_EINVAL;
    if (mode == RG_DISPATCH_HEURISTIC) {
        c->dispatch_mode = mode;
        return RG_OK;
    }
    if (mode == RG_DISPATCH_MLP) {
        if (!c->mlp_table) return fail(c, RG_EINVAL, "no network installed (rg_dispatch_set_mlp)");
        c->dispatch_mode = mode;
        return RG_OK;
    }
    if (mode == RG_DISPATCH_FIXED && variant >= RG_V_GENERIC && variant <= RG_V_THREAD) {
        c->dispatch_mode = mode;
        c->fixed_bin = variant;
        return RG_OK;
    }
    return fail(c, RG_EINVAL, "unknown dispatch mode or variant");
}

rg_status rg_set_thresholds(rg_ctx* c, uint32_t gallop_ratio, uint32_t thread_max) {
    if (!c) return RG_EINVAL;
    if (gallop_ratio == 0 || thread_max > 4096) return fail(c, RG_EINVAL, "gallop_ratio >= 1, thread_max <= 4096");
    c->gallop_ratio = gallop_ratio;
    c->thread_max = thread_max;
    return RG_OK;
}

rg_status roaring_and(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib, rg_out* out,
                      void* stream) {
    return single(c, RG_AND, A, ia, B, ib, RG_FLAG_MATERIALIZE, out, nullptr, nullptr, stream);
}
rg_status roaring_or(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib, rg_out* out,
                     void* stream) {
    return single(c, RG_OR, A, ia, B, ib, RG_FLAG_MATERIALIZE, out, nullptr, nullptr, stream);
}
rg_status roaring_xor(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib, rg_out* out,
                      void* stream) {
    return single(c, RG_XOR, A, ia, B, ib, RG_FLAG_MATERIALIZE, out, nullptr, nullptr, stream);
}
rg_status roaring_andnot(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib, rg_out* out,
                         void* stream) {
    return single(c, RG_ANDNOT, A, ia, B, ib, RG_FLAG_MATERIALIZE, out, nullptr, nullptr, stream);
}
rg_status roaring_and_cardinality(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib,
                                  uint64_t* d_card, void* stream) {
    return single(c, RG_AND, A, ia, B, ib, RG_FLAG_CARD, nullptr, d_card, nullptr, stream);
}
rg_status roaring_or_cardinality(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib,
                                 uint64_t* d_card, void* stream) {
    return single(c, RG_OR, A, ia, B, ib, RG_FLAG_CARD, nullptr, d_card, nullptr, stream);
}
rg_status roaring_xor_cardinality(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib,
                                  uint64_t* d_card, void* stream) {
    return single(c, RG_XOR, A, ia, B, ib, RG_FLAG_CARD, nullptr, d_card, nullptr, stream);
}
rg_status roaring_andnot_cardinality(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib,
                                     uint64_t* d_card, void* stream) {
    return single(c, RG_ANDNOT, A, ia, B, ib, RG_FLAG_CARD, nullptr, d_card, nullptr, stream);
}
rg_status roaring_jaccard(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib, double* d_j,
                          void* stream) {
    return single(c, RG_AND, A, ia, B, ib, RG_FLAG_JACCARD, nullptr, nullptr, d_j, stream);
}
rg_status roaring_jaccard_host(rg_ctx* c, const rg_pool* A, uint32_t ia, const rg_pool* B, uint32_t ib, double* h_j,
                               void* stream) {
    if (!c) return RG_EINVAL;
    if (!h_j) return fail(c, RG_EINVAL, "roaring_jaccard_host: null result pointer");
    // the device result goes to the context's 4 KiB block (a word no call uses)
    double* d_j = reinterpret_cast<double*>(reinterpret_cast<uint8_t*>(c->small) + 3840);
    if (rg_status s = single(c, RG_AND, A, ia, B, ib, RG_FLAG_JACCARD, nullptr, nullptr, d_j, stream)) return s;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, hipMemcpyAsync(c->host, d_j, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    memcpy(h_j, c->host, 8);
    return RG_OK;
}

rg_status roaring_batch(rg_ctx* c, int op, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia,
                        const uint32_t* d_ib, uint64_t n_pairs, uint32_t flags, rg_out* out, uint64_t* d_cards,
                        double* d_jacc, void* stream) {
    if (!c) return RG_EINVAL;
    if (n_pairs && (!d_ia || !d_ib)) return fail(c, RG_EINVAL, "null pair arrays");
    return run_batch(c, op, A, B, d_ia, d_ib, 0, 0, n_pairs, flags, out, d_cards, d_jacc, (hipStream_t)stream);
}

rg_status roaring_batch_static(rg_ctx* c, int op, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia,
                               const uint32_t* d_ib, uint64_t n_pairs, uint32_t flags, uint64_t* d_cards,
                               double* d_jacc, void* stream) {
    if (!c) return RG_EINVAL;
    if (op < RG_AND || op > RG_ANDNOT) return fail(c, RG_EINVAL, "op must be RG_AND..RG_ANDNOT");
    if (flags & RG_FLAG_MATERIALIZE)
        return fail(c, RG_ENOTSUP, "roaring_batch_static is count-only (RG_FLAG_CARD / RG_FLAG_JACCARD)");
    if (!(flags & (RG_FLAG_CARD | RG_FLAG_JACCARD))) return fail(c, RG_EINVAL, "flags select no output");
    if ((flags & RG_FLAG_CARD) && !d_cards) return fail(c, RG_EINVAL, "RG_FLAG_CARD needs d_cards");
    if ((flags & RG_FLAG_JACCARD) && !d_jacc) return fail(c, RG_EINVAL, "RG_FLAG_JACCARD needs d_jacc");
    if (!pool_ok(A) || !pool_ok(B)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    if (n_pairs > RG_STATIC_MAX_PAIRS)
        return fail(c, RG_ECAPACITY,
                    "roaring_batch_static takes at most RG_STATIC_MAX_PAIRS (" + std::to_string(RG_STATIC_MAX_PAIRS) +
                        ") pairs per call");
    if (n_pairs && (!d_ia || !d_ib)) return fail(c, RG_EINVAL, "null pair arrays");
    if (!c->static_ws) return fail(c, RG_EDEVICE, "static scratch unavailable on this device");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    // ordered after the context's previous call (the asynchronous error word
    // is shared); calls from other contexts on this GPU are not ordered
    WorkspaceOrder order(c, st);
    if (n_pairs == 0) return RG_OK;
    return run_count_async(c, op, A, B, d_ia, d_ib, 0, 0, n_pairs, flags, d_cards, d_jacc, st, c->static_ws,
                           RG_STATIC_SCRATCH_BYTES);
}

rg_status rg_pool_recount(rg_ctx* c, const rg_pool* p, void* stream) {
    if (!c) return RG_EINVAL;
    if (!p || !p->bm_begin || !p->bm_card || !p->bm_wbytes) return fail(c, RG_EINVAL, "incomplete pool");
    HIPCHK(c, hipSetDevice(c->device));
    launch_pool_recount(*p, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_pool_init_dense(rg_ctx* c, const rg_pool* p, uint32_t n_keys, void* stream) {
    if (!c) return RG_EINVAL;
    if (!p || n_keys < 1 || n_keys > 65536) return fail(c, RG_EINVAL, "rg_pool_init_dense: 1 <= n_keys <= 65536");
    if (!pool_ok(p) || p->n_containers != (uint64_t)p->n_bitmaps * n_keys ||
        p->payload_bytes < p->n_containers * 8192ull)
        return fail(c, RG_EINVAL, "rg_pool_init_dense: pool arrays, n_containers or payload do not match");
    HIPCHK(c, hipSetDevice(c->device));
    launch_pool_dense_init(*p, n_keys, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_pool_pack_meta(rg_ctx* c, const rg_pool* p, uint32_t* d_meta, void* stream) {
    if (!c) return RG_EINVAL;
    if (!pool_ok(p) || (!d_meta && p->n_containers)) return fail(c, RG_EINVAL, "incomplete pool or no d_meta");
    if (reinterpret_cast<uintptr_t>(d_meta) & 15) return fail(c, RG_EINVAL, "d_meta must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    launch_pack_meta(view(*p), p->n_containers, reinterpret_cast<u32x4*>(d_meta), (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_pool_key_index(rg_ctx* c, const rg_pool* p, uint8_t* d_index, void* stream) {
    if (!c) return RG_EINVAL;
    if (!pool_ok(p) || (!d_index && p->n_bitmaps)) return fail(c, RG_EINVAL, "incomplete pool or no d_index");
    if (reinterpret_cast<uintptr_t>(d_index) & 15) return fail(c, RG_EINVAL, "d_index must be 16-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    launch_key_index(view(*p), p->n_bitmaps, d_index, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_pool_validate(rg_ctx* c, const rg_pool* p, uint64_t* n_bad, void* stream) {
    return rg_pool_check(c, p, RG_RULES_P1, n_bad, stream);
}

rg_status rg_pool_canonicalize(rg_ctx* c, const rg_pool* in, rg_out* out, void* stream) {
    if (!c) return RG_EINVAL;
    if (!pool_ok(in)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    // pair p = (bitmap p, bitmap p); each result is the union of bitmap p alone
    return run_batch(c, RG_ANDNOT, in, in, nullptr, nullptr, NONE, NONE, in->n_bitmaps, RG_FLAG_MATERIALIZE, out,
                     nullptr, nullptr, (hipStream_t)stream, /*single=*/true);
}

rg_status rg_pool_check(rg_ctx* c, const rg_pool* p, uint32_t rules, uint64_t* n_bad, void* stream) {
    if (!c) return RG_EINVAL;
    if (!pool_ok(p) || !n_bad) return fail(c, RG_EINVAL, "incomplete pool");
    if (rules & ~(uint32_t)RG_RULES_P1) return fail(c, RG_EINVAL, "rg_pool_check: unknown rules");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    WorkspaceOrder order(c, st);  // the context's device block and staging are shared with other calls
    uint64_t* d_bad = reinterpret_cast<uint64_t*>((uint8_t*)c->small + 2048);
    launch_pool_validate(*p, d_bad, (rules & RG_RULES_P1) != 0, st);
    HIPCHK(c, hipMemcpyAsync(c->host, d_bad, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    *n_bad = *reinterpret_cast<uint64_t*>(c->host);
    return RG_OK;
}

rg_status rg_pool_digest(rg_ctx* c, const rg_pool* p, uint64_t* d_digest, void* stream) {
    if (!c) return RG_EINVAL;
    if (!pool_ok(p) || !d_digest) return fail(c, RG_EINVAL, "incomplete pool");
    HIPCHK(c, hipSetDevice(c->device));
    launch_pool_digest(*p, d_digest, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

}  // extern "C"

// ===========================================================================
// Batched count-only plans: fixed pairs, pools and outputs; sync-free execution
// (graph-capturable); persistent work-stealing kernel; autotuned grid and
// galloping ratio.
// ===========================================================================

struct rg_plan {
    rg_ctx* ctx = nullptr;
    int op = RG_AND;
    uint32_t flags = 0;
    rg_pool A{}, B{};
    const uint32_t* d_ia = nullptr;
    const uint32_t* d_ib = nullptr;
    uint64_t n_pairs = 0;
    uint64_t* d_cards = nullptr;
    double* d_jacc = nullptr;
    struct Wave {
        uint64_t p0;
        uint32_t np;
        uint64_t C;
        uint64_t* cand_off;
    };
    std::vector<Wave> waves;
    void* mem = nullptr;
    uint32_t* n_cand = nullptr;
    long long* acc = nullptr;
    uint32_t* err = nullptr;
    uint64_t* cand_all = nullptr;  // count plans: candidate offsets of all pairs (scanned on the device)
    uint32_t* next = nullptr;      // count plans: the fused kernel's block counter
    Task* tasks = nullptr;
    uint32_t* res_card = nullptr;
    uint64_t S_max = 0;
    uint32_t grid = 0;
    int dispatch_mode = RG_DISPATCH_HEURISTIC;
    int fixed_bin = BIN_GEN;
    uint32_t gallop_ratio = 64;
    uint32_t thread_max = 8;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // packed container metadata of both pools (null: not packed)
    void* meta_mem = nullptr;
    const u32x4* metaA = nullptr;
    const u32x4* metaB = nullptr;
    // key-presence indexes (the pools' own, or built at creation; null: none)
    void* kidx_mem = nullptr;
    const uint8_t* kidxA = nullptr;
    const uint8_t* kidxB = nullptr;
    // materialising plans: results into `out` through the k-way kernels (two
    // bitmaps per query), with the arena offsets carried from wave to wave on
    // the device (totals[0] payload end, totals[1] containers written)
    bool mat = false;
    rg_out out{};
    uint64_t* totals = nullptr;
    uint32_t* ub = nullptr;
    uint64_t* slot_off = nullptr;
    uint8_t* res_type = nullptr;
    uint32_t* res_size = nullptr;
    uint64_t* out_idx = nullptr;
    uint64_t* partials = nullptr;
    KwQuery* kw_queries = nullptr;
    uint32_t* kw_ids = nullptr;
};

namespace {

void plan_enqueue_mat(rg_plan* p, hipStream_t st);

void plan_enqueue(rg_plan* p, hipStream_t st) {
    if (p->mat) return plan_enqueue_mat(p, st);
    PoolView pa = view(p->A), pb = view(p->B);
    pa.meta = p->metaA;  // the plan's records (its own, or the pools' when they carry them)
    pb.meta = p->metaB;
    pa.kidx = p->kidxA;
    pb.kidx = p->kidxB;
    launch_fill_u32(p->err, 0, 1, st);
    // the plan accumulates |A n B| for every operation; the requested count
    // follows from the Section 5.9 identities in the last step
    launch_pair_prep(RG_AND, false, pa, pb, p->A.n_bitmaps, p->B.n_bitmaps, p->d_ia, p->d_ib, 0, 0, p->n_pairs,
                     p->n_cand, nullptr, nullptr, p->acc, p->err, st, p->next);
    launch_scan_u32_u64(p->n_cand, p->cand_all, p->n_pairs, 0, p->partials, p->cand_all + p->n_pairs, st);
    MatchArgs m{};
    m.op = RG_AND;
    m.materialize = false;
    m.A = pa;
    m.B = pb;
    m.ia = p->d_ia;
    m.ib = p->d_ib;
    m.pair0 = 0;
    m.n_pairs = (uint32_t)p->n_pairs;
    m.cand_off = p->cand_all;
    m.n_cand = 0;  // read on the device
    m.dispatch_mode = p->dispatch_mode;
    m.fixed_bin = p->fixed_bin;
    m.gallop_ratio = p->gallop_ratio;
    m.thread_max = p->thread_max;
    m.mlp_table = p->ctx->mlp_table;
    m.fuse_thread = true;
    m.acc = p->acc;
    launch_count_fused(m, p->next, p->grid, st);
    launch_finish_counts(RG_AND, p->op, p->acc, pa, pb, p->A.n_bitmaps, p->B.n_bitmaps, p->d_ia, p->d_ib, 0, 0, 0,
                         (uint32_t)p->n_pairs, (p->flags & RG_FLAG_CARD) ? p->d_cards : nullptr,
                         (p->flags & RG_FLAG_JACCARD) ? p->d_jacc : nullptr, st);
}

// Materialising plan: every wave through the k-way kernels, no host readback.
void plan_enqueue_mat(rg_plan* p, hipStream_t st) {
    const rg_out& o = p->out;
    PoolView pa = view(p->A), pb = view(p->B);
    launch_fill_u32(p->err, 0, 1, st);
    launch_fill_u64(p->totals, 0, 2, st);
    launch_fill_u64(o.bm_card, 0, p->n_pairs, st);
    if (o.bm_wbytes) launch_fill_u64(o.bm_wbytes, 0, p->n_pairs, st);
    const size_t nw = p->waves.size();
    for (size_t w = 0; w < nw; ++w) {
        const auto& wv = p->waves[w];
        const bool last = w + 1 == nw;
        if (!wv.C) {
            launch_bm_begin(wv.cand_off, p->out_idx, 0, p->totals + 1, wv.np, wv.p0, o.bm_begin, last, st);
            continue;
        }
        launch_kw_pair_queries(p->op, p->d_ia, p->d_ib, 0, 0, wv.p0, wv.np, wv.cand_off, p->kw_queries, p->kw_ids,
                               st);
        KwArgs ka;
        ka.P0 = pa;
        ka.P1 = pb;
        ka.pair_base = (uint32_t)wv.p0;
        ka.queries = p->kw_queries;
        ka.n_queries = wv.np;
        ka.ids = p->kw_ids;
        ka.tasks = p->tasks;
        ka.n_slots = wv.C;
        ka.ub = p->ub;
        ka.res_card = p->res_card;
        ka.so = SlotOut{p->slot_off, o.payload, p->res_card, p->res_type, p->res_size};
        ka.so.cap = o.cap_payload_bytes;
        ka.so.err = p->err;
        ka.acc = nullptr;
        ka.err = p->err;
        ka.small = !(p->ctx->dispatch_mode == 2 && p->ctx->fixed_bin == BIN_GEN);
        launch_kw_keys(ka, st);
        launch_kw_bounds(ka, st, true);  // pairwise queries only
        // slot payload offsets continue from the previous wave's payload end
        launch_scan_u32_u64(p->ub, p->slot_off, wv.C, 0, p->partials, p->totals, st, p->totals);
        launch_kw_small(ka, st);
        launch_kw_bb(ka, st);
        launch_kw_eval(ka, st);
        // output indices continue from the previous wave's container count
        launch_scan_nonzero_u64(p->res_card, p->out_idx, wv.C, 0, p->partials, p->totals + 1, st, p->totals + 1);
        CompactArgs cp;
        cp.tasks = p->tasks;
        cp.n_slots = wv.C;
        cp.res_card = p->res_card;
        cp.res_type = p->res_type;
        cp.res_size = p->res_size;
        cp.slot_off = p->slot_off;
        cp.out_idx = p->out_idx;
        cp.keys = o.keys;
        cp.types = o.types;
        cp.card = o.card;
        cp.size = o.size;
        cp.off = o.off;
        cp.bm_card = o.bm_card;
        cp.bm_wbytes = o.bm_wbytes;
        cp.pair0 = wv.p0;
        launch_compact(cp, st);
        launch_bm_begin(wv.cand_off, p->out_idx, wv.C, p->totals + 1, wv.np, wv.p0, o.bm_begin, last, st);
    }
    if (p->flags & (RG_FLAG_CARD | RG_FLAG_JACCARD))
        launch_mat_counts(p->op, o.bm_card, pa, pb, p->d_ia, p->d_ib, 0, 0, p->n_pairs,
                          (p->flags & RG_FLAG_CARD) ? p->d_cards : nullptr,
                          (p->flags & RG_FLAG_JACCARD) ? p->d_jacc : nullptr, st);
}

void plan_drop_graph(rg_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

}  // namespace

extern "C" {

rg_status rg_plan_create(rg_ctx* c, int op, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia,
                         const uint32_t* d_ib, uint64_t n_pairs, uint32_t flags, uint64_t* d_cards, double* d_jacc,
                         rg_plan** out_plan, void* stream) {
    if (!c) return RG_EINVAL;
    if (!out_plan) return fail(c, RG_EINVAL, "null plan pointer");
    *out_plan = nullptr;
    if (op < RG_AND || op > RG_ANDNOT) return fail(c, RG_EINVAL, "op must be RG_AND..RG_ANDNOT");
    if (!pool_ok(A) || !pool_ok(B)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    if (flags & RG_FLAG_MATERIALIZE) return fail(c, RG_ENOTSUP, "plans are count-only (RG_FLAG_CARD/JACCARD)");
    if (!(flags & (RG_FLAG_CARD | RG_FLAG_JACCARD))) return fail(c, RG_EINVAL, "flags select no output");
    if ((flags & RG_FLAG_CARD) && !d_cards) return fail(c, RG_EINVAL, "RG_FLAG_CARD needs d_cards");
    if ((flags & RG_FLAG_JACCARD) && !d_jacc) return fail(c, RG_EINVAL, "RG_FLAG_JACCARD needs d_jacc");
    if (n_pairs == 0 || n_pairs > 0xFFFFFFFFull || !d_ia || !d_ib)
        return fail(c, RG_EINVAL, "a plan needs 1..2^32-1 pairs and device pair arrays");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    rg_plan* p = new rg_plan();
    p->ctx = c;
    p->op = op;
    p->flags = flags;
    p->A = *A;
    p->B = *B;
    p->d_ia = d_ia;
    p->d_ib = d_ib;
    p->n_pairs = n_pairs;
    p->d_cards = d_cards;
    p->d_jacc = d_jacc;
    p->dispatch_mode = c->dispatch_mode;
    p->fixed_bin = c->fixed_bin;
    p->gallop_ratio = c->gallop_ratio;
    p->thread_max = c->thread_max;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    p->grid = (uint32_t)cus * count_fused_blocks_per_cu();

    // candidate counts: one preparation pass, read back once
    auto cleanup = [&](rg_status s) {
        if (p->mem) (void)hipFree(p->mem);
        if (p->meta_mem) (void)hipFree(p->meta_mem);
        if (p->kidx_mem) (void)hipFree(p->kidx_mem);
        delete p;
        return s;
    };
    const size_t pair_bytes = align256(4 * n_pairs) + align256(8 * n_pairs) + align256(4 * n_pairs) +
                              align256(8 * n_pairs) + 256;
    std::vector<uint32_t> h_cand(n_pairs);
    {
        void* tmp = nullptr;
        if (hipMalloc(&tmp, pair_bytes) != hipSuccess) return cleanup(fail(c, RG_EDEVICE, "hipMalloc failed"));
        Bump b{(uint8_t*)tmp};
        uint32_t* nc = b.take<uint32_t>(n_pairs);
        uint64_t* bd = b.take<uint64_t>(n_pairs);
        uint32_t* mc = b.take<uint32_t>(n_pairs);
        long long* ac = b.take<long long>(n_pairs);
        uint32_t* er = b.take<uint32_t>(1);
        launch_fill_u32(er, 0, 1, st);
        launch_pair_prep(RG_AND, false, view(*A), view(*B), A->n_bitmaps, B->n_bitmaps, d_ia, d_ib, 0, 0, n_pairs,
                         nc, bd, mc, ac, er, st);
        uint32_t h_err = 0;
        hipError_t e1 = hipMemcpyAsync(h_cand.data(), nc, 4 * n_pairs, hipMemcpyDeviceToHost, st);
        hipError_t e2 = hipMemcpyAsync(&h_err, er, 4, hipMemcpyDeviceToHost, st);
        hipError_t e3 = hipStreamSynchronize(st);
        (void)hipFree(tmp);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
            return cleanup(fail(c, RG_EDEVICE, "plan preparation failed"));
        if (h_err) return cleanup(fail(c, RG_EINVAL, "pair index out of range of its pool"));
    }
    // One launch of the fused match-and-count kernel takes every pair: the
    // candidate offsets are scanned on the device at each execution, so the
    // plan keeps only per-pair arrays.
    uint64_t slots = 0;
    for (uint64_t q = 0; q < n_pairs; ++q) slots += h_cand[q];
    const size_t total = align256(4 * n_pairs) + align256(8 * n_pairs) + align256(8 * (n_pairs + 1)) +
                         align256(8 * scan_partials_needed(n_pairs)) + 2 * 256;
    if (hipMalloc(&p->mem, total) != hipSuccess) return cleanup(fail(c, RG_EDEVICE, "hipMalloc failed"));
    Bump b{(uint8_t*)p->mem};
    p->n_cand = b.take<uint32_t>(n_pairs);
    p->acc = b.take<long long>(n_pairs);
    p->cand_all = b.take<uint64_t>(n_pairs + 1);
    p->partials = b.take<uint64_t>(scan_partials_needed(n_pairs));
    p->err = b.take<uint32_t>(1);
    p->next = b.take<uint32_t>(1);
    p->waves.push_back(rg_plan::Wave{0, (uint32_t)n_pairs, slots, p->cand_all});
    // Key matching reads every matched container's type, cardinality, size and
    // offset; the plan packs them into one 16-byte record per container once
    // (both pools, or one when A and B are the same pool). Without the memory
    // the plan runs from the separate arrays.
    if (A->meta && B->meta) {
        // the caller packed them (rg_pool_pack_meta): use those
        p->metaA = reinterpret_cast<const u32x4*>(A->meta);
        p->metaB = reinterpret_cast<const u32x4*>(B->meta);
    } else {
        const bool same = A->keys == B->keys && A->off == B->off && A->n_containers == B->n_containers;
        const uint64_t nA = A->n_containers, nB = same ? 0 : B->n_containers;
        if (nA + nB) {
            if (hipMalloc(&p->meta_mem, 16 * (nA + nB)) == hipSuccess) {
                u32x4* ma = reinterpret_cast<u32x4*>(p->meta_mem);
                u32x4* mb = same ? ma : ma + nA;
                launch_pack_meta(view(*A), nA, ma, st);
                if (!same) launch_pack_meta(view(*B), nB, mb, st);
                // complete before the plan runs on any stream
                if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
                    return cleanup(fail(c, RG_EDEVICE, "plan metadata packing failed"));
                p->metaA = ma;
                p->metaB = mb;
            } else {
                p->meta_mem = nullptr;
                (void)hipGetLastError();  // the failed allocation is not an error of the plan
            }
        }
    }
    // key-presence indexes of pools with many keys per bitmap
    p->kidxA = A->key_index;
    p->kidxB = B->key_index;
    {
        const bool same = A->keys == B->keys && A->bm_begin == B->bm_begin;
        const uint64_t nA = kidx_pays(A, n_pairs) ? A->n_bitmaps : 0, nB = (!same && kidx_pays(B, n_pairs)) ? B->n_bitmaps : 0;
        if (nA + nB) {
            if (hipMalloc(&p->kidx_mem, (size_t)RG_KEY_INDEX_BYTES * (nA + nB)) == hipSuccess) {
                uint8_t* kb = static_cast<uint8_t*>(p->kidx_mem);
                if (nA) {
                    launch_key_index(view(*A), A->n_bitmaps, kb, st);
                    p->kidxA = kb;
                    if (same) p->kidxB = kb;
                }
                if (nB) {
                    launch_key_index(view(*B), B->n_bitmaps, kb + (size_t)RG_KEY_INDEX_BYTES * nA, st);
                    p->kidxB = kb + (size_t)RG_KEY_INDEX_BYTES * nA;
                }
                if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
                    return cleanup(fail(c, RG_EDEVICE, "plan key indexing failed"));
            } else {
                p->kidx_mem = nullptr;
                (void)hipGetLastError();
            }
        }
    }
    *out_plan = p;
    return RG_OK;
}

rg_status rg_plan_create_mat(rg_ctx* c, int op, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia,
                             const uint32_t* d_ib, uint64_t n_pairs, uint32_t flags, rg_out* out, uint64_t* d_cards,
                             double* d_jacc, rg_plan** out_plan, void* stream) {
    if (!c) return RG_EINVAL;
    if (!out_plan) return fail(c, RG_EINVAL, "null plan pointer");
    *out_plan = nullptr;
    if (op < RG_AND || op > RG_ANDNOT) return fail(c, RG_EINVAL, "op must be RG_AND..RG_ANDNOT");
    if (!pool_ok(A) || !pool_ok(B)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    if (!(flags & RG_FLAG_MATERIALIZE)) return fail(c, RG_EINVAL, "rg_plan_create_mat needs RG_FLAG_MATERIALIZE");
    if ((flags & RG_FLAG_CARD) && !d_cards) return fail(c, RG_EINVAL, "RG_FLAG_CARD needs d_cards");
    if ((flags & RG_FLAG_JACCARD) && !d_jacc) return fail(c, RG_EINVAL, "RG_FLAG_JACCARD needs d_jacc");
    if (!out || !out->bm_begin || !out->keys || !out->types || !out->card || !out->size || !out->off ||
        !out->payload || !out->bm_card)
        return fail(c, RG_EINVAL, "materialisation needs a complete rg_out");
    if (n_pairs == 0 || n_pairs > 0xFFFFFFFFull || !d_ia || !d_ib)
        return fail(c, RG_EINVAL, "a plan needs 1..2^32-1 pairs and device pair arrays");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    out->needed_containers = out->needed_payload_bytes = out->n_containers = out->payload_used = 0;
    // per pair: result slots, payload bound and container bound, read back once
    std::vector<uint32_t> h_cand(n_pairs), h_minc(n_pairs);
    std::vector<uint64_t> h_bound(n_pairs);
    {
        const size_t pb = align256(4 * n_pairs) + align256(8 * n_pairs) + align256(4 * n_pairs) +
                          align256(8 * n_pairs) + 256;
        void* tmp = nullptr;
        if (hipMalloc(&tmp, pb) != hipSuccess) return fail(c, RG_EDEVICE, "hipMalloc failed");
        Bump b{(uint8_t*)tmp};
        uint32_t* nc = b.take<uint32_t>(n_pairs);
        uint64_t* bd = b.take<uint64_t>(n_pairs);
        uint32_t* mc = b.take<uint32_t>(n_pairs);
        long long* ac = b.take<long long>(n_pairs);
        uint32_t* er = b.take<uint32_t>(1);
        launch_fill_u32(er, 0, 1, st);
        launch_pair_prep(op, true, view(*A), view(*B), A->n_bitmaps, B->n_bitmaps, d_ia, d_ib, 0, 0, n_pairs, nc, bd,
                         mc, ac, er, st);
        uint32_t h_err = 0;
        hipError_t e1 = hipMemcpyAsync(h_cand.data(), nc, 4 * n_pairs, hipMemcpyDeviceToHost, st);
        hipError_t e2 = hipMemcpyAsync(h_bound.data(), bd, 8 * n_pairs, hipMemcpyDeviceToHost, st);
        hipError_t e3 = hipMemcpyAsync(h_minc.data(), mc, 4 * n_pairs, hipMemcpyDeviceToHost, st);
        hipError_t e4 = hipMemcpyAsync(&h_err, er, 4, hipMemcpyDeviceToHost, st);
        hipError_t e5 = hipStreamSynchronize(st);
        (void)hipFree(tmp);
        if (e1 || e2 || e3 || e4 || e5) return fail(c, RG_EDEVICE, "plan preparation failed");
        if (h_err) return fail(c, RG_EINVAL, "pair index out of range of its pool");
    }
    uint64_t tb = 0, tcont = 0;
    for (uint64_t q = 0; q < n_pairs; ++q) {
        tb += h_bound[q];
        tcont += h_minc[q];
    }
    out->needed_payload_bytes = tb;
    out->needed_containers = tcont;
    if (out->cap_payload_bytes < tb || out->cap_containers < tcont)
        return fail(c, RG_ECAPACITY, "output arena too small");
    rg_plan* p = new rg_plan();
    p->ctx = c;
    p->op = op;
    p->flags = flags;
    p->A = *A;
    p->B = *B;
    p->d_ia = d_ia;
    p->d_ib = d_ib;
    p->n_pairs = n_pairs;
    p->d_cards = d_cards;
    p->d_jacc = d_jacc;
    p->mat = true;
    p->out = *out;
    auto cleanup = [&](rg_status s) {
        if (p->mem) (void)hipFree(p->mem);
        delete p;
        return s;
    };
    std::vector<uint64_t> starts{0};
    uint64_t accs = 0, P_max = 0;
    for (uint64_t q = 0; q < n_pairs; ++q) {
        if (accs + h_cand[q] > c->max_wave_slots && accs > 0) {
            p->S_max = std::max(p->S_max, accs);
            P_max = std::max(P_max, q - starts.back());
            starts.push_back(q);
            accs = 0;
        }
        accs += h_cand[q];
    }
    p->S_max = std::max(p->S_max, accs);
    P_max = std::max(P_max, n_pairs - starts.back());
    starts.push_back(n_pairs);
    size_t offs_bytes = 0;
    for (size_t w = 0; w + 1 < starts.size(); ++w) offs_bytes += align256(8 * (starts[w + 1] - starts[w] + 1));
    const uint64_t S = std::max<uint64_t>(p->S_max, 1);
    size_t total = offs_bytes + 2 * 256;  // + err, totals
    for (size_t x : {sizeof(Task) * S, 4 * S, 8 * S, 4 * S, 1 * S, 4 * S, 8 * S, 8 * scan_partials_needed(S),
                     sizeof(KwQuery) * P_max, 8 * P_max})
        total += align256(x);
    if (hipMalloc(&p->mem, total) != hipSuccess) return cleanup(fail(c, RG_EDEVICE, "hipMalloc failed"));
    Bump b{(uint8_t*)p->mem};
    p->err = b.take<uint32_t>(1);
    p->totals = b.take<uint64_t>(2);
    p->tasks = b.take<Task>(S);
    p->ub = b.take<uint32_t>(S);
    p->slot_off = b.take<uint64_t>(S);
    p->res_card = b.take<uint32_t>(S);
    p->res_type = b.take<uint8_t>(S);
    p->res_size = b.take<uint32_t>(S);
    p->out_idx = b.take<uint64_t>(S);
    p->partials = b.take<uint64_t>(scan_partials_needed(S));
    p->kw_queries = b.take<KwQuery>(P_max);
    p->kw_ids = b.take<uint32_t>(2 * P_max);
    std::vector<uint64_t> h_off;
    for (size_t w = 0; w + 1 < starts.size(); ++w) {
        rg_plan::Wave wv;
        wv.p0 = starts[w];
        wv.np = (uint32_t)(starts[w + 1] - starts[w]);
        h_off.assign(wv.np + 1, 0);
        for (uint32_t q = 0; q < wv.np; ++q) h_off[q + 1] = h_off[q] + h_cand[wv.p0 + q];
        wv.C = h_off[wv.np];
        wv.cand_off = b.take<uint64_t>(wv.np + 1);
        if (hipMemcpy(wv.cand_off, h_off.data(), 8 * (wv.np + 1), hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(c, RG_EDEVICE, "plan upload failed"));
        p->waves.push_back(wv);
    }
    *out_plan = p;
    return RG_OK;
}

rg_status rg_plan_result(rg_plan* p, uint64_t* n_containers, uint64_t* payload_used, void* stream) {
    if (!p) return RG_EINVAL;
    rg_ctx* c = p->ctx;
    if (!p->mat) return fail(c, RG_EINVAL, "rg_plan_result: the plan does not materialise");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    uint64_t h[2] = {0, 0};
    uint32_t e = 0;
    HIPCHK(c, hipMemcpyAsync(h, p->totals, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(&e, p->err, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (e & 2u)
        return fail(c, RG_ECAPACITY, "result payload exceeds the arena (pool cardinalities inconsistent with the payload)");
    if (e) return fail(c, RG_EDEVICE, "result key set exceeded its bound (internal error)");
    if (n_containers) *n_containers = h[1];
    if (payload_used) *payload_used = h[0];
    return RG_OK;
}

rg_status rg_plan_totals(const rg_plan* p, const uint64_t** d_totals) {
    if (!p || !d_totals || !p->mat) return RG_EINVAL;
    *d_totals = p->totals;
    return RG_OK;
}

rg_status rg_set_wave_slots(rg_ctx* c, uint64_t max_slots) {
    if (!c) return RG_EINVAL;
    if (max_slots < 1 || max_slots > (1ull << 30)) return fail(c, RG_EINVAL, "rg_set_wave_slots: 1 <= slots <= 2^30");
    c->max_wave_slots = max_slots;
    return RG_OK;
}

rg_status rg_plan_execute(rg_plan* p, void* stream) {
    if (!p) return RG_EINVAL;
    rg_ctx* c = p->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (p->exec) {
        HIPCHK(c, hipGraphLaunch(p->exec, st));
    } else {
        plan_enqueue(p, st);
        HIPCHK(c, hipGetLastError());
    }
    return RG_OK;
}

rg_status rg_plan_capture(rg_plan* p, void* stream) {
    if (!p) return RG_EINVAL;
    rg_ctx* c = p->ctx;
    if (!stream) return fail(c, RG_EINVAL, "graph capture needs a non-default stream");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    plan_drop_graph(p);
    HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    plan_enqueue(p, st);
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamEndCapture(st, &g));
    p->graph = g;
    HIPCHK(c, hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0));
    return RG_OK;
}

rg_status rg_plan_tune(rg_plan* p, void* stream, int reps) {
    if (!p) return RG_EINVAL;
    if (p->mat) return RG_OK;  // the k-way kernels of materialising plans have no knobs to tune
    rg_ctx* c = p->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const bool had_graph = p->exec != nullptr;
    plan_drop_graph(p);
    if (reps < 1) reps = 3;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    auto measure = [&](float* ms_out) -> rg_status {
        plan_enqueue(p, st);  // warm-up
        float tot = 0;
        for (int i = 0; i < reps; ++i) {
            (void)hipEventRecord(e0, st);
            plan_enqueue(p, st);
            (void)hipEventRecord(e1, st);
            HIPCHK(c, hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
            tot += ms;
        }
        *ms_out = tot;
        return RG_OK;
    };
    // coordinate descent: thread-size threshold, then grid, then galloping ratio
    const bool heur = p->dispatch_mode == RG_DISPATCH_HEURISTIC;
    // (no threshold 0: without a thread variant the many one-value arrays of a
    // typical pool become workgroup merges, hundreds of times slower)
    std::vector<uint32_t> tvals = heur ? std::vector<uint32_t>{4, 16, 64} : std::vector<uint32_t>{};
    std::vector<uint32_t> gvals;
    // multiples of the CUs, and the resident grid itself
    for (uint32_t f : {1u, 2u, 4u, 8u, 16u}) gvals.push_back((uint32_t)cus * f);
    if (count_fused_blocks_per_cu() != 4u) gvals.push_back((uint32_t)cus * count_fused_blocks_per_cu());
    std::vector<uint32_t> rvals = heur ? std::vector<uint32_t>{8, 32, 128, 512} : std::vector<uint32_t>{};
    uint32_t* knobs[3] = {&p->thread_max, &p->grid, &p->gallop_ratio};
    const std::vector<uint32_t>* vals[3] = {&tvals, &gvals, &rvals};
    rg_status s = RG_OK;
    for (int k = 0; k < 3 && s == RG_OK; ++k) {
        float best = 1e30f;
        uint32_t bv = *knobs[k];
        for (uint32_t v : *vals[k]) {
            *knobs[k] = v;
            float ms = 0;
            if ((s = measure(&ms)) != RG_OK) break;
            if (ms < best) {
                best = ms;
                bv = v;
            }
        }
        *knobs[k] = bv;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != RG_OK) return s;
    if (had_graph) return rg_plan_capture(p, stream);
    return RG_OK;
}

rg_status rg_plan_info(const rg_plan* p, uint32_t* grid, uint32_t* gallop_ratio, uint32_t* thread_max, uint64_t* slots,
                       uint32_t* waves, int* graph) {
    if (!p) return RG_EINVAL;
    if (grid) *grid = p->grid;
    if (gallop_ratio) *gallop_ratio = p->gallop_ratio;
    if (thread_max) *thread_max = p->thread_max;
    if (slots) {
        uint64_t s = 0;
        for (const auto& w : p->waves) s += w.C;
        *slots = s;
    }
    if (waves) *waves = (uint32_t)p->waves.size();
    if (graph) *graph = p->exec != nullptr;
    return RG_OK;
}

rg_status rg_plan_set(rg_plan* p, uint32_t grid, uint32_t gallop_ratio, uint32_t thread_max) {
    if (!p || grid == 0 || gallop_ratio == 0 || thread_max > 4096) return RG_EINVAL;
    const bool had_graph = p->exec != nullptr;
    plan_drop_graph(p);
    p->grid = grid;
    p->gallop_ratio = gallop_ratio;
    p->thread_max = thread_max;
    return had_graph ? RG_ENOTSUP : RG_OK;  // caller re-captures explicitly
}

void rg_plan_destroy(rg_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    plan_drop_graph(p);
    if (p->mem) (void)hipFree(p->mem);
    if (p->meta_mem) (void)hipFree(p->meta_mem);
    if (p->kidx_mem) (void)hipFree(p->kidx_mem);
    delete p;
}

}  // extern "C"
