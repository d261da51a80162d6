// rg_host.h - host-side internals shared by the C ABI sources: the context,
// error reporting, workspace growth and small helpers.
#pragma once
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "rg_internal.h"

using namespace rg;

struct rg_ctx {
    int device = 0;
    std::string err;
    void* ws_pairs = nullptr;  // per-pair arrays
    size_t ws_pairs_bytes = 0;
    void* ws_wave = nullptr;   // per-slot arrays of one wave
    size_t ws_wave_bytes = 0;
    void* small = nullptr;     // 4 KiB of counters
    void* host = nullptr;      // pinned staging
    size_t host_bytes = 0;
    void* ws_meta = nullptr;   // packed container metadata of a large count-only call
    size_t ws_meta_bytes = 0;
    void* ws_kidx = nullptr;   // key-presence indexes of a count-only call's pools
    size_t ws_kidx_bytes = 0;
    // caller-owned device workspace (rg_set_workspace): when set, calls carve
    // their scratch out of it and never allocate device memory
    void* user_ws = nullptr;
    size_t user_ws_bytes = 0;
    // device address of the library's static scratch on this context's device
    // (roaring_batch_static), found at rg_create
    void* static_ws = nullptr;
    // host buffer for readbacks larger than the pinned staging when calls may
    // not allocate pinned memory (caller workspace set)
    std::vector<uint8_t> host_pageable;
    // completion of the last call that used the workspaces, on its stream: the
    // next call waits for it on its own stream (no host synchronisation)
    hipEvent_t ws_event = nullptr;
    bool ws_event_live = false;
    // kernel timing (rg_profile_*): events around each compute-kernel launch
    struct Pending {
        hipEvent_t a, b;
        int cls;
        int mat;
        uint64_t items;
    };
    bool prof = false;
    bool prof_fused_pending = false;  // timed fused launches have counted into the device block
    std::vector<Pending> pend;
    std::vector<hipEvent_t> evpool;
    double prof_ms[NPROF][2] = {};
    uint64_t prof_launches[NPROF][2] = {};
    uint64_t prof_items[NPROF][2] = {};
    int dispatch_mode = RG_DISPATCH_HEURISTIC;
    int fixed_bin = BIN_GEN;
    uint32_t gallop_ratio = 64;
    uint32_t thread_max = 8;
    uint64_t max_wave_slots = 1ull << 24;
    uint8_t* mlp_table = nullptr;      // learned dispatch table (device, MLP_TABLE bytes)
    // dispatcher training: when cost_out is set, the count kernels record per-slot costs
    float* cost_out = nullptr;
    uint64_t cost_cap = 0;
    uint64_t cost_slots = 0;
    const Task* cost_tasks = nullptr;
};


// Kernel timing (rg_profile_*): an event from the context's pool, or a new one.
inline hipEvent_t take_event(rg_ctx* c) {
    if (!c->evpool.empty()) {
        hipEvent_t e = c->evpool.back();
        c->evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launches `fn` on st; when profiling, brackets it with events on the same stream.
template <class F>
void timed(rg_ctx* c, int cls, bool mat, uint64_t items, hipStream_t st, F&& fn) {
    if (!c->prof) {
        fn();
        return;
    }
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) {
        fn();
        return;
    }
    (void)hipEventRecord(a, st);
    fn();
    (void)hipEventRecord(b, st);
    c->pend.push_back({a, b, cls, mat ? 1 : 0, items});
}

inline rg_status fail(rg_ctx* c, rg_status s, const std::string& m) {
    if (c) c->err = m;
    return s;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(ctx, RG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline rg_status grow_device(rg_ctx* c, void** buf, size_t* cap, size_t need) {
    if (need <= *cap) return RG_OK;
    const size_t old = *cap;
    if (*buf) {
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipFree(*buf));
        *buf = nullptr;
        *cap = 0;
    }
    size_t nb = std::max(need, old + old / 2);
    nb = (nb + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1);
    HIPCHK(c, hipMalloc(buf, nb));
    *cap = nb;
    return RG_OK;
}

// Orders a call that uses the context's workspaces after the previous such
// call, whatever streams they are on: waits (on the device) for the previous
// call's completion event, and records its own when it goes out of scope.
struct WorkspaceOrder {
    rg_ctx* c;
    hipStream_t st;
    WorkspaceOrder(rg_ctx* c_, hipStream_t st_) : c(c_), st(st_) {
        if (c->ws_event_live) (void)hipStreamWaitEvent(st, c->ws_event, 0);
    }
    ~WorkspaceOrder() {
        if (!c->ws_event && hipEventCreateWithFlags(&c->ws_event, hipEventDisableTiming) != hipSuccess) {
            c->ws_event = nullptr;
            return;
        }
        c->ws_event_live = hipEventRecord(c->ws_event, st) == hipSuccess;
    }
};

// The context's 4 KiB device block (c->small): bytes 0..767 the counters of
// one materialising call (error word, bin counts and offsets, totals), 2048
// rg_pool_validate's count, 3584 roaring_to_uint32's range (3 x u64), 3840
// roaring_jaccard_host's result, 3616 the fused count kernel's matched
// container pairs while timing is on, u32 word 1020 the asynchronous error flag.
constexpr size_t SMALL_ASYNC_ERR = 1020;  // u32: sticky flag of asynchronous calls, cleared by rg_sync
constexpr size_t SMALL_EXPORT_RANGE = 3584;  // bytes
constexpr size_t SMALL_FUSED_MATCHED = 3616;  // bytes

inline unsigned long long* fused_matched_word(rg_ctx* c) {
    return reinterpret_cast<unsigned long long*>(static_cast<uint8_t*>(c->small) + SMALL_FUSED_MATCHED);
}

inline uint32_t* async_err_word(rg_ctx* c) { return reinterpret_cast<uint32_t*>(c->small) + SMALL_ASYNC_ERR; }

// Pinned host staging allocated with the context; larger readbacks grow it
// (or, with a caller workspace, use pageable memory instead).
constexpr size_t HOST_STAGING_BYTES = 1u << 20;

// Device scratch of one call, in regions taken one after another. With a
// fixed region (the caller's workspace, or the library's static scratch for
// roaring_batch_static) the regions are carved from it in order and a region
// that does not fit fails with RG_ECAPACITY (nothing is allocated); otherwise
// each region is one of the context's own buffers, grown on demand.
enum WsRegion { WS_PAIRS = 0, WS_WAVE = 1, WS_META = 2, WS_KIDX = 3 };
struct Scratch {
    rg_ctx* c;
    uint8_t* fixed = nullptr;
    size_t fixed_bytes = 0;
    size_t used = 0;
    explicit Scratch(rg_ctx* c_) : c(c_) {
        if (c->user_ws) {
            fixed = static_cast<uint8_t*>(c->user_ws);
            fixed_bytes = c->user_ws_bytes;
        }
    }
    Scratch(rg_ctx* c_, void* base, size_t bytes) : c(c_), fixed(static_cast<uint8_t*>(base)), fixed_bytes(bytes) {}
    bool caller() const { return fixed != nullptr; }
    // bytes still free in a fixed region (unbounded for the context's own)
    size_t left() const { return caller() ? fixed_bytes - used : ~(size_t)0; }
    rg_status take(WsRegion r, size_t need, void** out);
};

inline rg_status grow_host(rg_ctx* c, size_t need) {
    if (need <= c->host_bytes) return RG_OK;
    if (c->host) {
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipHostFree(c->host));
        c->host = nullptr;
        c->host_bytes = 0;
    }
    size_t nb = std::max(need, (size_t)1 << 20);
    HIPCHK(c, hipHostMalloc(&c->host, nb, hipHostMallocDefault));
    c->host_bytes = nb;
    return RG_OK;
}

inline rg_status Scratch::take(WsRegion r, size_t need, void** out) {
    need = align256(need ? need : 1);
    if (caller()) {
        if (need > left())
            return fail(c, RG_ECAPACITY,
                        "workspace too small: the call needs at least " + std::to_string(used + need) + " bytes of " +
                            std::to_string(fixed_bytes));
        *out = fixed + used;
        used += need;
        return RG_OK;
    }
    void** buf = r == WS_PAIRS ? &c->ws_pairs : r == WS_WAVE ? &c->ws_wave : r == WS_META ? &c->ws_meta : &c->ws_kidx;
    size_t* cap = r == WS_PAIRS  ? &c->ws_pairs_bytes
                  : r == WS_WAVE ? &c->ws_wave_bytes
                  : r == WS_META ? &c->ws_meta_bytes
                                 : &c->ws_kidx_bytes;
    if (rg_status s = grow_device(c, buf, cap, need)) return s;
    *out = *buf;
    return RG_OK;
}

// Host memory for a readback of `need` bytes: the pinned staging when it is
// large enough; beyond it, grown pinned memory, or pageable memory when the
// call may not allocate through HIP (caller workspace).
inline rg_status host_buffer(rg_ctx* c, size_t need, uint8_t** out) {
    if (need <= c->host_bytes) {
        *out = static_cast<uint8_t*>(c->host);
        return RG_OK;
    }
    if (c->user_ws) {
        if (c->host_pageable.size() < need) c->host_pageable.resize(need);
        *out = c->host_pageable.data();
        return RG_OK;
    }
    if (rg_status s = grow_host(c, need)) return s;
    *out = static_cast<uint8_t*>(c->host);
    return RG_OK;
}

struct Bump {
    uint8_t* base;
    size_t used = 0;
    template <class T>
    T* take(size_t n) {
        T* p = reinterpret_cast<T*>(base + used);
        used += align256(n * sizeof(T));
        return p;
    }
};

inline PoolView view(const rg_pool& p) {
    return PoolView{p.bm_begin, p.keys,    p.types,     p.card,      p.size,
                    p.off,      p.payload, p.bm_card,   p.bm_wbytes, reinterpret_cast<const u32x4*>(p.meta),
                    p.key_index};
}

inline bool pool_ok(const rg_pool* p) {
    return p && p->bm_begin && p->bm_card && p->bm_wbytes && (p->n_containers == 0 ||
           (p->keys && p->types && p->card && p->size && p->off && p->payload)) &&
           p->n_containers < 0xFFFFFFFFull;
}

// One batched call (rg_api.cpp): pair preparation, key matching in waves,
// binned kernels, output assembly or count finishing. single: see
// rg_pool_canonicalize.
rg_status run_batch(rg_ctx* c, int op, const rg_pool* A, const rg_pool* B, const uint32_t* d_ia,
                    const uint32_t* d_ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs, uint32_t flags, rg_out* out,
                    uint64_t* d_cards, double* d_jacc, hipStream_t st, bool single = false);

// Whether a pool is worth a key-presence index for count-only matching over
// n_pairs pairs: it has none, its bitmaps hold at least KIDX_MIN_MEAN_KEYS keys
// on average, and the call is expected to look up more candidate keys (pairs x
// the mean key count) than building the index reads keys (all of the pool's)
// and writes index words (1024 per bitmap).
inline bool kidx_pays(const rg_pool* P, uint64_t n_pairs) {
    if (P->key_index || !P->n_bitmaps) return false;
    const uint64_t mean = P->n_containers / P->n_bitmaps;
    if (mean < KIDX_MIN_MEAN_KEYS) return false;
    const double cand = (double)n_pairs * (double)mean;
    return cand >= (double)P->n_containers + (double)KIDX_WORDS * (double)P->n_bitmaps;
}
