// rg_mutable_api.cpp - C ABI of mutable pools: in-place A op= B with the
// bitmaps' cardinalities maintained, over a device slot allocator.
#include <algorithm>
#include <vector>

#include "rg_host.h"
#include "rg_mutable.h"

struct rg_mpool {
    rg_ctx* ctx = nullptr;
    MutView v{};
    void* mem = nullptr;   // everything but the slab
    void* slab = nullptr;
};

namespace {

rg_status check_args(rg_mpool* mp, uint32_t b, const rg_pool* P, uint32_t src) {
    rg_ctx* c = mp->ctx;
    if (b >= mp->v.n_bitmaps) return fail(c, RG_EINVAL, "mutable pool: bitmap index out of range");
    if (P && !pool_ok(P)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    if (P && src >= P->n_bitmaps) return fail(c, RG_EINVAL, "source bitmap index out of range of its pool");
    return RG_OK;
}

}  // namespace

extern "C" {

rg_status rg_mpool_create(rg_ctx* c, uint32_t n_bitmaps, uint32_t n_slots, rg_mpool** out) {
    if (!c) return RG_EINVAL;
    if (!out) return fail(c, RG_EINVAL, "null mutable pool pointer");
    *out = nullptr;
    if (n_bitmaps < 1 || n_bitmaps > 16384 || n_slots < 1 || n_slots > (1u << 27))
        return fail(c, RG_EINVAL, "rg_mpool_create: 1 <= n_bitmaps <= 16384, 1 <= n_slots <= 2^27");
    HIPCHK(c, hipSetDevice(c->device));
    rg_mpool* mp = new rg_mpool();
    mp->ctx = c;
    MutView& v = mp->v;
    v.n_bitmaps = n_bitmaps;
    v.n_slots = n_slots;
    const uint64_t nd = (uint64_t)n_bitmaps * MUT_KEYS;
    size_t total = 0;
    for (size_t x : {4 * nd, (size_t)n_slots, 4 * (size_t)n_slots, 4 * (size_t)n_slots, 8 * (size_t)n_slots,
                     4 * (size_t)n_slots, (size_t)16, 8 * (size_t)n_bitmaps, 8 * (size_t)MUT_KEYS,
                     4 * (size_t)MUT_KEYS, (size_t)8, 8 * (size_t)(MUT_BATCH_MAX + 1),
                     8 * (size_t)MUT_BATCH_MAX * MUT_KEYS / 64})
        total += align256(x);
    if (hipMalloc(&mp->mem, total) != hipSuccess) {
        delete mp;
        return fail(c, RG_EDEVICE, "rg_mpool_create: hipMalloc failed");
    }
    if (hipMalloc(&mp->slab, (size_t)n_slots * MUT_SLOT_BYTES) != hipSuccess) {
        (void)hipFree(mp->mem);
        delete mp;
        return fail(c, RG_EDEVICE, "rg_mpool_create: hipMalloc of the slot slab failed");
    }
    Bump bp{static_cast<uint8_t*>(mp->mem)};
    v.dir = bp.take<uint32_t>(nd);
    v.s_type = bp.take<uint8_t>(n_slots);
    v.s_card = bp.take<uint32_t>(n_slots);
    v.s_size = bp.take<uint32_t>(n_slots);
    v.s_off = bp.take<uint64_t>(n_slots);
    v.free_list = bp.take<uint32_t>(n_slots);
    v.ctl = bp.take<int32_t>(4);
    v.bm_card = bp.take<uint64_t>(n_bitmaps);
    v.present = bp.take<uint32_t>(2 * (size_t)MUT_KEYS);
    v.absent = bp.take<uint32_t>(MUT_KEYS);
    v.counts = bp.take<uint32_t>(2);
    v.bbase = bp.take<uint64_t>(MUT_BATCH_MAX + 1);
    v.tbits = bp.take<uint64_t>((size_t)MUT_BATCH_MAX * MUT_KEYS / 64);
    v.slab = static_cast<uint8_t*>(mp->slab);
    launch_mut_init(v, nullptr);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(nullptr) != hipSuccess) {
        (void)hipFree(mp->slab);
        (void)hipFree(mp->mem);
        delete mp;
        return fail(c, RG_EDEVICE, "rg_mpool_create: initialisation failed");
    }
    *out = mp;
    return RG_OK;
}

void rg_mpool_destroy(rg_mpool* mp) {
    if (!mp) return;
    (void)hipSetDevice(mp->ctx->device);
    (void)hipDeviceSynchronize();
    if (mp->slab) (void)hipFree(mp->slab);
    if (mp->mem) (void)hipFree(mp->mem);
    delete mp;
}

rg_status rg_mpool_op(rg_mpool* mp, int op, uint32_t b, const rg_pool* P, uint32_t src, void* stream) {
    if (!mp) return RG_EINVAL;
    rg_ctx* c = mp->ctx;
    if (op < RG_AND || op > RG_ANDNOT) return fail(c, RG_EINVAL, "op must be RG_AND..RG_ANDNOT");
    if (!P) return fail(c, RG_EINVAL, "null pool");
    if (rg_status s = check_args(mp, b, P, src)) return s;
    HIPCHK(c, hipSetDevice(c->device));
    launch_mut_op(mp->v, op, b, *P, src, (hipStream_t)stream);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_mpool_op_batch(rg_mpool* mp, uint32_t n, const int* ops, const uint32_t* bitmaps, const rg_pool* P,
                            const uint32_t* srcs, void* stream) {
    if (!mp) return RG_EINVAL;
    rg_ctx* c = mp->ctx;
    if (n == 0) return RG_OK;
    if (!ops || !bitmaps || !srcs) return fail(c, RG_EINVAL, "rg_mpool_op_batch: null operation arrays");
    if (!P) return fail(c, RG_EINVAL, "null pool");
    std::vector<uint8_t> seen(mp->v.n_bitmaps, 0);
    for (uint32_t i = 0; i < n; ++i) {
        if (ops[i] < RG_AND || ops[i] > RG_ANDNOT) return fail(c, RG_EINVAL, "op must be RG_AND..RG_ANDNOT");
        if (rg_status s = check_args(mp, bitmaps[i], P, srcs[i])) return s;
        if (seen[bitmaps[i]]++) return fail(c, RG_EINVAL, "rg_mpool_op_batch: a bitmap appears twice");
    }
    HIPCHK(c, hipSetDevice(c->device));
    for (uint32_t i0 = 0; i0 < n; i0 += MUT_BATCH_MAX) {
        MutBatch bt{};
        bt.n = std::min<uint32_t>(MUT_BATCH_MAX, n - i0);
        for (uint32_t i = 0; i < bt.n; ++i) {
            bt.op[i] = ops[i0 + i];
            bt.b[i] = bitmaps[i0 + i];
            bt.src[i] = srcs[i0 + i];
        }
        launch_mut_batch(mp->v, bt, *P, (hipStream_t)stream);
    }
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status rg_mpool_clear(rg_mpool* mp, uint32_t b, void* stream) {
    if (!mp) return RG_EINVAL;
    if (rg_status s = check_args(mp, b, nullptr, 0)) return s;
    HIPCHK(mp->ctx, hipSetDevice(mp->ctx->device));
    launch_mut_clear(mp->v, b, (hipStream_t)stream);
    HIPCHK(mp->ctx, hipGetLastError());
    return RG_OK;
}

rg_status rg_mpool_assign(rg_mpool* mp, uint32_t b, const rg_pool* P, uint32_t src, void* stream) {
    if (!mp) return RG_EINVAL;
    if (!P) return fail(mp->ctx, RG_EINVAL, "null pool");
    if (rg_status s = check_args(mp, b, P, src)) return s;
    if (rg_status s = rg_mpool_clear(mp, b, stream)) return s;
    return rg_mpool_op(mp, RG_OR, b, P, src, stream);
}

rg_status rg_mpool_cards(rg_mpool* mp, uint64_t* d_cards, void* stream) {
    if (!mp) return RG_EINVAL;
    if (!d_cards) return fail(mp->ctx, RG_EINVAL, "rg_mpool_cards: null d_cards");
    HIPCHK(mp->ctx, hipSetDevice(mp->ctx->device));
    HIPCHK(mp->ctx, hipMemcpyAsync(d_cards, mp->v.bm_card, 8 * (size_t)mp->v.n_bitmaps, hipMemcpyDeviceToDevice,
                                   (hipStream_t)stream));
    return RG_OK;
}

rg_status rg_mpool_status(rg_mpool* mp, uint32_t* free_slots, void* stream) {
    if (!mp) return RG_EINVAL;
    rg_ctx* c = mp->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    int32_t h[4] = {0, 0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(h, mp->v.ctl, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (free_slots) *free_slots = (uint32_t)h[0];
    if (h[1]) {
        const int32_t zero = 0;
        HIPCHK(c, hipMemcpyAsync(mp->v.ctl + 1, &zero, 4, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
        return fail(c, RG_ECAPACITY, "an in-place operation was skipped: fewer free slots than keys to insert");
    }
    return RG_OK;
}

rg_status rg_mpool_export(rg_mpool* mp, uint32_t b0, uint32_t n, rg_out* out, void* stream) {
    if (!mp) return RG_EINVAL;
    rg_ctx* c = mp->ctx;
    if ((uint64_t)b0 + n > mp->v.n_bitmaps || n == 0) return fail(c, RG_EINVAL, "rg_mpool_export: bad bitmap range");
    if (!out || !out->bm_begin || !out->keys || !out->types || !out->card || !out->size || !out->off ||
        !out->payload || !out->bm_card)
        return fail(c, RG_EINVAL, "rg_mpool_export needs a complete rg_out");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    WorkspaceOrder order(c, st);
    Scratch sc(c);
    void* base = nullptr;
    if (rg_status s = sc.take(WS_PAIRS, 4 * align256(8 * ((size_t)n + 1)), &base)) return s;
    Bump bp{static_cast<uint8_t*>(base)};
    uint64_t* cnt = bp.take<uint64_t>(n + 1);
    uint64_t* bytes = bp.take<uint64_t>(n + 1);
    uint64_t* cbase = bp.take<uint64_t>(n + 1);
    uint64_t* pbase = bp.take<uint64_t>(n + 1);
    launch_mut_measure(mp->v, b0, n, cnt, bytes, st);
    uint8_t* hb = nullptr;
    if (rg_status s = host_buffer(c, 4 * 8 * ((size_t)n + 1), &hb)) return s;
    uint64_t* hc = reinterpret_cast<uint64_t*>(hb);
    uint64_t* hy = hc + (n + 1);
    uint64_t* hcb = hy + (n + 1);
    uint64_t* hpb = hcb + (n + 1);
    HIPCHK(c, hipMemcpyAsync(hc, cnt, 8 * n, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(hy, bytes, 8 * n, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    uint64_t tc = 0, tp = 0;
    for (uint32_t j = 0; j < n; ++j) {
        hcb[j] = tc;
        hpb[j] = tp;
        tc += hc[j];
        tp += hy[j];
    }
    hcb[n] = tc;
    hpb[n] = tp;
    out->needed_containers = tc;
    out->needed_payload_bytes = tp;
    out->n_containers = 0;
    out->payload_used = 0;
    if (out->cap_containers < tc || out->cap_payload_bytes < tp)
        return fail(c, RG_ECAPACITY, "rg_mpool_export: output arena too small");
    void* sbase = nullptr;
    if (rg_status s = sc.take(WS_WAVE, 4 * (size_t)std::max<uint64_t>(tc, 1), &sbase)) return s;
    HIPCHK(c, hipMemcpyAsync(cbase, hcb, 8 * (n + 1), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(pbase, hpb, 8 * (n + 1), hipMemcpyHostToDevice, st));
    launch_mut_export(mp->v, b0, n, cbase, pbase, tc, static_cast<uint32_t*>(sbase), *out, st);
    HIPCHK(c, hipGetLastError());
    // the staging above is read by the copies: finish before the next call reuses it
    HIPCHK(c, hipStreamSynchronize(st));
    out->n_containers = tc;
    out->payload_used = tp;
    return RG_OK;
}

}  // extern "C"
