// rg_access_api.cpp - C ABI of the access calls: batched membership and
// export of bitmaps to sorted uint32 values.
#include "rg_access.h"
#include "rg_host.h"

extern "C" {

rg_status roaring_contains(rg_ctx* c, const rg_pool* P, const uint32_t* d_ids, const uint32_t* d_values, uint64_t n,
                           uint8_t* d_out, void* stream) {
    if (!c) return RG_EINVAL;
    if (!pool_ok(P)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    if (n && (!d_ids || !d_values || !d_out)) return fail(c, RG_EINVAL, "roaring_contains: null device array");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    WorkspaceOrder order(c, st);  // the asynchronous error word is the context's
    launch_contains(*P, d_ids, d_values, n, d_out, async_err_word(c), st);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

rg_status roaring_to_uint32(rg_ctx* c, const rg_pool* P, uint32_t b0, uint32_t n, uint64_t* d_offsets,
                            uint32_t* d_values, uint64_t cap_values, uint64_t* needed_values, void* stream) {
    if (!c) return RG_EINVAL;
    if (!pool_ok(P)) return fail(c, RG_EINVAL, "incomplete pool (null pointer)");
    if ((uint64_t)b0 + n > P->n_bitmaps) return fail(c, RG_EINVAL, "roaring_to_uint32: bitmaps outside the pool");
    if (!d_offsets) return fail(c, RG_EINVAL, "roaring_to_uint32: null d_offsets");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    WorkspaceOrder order(c, st);
    // the containers of the range and its value count, read back once
    uint64_t* d_range = reinterpret_cast<uint64_t*>(static_cast<uint8_t*>(c->small) + SMALL_EXPORT_RANGE);
    launch_export_range(*P, b0, n, d_range, st);
    uint64_t* h = static_cast<uint64_t*>(c->host);
    HIPCHK(c, hipMemcpyAsync(h, d_range, 24, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const uint64_t c0 = h[0], c1 = h[1], total = h[2];
    if (needed_values) *needed_values = total;
    if (c1 < c0 || c1 > P->n_containers) return fail(c, RG_EINVAL, "roaring_to_uint32: inconsistent bm_begin");
    if (total > cap_values) return fail(c, RG_ECAPACITY, "roaring_to_uint32: d_values holds fewer than the values");
    if (total && !d_values) return fail(c, RG_EINVAL, "roaring_to_uint32: null d_values");
    const uint64_t nc = c1 - c0;
    Scratch sc(c);
    void* base = nullptr;
    if (rg_status s = sc.take(WS_PAIRS, align256(8 * (nc + 1)) + align256(8 * scan_partials_needed(nc)), &base))
        return s;
    Bump bp{static_cast<uint8_t*>(base)};
    uint64_t* val_off = bp.take<uint64_t>(nc + 1);
    uint64_t* partials = bp.take<uint64_t>(scan_partials_needed(nc));
    launch_scan_u32_u64(P->card + c0, val_off, nc, 0, partials, val_off + nc, st);
    launch_export_offsets(*P, b0, n, c0, val_off, total, d_offsets, st);
    launch_export_values(*P, c0, c1, val_off, d_values, cap_values, st);
    HIPCHK(c, hipGetLastError());
    return RG_OK;
}

}  // extern "C"
