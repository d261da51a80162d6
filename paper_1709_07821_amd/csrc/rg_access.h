// rg_access.h - launchers of the access kernels (rg_access.hip): batched
// membership queries, and export of bitmaps to sorted uint32 values.
#pragma once
#include "rg_internal.h"

namespace rg {

// out[i] = 1 if values[i] is in bitmap ids[i] of P, else 0. An id outside the
// pool gives 0 and sets *err.
void launch_contains(const rg_pool& P, const uint32_t* ids, const uint32_t* values, uint64_t n, uint8_t* out,
                     uint32_t* err, hipStream_t st);

// range[0] = bm_begin[b0], range[1] = bm_begin[b0 + n], range[2] = sum of
// bm_card over bitmaps b0 .. b0 + n - 1 (one workgroup).
void launch_export_range(const rg_pool& P, uint32_t b0, uint32_t n, uint64_t* range, hipStream_t st);

// Export of containers [c0, c1) (the containers of bitmaps b0 .. b0 + n - 1):
// val_off[i - c0] is the exclusive prefix sum of their cardinalities; writes
// offsets[j] = val_off[bm_begin[b0 + j] - c0] for j <= n, then every value of
// container i as key << 16 | low at values[val_off[i - c0] ...], ascending
// (no write at or past values[cap]).
void launch_export_offsets(const rg_pool& P, uint32_t b0, uint32_t n, uint64_t c0, const uint64_t* val_off,
                           uint64_t total, uint64_t* offsets, hipStream_t st);
void launch_export_values(const rg_pool& P, uint64_t c0, uint64_t c1, const uint64_t* val_off, uint32_t* values,
                          uint64_t cap, hipStream_t st);

}  // namespace rg
