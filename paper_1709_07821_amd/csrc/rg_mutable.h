// rg_mutable.h - mutable pools: bitmaps changed in place (A op= B) with their
// cardinalities kept up to date, over a device slot allocator.
#pragma once
#include "rg_internal.h"

namespace rg {

constexpr uint32_t MUT_KEYS = 65536;     // directory entries per bitmap (every possible key)
constexpr uint32_t MUT_SLOT_BYTES = 8192;  // one slot holds any container in P1 form

// Device arrays of a mutable pool.
struct MutView {
    uint32_t n_bitmaps;
    uint32_t n_slots;
    uint32_t* dir;         // [n_bitmaps][65536]: slot of the container of each key, or NONE
    uint8_t* s_type;       // per slot
    uint32_t* s_card;
    uint32_t* s_size;
    uint64_t* s_off;       // per slot: its byte offset in slab (slot * 8192)
    uint8_t* slab;         // [n_slots][8192]
    uint32_t* free_list;   // [n_slots]: free slots, the first ctl[0] entries
    int32_t* ctl;          // [0] free slots, [1] sticky capacity error, [2] keys to insert, [3] abort current op
    uint64_t* bm_card;     // [n_bitmaps]
    uint32_t* present;     // [65536 x 2]: (container of B, slot of A) for keys in both
    uint32_t* absent;      // [65536]: containers of B whose key A lacks
    uint32_t* counts;      // [2]: entries of present, absent
    // batches of operations on distinct bitmaps (launch_mut_batch)
    uint64_t* bbase;       // [MUT_BATCH_MAX + 1]: exclusive prefix of the B operands' key counts
    uint64_t* tbits;       // [MUT_BATCH_MAX * 65536 / 64]: per (operation, key of B), set when A lacks the key
};

constexpr uint32_t MUT_BATCH_MAX = 64;  // operations per device batch

// one batch: M[b[i]] op[i]= P[src[i]] for i < n, the b[i] distinct (passed by value)
struct MutBatch {
    uint32_t n;
    int32_t op[MUT_BATCH_MAX];
    uint32_t b[MUT_BATCH_MAX];
    uint32_t src[MUT_BATCH_MAX];
};

void launch_mut_init(const MutView& m, hipStream_t st);
// M[b] op= P[src]: classify B's keys, check the free slots, drop / evaluate /
// insert, adjusting bm_card[b] by each key's change of cardinality
void launch_mut_op(const MutView& m, int op, uint32_t b, const rg_pool& P, uint32_t src, hipStream_t st);
// a batch of operations on distinct bitmaps in six launches: the keys every
// union / symmetric difference inserts are counted and checked against the
// free slots for the whole batch (skipped as a whole, sticky error, when they
// do not fit), then drop (intersections), evaluate, insert as for one op
void launch_mut_batch(const MutView& m, const MutBatch& bt, const rg_pool& P, hipStream_t st);
void launch_mut_clear(const MutView& m, uint32_t b, hipStream_t st);
// export of bitmaps b0 .. b0+n-1: per bitmap container count and payload bytes
void launch_mut_measure(const MutView& m, uint32_t b0, uint32_t n, uint64_t* cnt, uint64_t* bytes, hipStream_t st);
// writes out (metadata at the given per-bitmap container and payload bases) and copies payloads
void launch_mut_export(const MutView& m, uint32_t b0, uint32_t n, const uint64_t* cbase, const uint64_t* pbase,
                       uint64_t n_out, uint32_t* src_slot, const rg_out& out, hipStream_t st);

}  // namespace rg
