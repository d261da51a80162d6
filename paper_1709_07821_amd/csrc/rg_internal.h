// rg_internal.h - shared declarations of the HIP kernels and the host
// orchestration of the Roaring set-operation library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/roaring_gpu.h"

namespace rg {

constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr int WAVE = 64;

// native 16-byte vector (global_load_dwordx4 / global_store_dwordx4)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// What one slot of the work space does. Slots are laid out per pair in key
// order of the result, so compaction of non-empty slots yields the result
// containers in ascending key order.
enum : uint8_t { KIND_NOOP = 0, KIND_MATCH = 1 };

// Kernel classes (bins). Variant selection decides the bin of every slot.
enum : uint8_t {
    BIN_BB = 0,     // bitset op bitset: one wave per pair, words in registers
    BIN_UNUSED = 1, // (no kernel class; keeps the variant numbers of the C ABI)
    BIN_GEN = 2,    // any pair: expand both sides into LDS bitsets, op, finalize
    BIN_AA = 3,     // array op array: LDS merge
    BIN_GALLOP = 4, // array op array, very unequal sizes: galloping search
    BIN_AB = 5,     // array op bitset (either order): probe / set / clear / flip
    BIN_RR = 6,     // run op run / run op array: interval merge
    BIN_THREAD = 7, // small array side: one thread per pair probes the other container
    PROF_REDO = 8,  // no bin: unused (a class number kept for the C ABI's variant numbering)
    BIN_FUSED = 9,  // small array sides counted inside key matching (count-only); never listed
    NBINS = 10
};
// profile classes beyond the bins
constexpr int PROF_FUSED = 10;  // the fused match-and-count kernel of asynchronous count-only calls
constexpr int PROF_KWEVAL = 11; // k-way evaluation of materialised unions, differences, symmetric differences
constexpr int PROF_KWSMALL = 12; // the one-wave array kernel on k-way slots
constexpr int PROF_KWBB = 13;    // the one-wave bitset kernel on k-way slots
constexpr int PROF_KWWAVE = 14;  // the one-wave fold of k-way unions and symmetric differences
constexpr int NPROF = 15;

struct Task {
    uint32_t pair;
    uint32_t ia;   // container index in pool A, or NONE
    uint32_t ib;   // container index in pool B, or NONE
    uint16_t key;
    uint8_t kind;
    uint8_t bin;
};
static_assert(sizeof(Task) == 16, "task record is 16 bytes");

struct PoolView {
    const uint64_t* bm_begin;
    const uint16_t* keys;
    const uint8_t* types;
    const uint32_t* card;
    const uint32_t* size;
    const uint64_t* off;
    const uint8_t* payload;
    const uint64_t* bm_card;
    const uint64_t* bm_wbytes;
    // Optional (plans): every container's metadata packed in one 16-byte record,
    // {data low word, data high word, card, size | inline << 21 | type << 24},
    // where data is the payload offset or, for an array of at most 4 values
    // (inline = 1), the values themselves (value i in bits 16i..16i+15). Key
    // matching reads one record per side instead of four arrays, and no payload
    // for the smallest arrays. Null: use the arrays.
    const u32x4* meta;
    // Optional: key-presence index, RG_KEY_INDEX_BYTES per bitmap (1024 u64
    // presence words, then 1024 u16 ranks: keys in the words before each word).
    // A key of bitmap b is found with one bit test and a popcount. Null: none.
    const uint8_t* kidx;
};

constexpr uint32_t META_INLINE_MAX = 4;  // array values held in a packed record
constexpr uint32_t KIDX_WORDS = 1024;
// Whether count-only calls and plans build a key index for their pools: when a
// bitmap has at least this many keys on average (fewer fit the LDS window).
constexpr uint64_t KIDX_MIN_MEAN_KEYS = 1024;
void launch_key_index(const PoolView& P, uint32_t n_bitmaps, uint8_t* out, hipStream_t st);
// A count-only call packs its pools' metadata when it visits at least this many
// candidate keys per container of the pools (packing costs one pass over them).
constexpr uint64_t META_PACK_FACTOR = 4;
// Packs the metadata records of a pool's n containers (PoolView::meta).
void launch_pack_meta(const PoolView& P, uint64_t n, u32x4* out, hipStream_t st);

// Per-wave result slots written by the compute kernels.
struct SlotOut {
    const uint64_t* slot_off;   // payload byte offset of each slot (absolute in out payload)
    uint8_t* payload;           // out payload base
    uint32_t* res_card;         // 0 = empty / no container
    uint8_t* res_type;
    uint32_t* res_size;
    // bytes of `payload`: a result that would end past it is not written (the
    // slot stays empty) and bit 2 is set in *err - only a pool whose
    // cardinalities disagree with its payload can get there
    uint64_t cap = ~0ull;
    uint32_t* err = nullptr;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Values that are the same in every lane of a wave (task indices, container
// types and sizes, counts summed over the wave or workgroup) are passed through
// readfirstlane so the compiler holds them in scalar registers and every
// branch, loop exit and early return that depends on them is scalar control
// flow. Barriers and cross-lane operations must only sit under such branches.
__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// lane l's value, in every lane (l uniform)
__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t l) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), l);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// index of the calling wave in a grid of 256-thread workgroups, as a scalar
__device__ __forceinline__ uint32_t wave_index() { return uniform(blockIdx.x * 4 + (threadIdx.x >> 6)); }

// a task record read by every lane of a wave, with all fields made uniform
__device__ __forceinline__ Task uniform_task(const Task* tasks, uint32_t slot) {
    const Task t = tasks[slot];
    Task u;
    u.pair = uniform(t.pair);
    u.ia = uniform(t.ia);
    u.ib = uniform(t.ib);
    const uint32_t w = uniform((uint32_t)t.key | ((uint32_t)t.kind << 16) | ((uint32_t)t.bin << 24));
    u.key = (uint16_t)w;
    u.kind = (uint8_t)(w >> 16);
    u.bin = (uint8_t)(w >> 24);
    return u;
}

__device__ __forceinline__ uint32_t round16(uint32_t b) { return (b + 15u) & ~15u; }

// P1: least-memory container type allowed by the size rules
__host__ __device__ __forceinline__ uint8_t p1_type(uint32_t c, uint32_t r) {
    bool run_ok = (c <= 4096u) ? (2u * r < c) : (r <= 2047u);
    if (run_ok) return RG_RUN;
    return c <= 4096u ? RG_ARRAY : RG_BITSET;
}

__host__ __device__ __forceinline__ uint32_t payload_bytes_of(uint8_t type, uint32_t size) {
    return type == RG_ARRAY ? 2u * size : type == RG_BITSET ? 8192u : 4u * size;
}

// bound on the payload of any container holding at most c values (P1 form)
__host__ __device__ __forceinline__ uint32_t wbytes_of(uint64_t c) {
    uint64_t b = 2 * c < 8192 ? 2 * c : 8192;
    return (uint32_t)((b + 15) & ~15ull);
}

template <int OP>
__device__ __forceinline__ uint64_t apply_op(uint64_t a, uint64_t b) {
    if (OP == RG_AND) return a & b;
    if (OP == RG_OR) return a | b;
    if (OP == RG_XOR) return a ^ b;
    return a & ~b;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return uniform(v);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return uniform64(v);
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t t = __shfl_up(v, o);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Block of 256 threads (4 waves): exclusive prefix sum and total. `tmp` must
// hold 4 uint32 in LDS; contains two barriers.
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t* tmp, uint32_t* total) {
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan_u32(v);
    if (lane == 63) tmp[wid] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < 4; ++w) {
        uint32_t t = tmp[w];
        if (w < wid) base += t;
        tot += t;
    }
    __syncthreads();
    *total = uniform(tot);
    return base + inc - v;
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t* tmp) {
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    v = wave_sum_u64(v);
    if (lane == 0) tmp[wid] = v;
    __syncthreads();
    uint64_t s = uniform64(tmp[0] + tmp[1] + tmp[2] + tmp[3]);
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- launchers
// (defined in the .hip files; all enqueue on `st`)

struct MatchArgs {
    int op;
    bool materialize;
    PoolView A, B;
    const uint32_t* ia;       // pair -> bitmap in A (device), or null: use ia0
    const uint32_t* ib;
    uint32_t ia0, ib0;        // single-pair form
    uint64_t pair0;           // first pair of this wave
    uint32_t n_pairs;         // pairs in this wave
    const uint64_t* cand_off; // [n_pairs + 1], wave-local candidate offsets
    uint64_t n_cand;
    Task* tasks;              // [n_cand]
    uint32_t* ub;             // [n_cand] slot payload bound in bytes (materialize)
    uint32_t* res_card;       // [n_cand]
    uint32_t* blk_cnt;        // [NBINS][match_blocks(n_cand)]: per-block bin counts, bin-major
    int dispatch_mode;        // 0 heuristic, 1 learned (mlp_table), 2 fixed
    int fixed_bin;
    uint32_t gallop_ratio;
    uint32_t thread_max;  // largest array side handled one thread per pair
    const uint8_t* mlp_table;  // learned dispatch: bin per quantised feature cell (mode 1)
    // count-only: pairs that land in BIN_THREAD are counted by the matching
    // thread itself into acc[pair] (wave-aggregated atomics) and emitted as
    // no-op tasks; their number goes to bin BIN_FUSED of blk_cnt
    bool fuse_thread;
    long long* acc;
    // k_count_fused with kernel timing on: matched container pairs are added
    // here (one atomic per block); null otherwise
    unsigned long long* matched = nullptr;
};

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st);
// out[0..3] = sum of n_cand, sum of bound, sum of min_cont (either may be
// null), max of n_cand over n pairs
void launch_pair_totals(const uint32_t* n_cand, const uint64_t* bound, const uint32_t* min_cont, uint64_t n,
                        uint64_t* out, hipStream_t st);
void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t st);
void launch_pair_prep(int op, bool materialize, PoolView A, PoolView B, uint32_t nA, uint32_t nB,
                      const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs,
                      uint32_t* n_cand, uint64_t* bound, uint32_t* min_cont, long long* acc, uint32_t* err,
                      hipStream_t st, uint32_t* zero_word = nullptr);
void launch_match(const MatchArgs& m, hipStream_t st);
// Asynchronous count-only path: key matching and counting of every pair in one
// persistent kernel (m.materialize false, m.fuse_thread true, m.pair0 0, m.cand_off
// the exclusive scan over all pairs with the total at cand_off[n_pairs]).
// *next_blk must be 0 at launch (k_pair_prep's zero_word).
uint32_t count_fused_blocks_per_cu();
void launch_count_fused(const MatchArgs& m, uint32_t* next_blk, uint32_t grid, hipStream_t st);
// Binning without contended atomics: k_match leaves per-block bin counts; an
// exclusive scan of them (bin-major) gives each block's place in each bin's
// list, and the bins' counts and offsets (bin_info[0..NBINS) counts,
// bin_info[NBINS..2 NBINS) offsets; next[] work counters reset when given).
// A key-matching block takes MATCH_SLOTS consecutive candidate slots, each of
// its 256 threads MATCH_PER_THREAD of them.
constexpr uint32_t MATCH_PER_THREAD = 4;
constexpr uint32_t MATCH_SLOTS = 256 * MATCH_PER_THREAD;
inline uint32_t match_blocks(uint64_t n_cand) { return (uint32_t)((n_cand + MATCH_SLOTS - 1) / MATCH_SLOTS); }
void launch_bin_layout(const uint32_t* blk_cnt, uint32_t nblk, uint64_t* blk_off, uint64_t* partials, uint64_t* total,
                       uint32_t* bin_info, uint32_t* next, hipStream_t st);
void launch_bin_scatter(const Task* tasks, uint64_t n, const uint32_t* blk_cnt, const uint64_t* blk_off,
                        uint32_t* bin_lists, hipStream_t st);
// exclusive scan of u32 into u64 with an added base (plus *base_dev when
// given, read on the device; it may be total_out itself); writes the total to
// *total_out (device)
void launch_scan_u32_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t base, uint64_t* partials,
                         uint64_t* total_out, hipStream_t st, const uint64_t* base_dev = nullptr);
// The same exclusive scan over (in[i] != 0): output positions of the non-empty results.
void launch_scan_nonzero_u64(const uint32_t* in, uint64_t* out, uint64_t n, uint64_t base, uint64_t* partials,
                             uint64_t* total_out, hipStream_t st, const uint64_t* base_dev = nullptr);
size_t scan_partials_needed(uint64_t n);

struct ComputeArgs {
    int op;
    bool materialize;
    PoolView A, B;
    const Task* tasks;
    const uint32_t* list;     // slot ids of this bin
    uint32_t n;
    long long* acc;           // count mode: per-pair (wave-local) accumulators
    uint64_t pair0;
    SlotOut so;
    float* cost;              // if non-null: per-slot cost in wave-cycles (training samples)
};

void launch_bb(const ComputeArgs& a, hipStream_t st);
void launch_generic(const ComputeArgs& a, hipStream_t st);
void launch_aa(const ComputeArgs& a, hipStream_t st);
void launch_gallop(const ComputeArgs& a, hipStream_t st);
void launch_ab(const ComputeArgs& a, hipStream_t st);
void launch_rr(const ComputeArgs& a, hipStream_t st);
void launch_thread(const ComputeArgs& a, hipStream_t st);
// materialised intersections listed in bin BIN_AA (small_mat_ok): one wave per pair
void launch_small_list(const ComputeArgs& a, hipStream_t st);

struct CompactArgs {
    const Task* tasks;
    uint64_t n_slots;
    const uint32_t* res_card;
    const uint8_t* res_type;
    const uint32_t* res_size;
    const uint64_t* slot_off;
    const uint64_t* out_idx;  // exclusive scan of (res_card > 0), includes the wave's output base
    uint16_t* keys;
    uint8_t* types;
    uint32_t* card;
    uint32_t* size;
    uint64_t* off;
    uint64_t* bm_card;        // indexed by global pair
    uint64_t* bm_wbytes;      // may be null
    uint64_t pair0;
};
void launch_compact(const CompactArgs& c, hipStream_t st);
void launch_bm_begin(const uint64_t* cand_off, const uint64_t* out_idx, uint64_t n_slots, const uint64_t* out_total,
                     uint32_t n_pairs, uint64_t pair0, uint64_t* bm_begin, bool last_wave, hipStream_t st);
// acc_op: the operation whose cardinality the accumulator holds; out_op: the
// operation whose cardinality goes to d_cards (converted with the Section 5.9
// identities when they differ)
// Pairs with an index outside its pool (nA / nB bitmaps) get count 0 and Jaccard 0.
void launch_finish_counts(int acc_op, int out_op, const long long* acc, PoolView A, PoolView B, uint32_t nA,
                          uint32_t nB, const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0,
                          uint64_t pair0, uint32_t n_pairs, uint64_t* d_cards, double* d_jacc, hipStream_t st);
void launch_mat_counts(int op, const uint64_t* bm_card, PoolView A, PoolView B, const uint32_t* ia,
                       const uint32_t* ib, uint32_t ia0, uint32_t ib0, uint64_t n_pairs, uint64_t* d_cards,
                       double* d_jacc, hipStream_t st);


// Which count variants may take a matched pair (forced and learned dispatch;
// the generic variant takes any pair). A forced or learned thread-per-pair
// choice needs an array side of at most THREAD_FORCE_MAX values: a thread
// probing a long array would hold its whole wave.
constexpr uint32_t THREAD_FORCE_MAX = 62;  // floor(log2(1 + c)) <= 5
__host__ __device__ __forceinline__ bool variant_applies(int bin, uint8_t ta, uint8_t tb, uint32_t ca, uint32_t cb) {
    const bool aa = ta == RG_ARRAY && tb == RG_ARRAY;
    const bool ab = (ta == RG_ARRAY && tb == RG_BITSET) || (ta == RG_BITSET && tb == RG_ARRAY);
    const bool run = ta == RG_RUN || tb == RG_RUN;
    switch (bin) {
    case BIN_GEN: return true;
    case BIN_AA: return aa;
    case BIN_GALLOP: return aa;
    case BIN_AB: return ab;
    case BIN_RR: return run;
    case BIN_THREAD: return (ta == RG_ARRAY && ca <= THREAD_FORCE_MAX) || (tb == RG_ARRAY && cb <= THREAD_FORCE_MAX);
    default: return false;
    }
}

// learned dispatcher (rg_mlp.hip)
constexpr int MLP_IN = 12, MLP_H = 64, MLP_OUT = 6;
constexpr int MLP_PARAMS = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H * MLP_OUT + MLP_OUT;
constexpr uint32_t MLP_TABLE = 3 * 3 * 17 * 17 * 12 * 12;  // type_a, type_b, log2 c_a, c_b, log2 r_a, r_b
__host__ __device__ __forceinline__ uint32_t mlp_cell(uint8_t ta, uint8_t tb, uint32_t ca, uint32_t cb, uint32_t ra,
                                                      uint32_t rb) {
    auto q = [](uint32_t c, uint32_t hi) {
        const uint32_t l = 31u - (uint32_t)__builtin_clz(c + 1u);  // floor(log2(1 + c))
        return l < hi ? l : hi;
    };
    const uint32_t qra = ta == RG_RUN ? q(ra, 11) : 0u, qrb = tb == RG_RUN ? q(rb, 11) : 0u;
    return ((((uint32_t)(ta - 1) * 3 + (uint32_t)(tb - 1)) * 17 + q(ca, 16)) * 17 + q(cb, 16)) * 144 + qra * 12 + qrb;
}
void launch_mlp_forward(const float* P, const float* X, uint64_t n, float* Y, hipStream_t st);
uint32_t mlp_grad_blocks(uint64_t n);
// d_inv: device scratch float (1 / unmasked count, computed here)
void launch_mlp_grad(const float* P, const float* X, const float* T, const uint8_t* M, uint64_t n, float* d_inv,
                     float* partial, float* partial_loss, float* grad, float* loss, hipStream_t st);
void launch_mlp_adam(float* P, const float* G, float* m, float* v, float lr, float b1, float b2, float eps, float c1,
                     float c2, hipStream_t st);
// training rows: features, and target column `col` from the measured costs
void launch_slot_features(const Task* tasks, uint64_t n, PoolView A, PoolView B, int want_bin, const float* cost,
                          int col, float* F, float* T, uint8_t* M, hipStream_t st);
void launch_gather_rows(const float* X, const float* T, const uint8_t* M, const uint32_t* idx, uint64_t b0,
                        uint32_t nb, float* Xb, float* Tb, uint8_t* Mb, hipStream_t st);
void launch_accum_scaled(const float* x, float* acc, float scale, hipStream_t st);
void launch_mlp_table(const float* P, uint8_t* table, hipStream_t st);

// Materialised pairs built by the one-wave array kernels (rg_small.hip);
// types 0 = absent (size 0). Union and symmetric difference: two arrays, or
// one, with at most SMALL_MAX values together. Intersection: an array side
// (with fewer values when both are arrays); the other side any container, an
// array of at most SMALL_MAX values. Difference: an array first operand; the
// second any container or absent, an array of at most SMALL_MAX values. Every
// such result has at most SMALL_MAX values: an array or runs, never a bitset.
// Also a lone run container (the other operand absent: union, symmetric
// difference, difference by nothing), whose result is the container itself
// in P1 form (touching runs merged; an array or a bitset when smaller).
constexpr uint32_t SMALL_MAX = 4096;
// values staged per wave: 8 KiB, so that a workgroup of four waves takes 32 KiB
// of LDS and five workgroups fit on a compute unit
constexpr uint32_t SMALL_LDS = SMALL_MAX;
__host__ __device__ __forceinline__ bool lone_run(int op, uint8_t ta, uint8_t tb) {
    return (ta == RG_RUN && tb == 0 && op != RG_AND) || (ta == 0 && tb == RG_RUN && (op == RG_OR || op == RG_XOR));
}
__host__ __device__ __forceinline__ bool small_mat_ok(int op, uint8_t ta, uint8_t tb, uint32_t sa, uint32_t sb) {
    const bool aa = ta == RG_ARRAY, ba = tb == RG_ARRAY;
    if (lone_run(op, ta, tb)) return true;
    if (op == RG_OR || op == RG_XOR)
        return (aa || ta == 0) && (ba || tb == 0) && (ta || tb) && (uint64_t)sa + sb <= SMALL_MAX;
    if (op == RG_AND) {
        if (aa && ba) return sa <= SMALL_MAX && sb <= SMALL_MAX;
        return (aa && sa <= SMALL_MAX && tb != 0) || (ba && sb <= SMALL_MAX && ta != 0);
    }
    if (op == RG_ANDNOT) return aa && sa <= SMALL_MAX && (!ba || sb <= SMALL_MAX);
    return false;
}

// k-way queries over one pool (rg_kway.hip)
// Task.bin of a k-way result key whose containers are recorded in Task.ia
// (first bitmap) and Task.ib (second), NONE where absent: queries of k <= 2.
constexpr uint8_t KW_TASK_INDEXED = 1;
// ... and whose result the one-wave array kernel builds (set by the bounds kernel)
constexpr uint8_t KW_TASK_SMALL = 2;
// ... whose containers are bitsets (or one bitset, the other absent): the
// one-wave bitset kernel builds the result and marks the task KW_TASK_DONE
constexpr uint8_t KW_TASK_BB = 3;
constexpr uint8_t KW_TASK_DONE = 4;
// ... of a union or symmetric difference of more than two bitmaps with at most
// KW_WAVE_MAX_K bitmaps: one wave folds the key's containers (k_kw_wave) and
// marks the task KW_TASK_DONE
constexpr uint8_t KW_TASK_WAVE = 5;
constexpr uint32_t KW_WAVE_MAX_K = 64;
// steps with more slots use k_kw_wave (measured on serving steps: past about
// 32 queries of 1024 result keys the wave fold serves more queries per second,
// below it the workgroup kernel has the lower latency)
constexpr uint64_t KW_WAVE_MIN_SLOTS = 32768;
__host__ __device__ __forceinline__ bool bb_mat_ok(int op, uint8_t ta, uint8_t tb) {
    if (ta == RG_BITSET && tb == RG_BITSET) return true;
    if (ta == RG_BITSET && tb == 0) return op != RG_AND;             // A alone: union, xor, difference
    if (ta == 0 && tb == RG_BITSET) return op == RG_OR || op == RG_XOR;  // B alone
    return false;
}
constexpr uint32_t KW_MATERIALIZE = 1u;  // KwQuery.flags: build the result containers
// KwQuery.flags: the query's key set is built in parts (KwPart), one workgroup
// each, combined in a key mask in device memory (KwQuery.pad = its index)
constexpr uint32_t KW_SPLIT = 2u;
constexpr uint32_t KW_MAX_K = 256;       // bitmaps per query (one lookup thread each)
constexpr uint32_t KW_AND_GROUP = 4;     // bitmaps whose key masks an intersection fills at once
constexpr uint32_t KW_PART_KEYS = 4096;  // keys per part of a split union or symmetric difference
constexpr uint32_t KW_PART_BITMAPS = 16; // bitmaps per part of a split key pass from presence indexes
// One part of a split key pass: the query's bitmaps j0 .. j1-1.
struct KwPart {
    uint32_t q;     // query index
    uint32_t j01;   // j0 | j1 << 16
    uint32_t mi;    // key mask (and arrival counter) of the query
    uint32_t n;     // parts of the query
};
struct KwQuery {
    uint32_t op;       // RG_AND, RG_OR, RG_XOR (fold of k) or RG_ANDNOT (first minus the others)
    uint32_t k;        // number of bitmaps, 1..KW_MAX_K
    uint32_t ids_off;  // first of the query's bitmap ids in KwArgs.ids
    uint32_t flags;    // KW_MATERIALIZE or 0 (count only)
    uint64_t slot0;    // first slot of the query's range
    uint32_t kbound;   // slots in the range (bound on result containers)
    uint32_t pad;      // KW_SPLIT: the query's key mask index
};
static_assert(sizeof(KwQuery) == 32, "query record is 32 bytes");
struct KwArgs {
    PoolView P0;        // pool of each query's first bitmap
    PoolView P1;        // pool of its other bitmaps (the same pool for k-way queries)
    uint32_t pair_base; // Task.pair = pair_base + query index (output bitmap index)
    const KwQuery* queries;
    uint32_t n_queries;
    const uint32_t* ids;
    Task* tasks;        // one per slot; pair = query index
    uint64_t n_slots;
    uint32_t* ub;       // payload bound per slot
    uint32_t* res_card; // per slot, 0 = empty
    SlotOut so;
    long long* acc;     // per query, count-only results
    uint32_t* err;      // set when a query's key set exceeds its slot range
    uint32_t small = 1; // materialised results with an array side go to the one-wave kernel
    uint32_t eval_chunk = 0;  // slots per evaluation workgroup chunk (1..64; 0: by the slot count)
    uint32_t wave = 0;        // unions and symmetric differences of many bitmaps go to k_kw_wave
    const KwPart* parts = nullptr;  // parts of split key passes
    uint32_t n_parts = 0;
    uint64_t* kmask = nullptr;      // 1024 words per split query, zero before the key pass
    uint32_t* kdone = nullptr;      // parts finished, per split query, zero before the key pass
};
// The container of `key` in bitmap b (its global index), or NONE. With the
// pool's key-presence index: the presence bit, then the word's rank plus the
// popcount of the bits below (two independent loads); otherwise a binary
// search of the bitmap's keys.
__device__ __forceinline__ uint32_t kw_find_key(const uint64_t* bm_begin, const uint16_t* keys, const uint8_t* kidx,
                                                uint32_t b, uint16_t key) {
    const uint64_t s = bm_begin[b], e = bm_begin[b + 1];
    if (kidx) {
        const uint8_t* ix = kidx + (uint64_t)b * RG_KEY_INDEX_BYTES;
        const uint32_t wi = key >> 6, bit = key & 63u;
        const uint64_t x = reinterpret_cast<const uint64_t*>(ix)[wi];
        const uint32_t rank = reinterpret_cast<const uint16_t*>(ix + 8 * KIDX_WORDS)[wi];
        if (!((x >> bit) & 1ull)) return NONE;
        return (uint32_t)(s + rank + (uint32_t)__popcll(x & ((1ull << bit) - 1ull)));
    }
    uint64_t lo = s, hi = e;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < e && keys[lo] == key) ? (uint32_t)lo : NONE;
}

// kmask / kdone: the split queries' key masks (n_masks x 1024 words) and arrival counters, zeroed
void launch_kw_step_init(uint64_t* totals, uint32_t* err, long long* acc, uint64_t* bm_card, uint64_t* bm_wbytes,
                         uint32_t nq, uint64_t* kmask, uint32_t* kdone, uint32_t n_masks, hipStream_t st);
// the key pass: parts of split queries (when a.n_parts), then the others.
// pairs: some query has at most two bitmaps (the one-wave key kernel's);
// whole: some query of more is not split (the workgroup kernel's).
void launch_kw_keys(const KwArgs& a, hipStream_t st, bool pairs = true, bool whole = true);
// pairs_only: every query has at most two bitmaps (one thread per slot)
void launch_kw_bounds(const KwArgs& a, hipStream_t st, bool pairs_only = false);
// the two evaluation kernels: the one-wave array kernel for the slots the
// bounds kernel marked (rg_small.hip), the workgroup kernel for the others
void launch_kw_small(const KwArgs& a, hipStream_t st);
void launch_kw_bb(const KwArgs& a, hipStream_t st);
void launch_kw_wave(const KwArgs& a, hipStream_t st);
void launch_kw_eval(const KwArgs& a, hipStream_t st);
void launch_kw_cards(const KwArgs& a, const uint64_t* bm_card, uint64_t* cards, hipStream_t st);
// queries q < n_pairs for pairs pair0 + q (k = 2: A side, B side), slot ranges
// from cand_off; single: k = 1 union queries of the A side (its P1 form)
void launch_kw_pair_queries(int op, const uint32_t* ia, const uint32_t* ib, uint32_t ia0, uint32_t ib0,
                            uint64_t pair0, uint32_t n_pairs, const uint64_t* cand_off, KwQuery* queries,
                            uint32_t* ids, hipStream_t st, bool single = false);
// out[4j..4j+3] = key count, payload bound, 1, first key | last key << 16 (all 0 for an id
// outside the pool; the span 0 for a bitmap without keys). launch_kw_key_span: the span
// of every bitmap of a pool.
void launch_kw_gather_meta(const uint64_t* bm_begin, const uint16_t* keys, const uint64_t* bm_wbytes,
                           uint32_t n_bitmaps, const uint32_t* ids, uint32_t k, uint64_t* out, hipStream_t st);
void launch_kw_key_span(const uint64_t* bm_begin, const uint16_t* keys, uint32_t n, uint32_t* out, hipStream_t st);

// pool utilities
void launch_pool_recount(const rg_pool& p, hipStream_t st);
void launch_pool_dense_init(const rg_pool& p, uint32_t n_keys, hipStream_t st);
// p1: also require the least-memory (P1) container types and maximal runs
void launch_pool_validate(const rg_pool& p, uint64_t* d_bad, bool p1, hipStream_t st);
void launch_pool_digest(const rg_pool& p, uint64_t* d_digest, hipStream_t st);
// containers i >= *d_n (device count) are skipped
void launch_pool_digest_n(const rg_pool& p, const uint64_t* d_n, uint64_t* d_digest, hipStream_t st);

}  // namespace rg
