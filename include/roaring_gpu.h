/*
 * roaring_gpu.h - C ABI of the MI355X (gfx950) Roaring-bitmap set-operation
 * library. All device work runs in the library's own HIP kernels.
 *
 * Paper: Lemire et al., "Roaring Bitmaps: Implementation of an Optimized
 * Software Library" (arXiv:1709.07821).
 *
 * ---------------------------------------------------------------------------
 * Data format (Section 1, Figure 1; Section 2.2; Section 3.2)
 * ---------------------------------------------------------------------------
 * A bitmap is a set of uint32 values. Its values are grouped by their 16 high
 * bits (the key); each non-empty group is one container that stores the 16
 * low bits in one of three forms:
 *   RG_ARRAY  - c sorted distinct uint16 (c <= 4096), 2c bytes;
 *   RG_BITSET - 1024 uint64 words, value x at bit (x & 63) of word (x >> 6)
 *               (Section 3.2 bit addressing), 8192 bytes;
 *   RG_RUN    - r pairs (start, length-1) of uint16, sorted, disjoint and
 *               maximal (no two runs touch), 4r bytes. A full chunk is the
 *               single pair (0, 65535).
 * Every container is in the least-memory form allowed by the Section 1 size
 * rules ("P1"): run if (c <= 4096 ? 2r < c : r <= 2047), else array if
 * c <= 4096, else bitset (r = number of maximal runs). Empty containers are
 * never stored (Section 2.2). The library's outputs always obey these rules;
 * its inputs must (rg_pool_validate checks them).
 *
 * A pool holds many bitmaps in structure-of-arrays form in device memory.
 * Containers of bitmap b are [bm_begin[b], bm_begin[b+1]) with strictly
 * ascending keys. Every payload offset is a multiple of 16 and the payload
 * buffer may be read in whole 16-byte units up to the end of each container's
 * last 16-byte unit (so payload_bytes is a multiple of 16).
 *
 * Ownership: every pointer in rg_pool / rg_out is device memory owned by the
 * caller (in practice torch tensors). The library only reads pools and only
 * writes the rg_out buffers and its own workspace (held by the context).
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 * Calls enqueue work on it. Count-only calls (cardinalities, Jaccard) are
 * asynchronous: they never wait for the device. Materialising calls must size
 * their launches and report arena capacity, so they read small counters back
 * and synchronise the stream at those points. On return from a successful call
 * every result has been computed or is enqueued on `stream` (synchronise
 * before reading).
 *
 * Workspace: calls need device scratch. By default the context owns it and
 * grows it on demand (hipMalloc). A caller that must not see allocations gives
 * the context a workspace of its own (rg_set_workspace, sized with
 * rg_workspace_size); calls then carve their scratch from it, never allocate
 * device memory, and fail with RG_ECAPACITY when it is too small.
 *
 * Errors: every call returns an rg_status; on failure rg_last_error(ctx)
 * describes it. Outputs are unspecified after a failed call. Errors that only
 * the device can see in an asynchronous call (a pair index outside its pool)
 * give that pair count 0 / Jaccard 0 and raise a flag that rg_sync reports.
 */
#ifndef ROARING_GPU_H
#define ROARING_GPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RG_OK = 0,
    RG_EINVAL = -1,     /* bad argument (null pointer, index out of range, bad op) */
    RG_ECAPACITY = -2,  /* rg_out too small; needed_* fields say what is needed */
    RG_EDEVICE = -3,    /* a HIP runtime call failed */
    RG_EFORMAT = -4,    /* pool violates the container format (validation) */
    RG_ENOTSUP = -5     /* not supported */
} rg_status;

typedef enum { RG_ARRAY = 1, RG_BITSET = 2, RG_RUN = 3 } rg_ctype;

/* The four operations of Section 1: intersection, union, symmetric
 * difference, and difference A \ B (Section 4.4 direction). */
typedef enum { RG_AND = 0, RG_OR = 1, RG_XOR = 2, RG_ANDNOT = 3 } rg_op;

/* roaring_batch flags */
#define RG_FLAG_MATERIALIZE 1u /* build the result bitmaps into rg_out */
#define RG_FLAG_CARD 2u        /* write |result| per pair into d_cards (uint64) */
#define RG_FLAG_JACCARD 4u     /* write |A n B| / |A u B| per pair into d_jacc (binary64) */
#define RG_FLAG_DIGEST 8u      /* serving queries: also compute the result's fingerprint */

typedef struct rg_ctx rg_ctx;

/* Read-only pool of bitmaps (device pointers). */
typedef struct rg_pool {
    uint32_t n_bitmaps;
    uint64_t n_containers;     /* < 2^32 */
    uint64_t payload_bytes;    /* multiple of 16 */
    const uint64_t *bm_begin;  /* [n_bitmaps + 1], bm_begin[n_bitmaps] == n_containers; bm_begin[0] is 0
                                  except for a window into larger arrays (rg_result.view), where the
                                  containers before it belong to no bitmap of the view */
    const uint16_t *keys;      /* [n_containers], ascending within a bitmap */
    const uint8_t *types;      /* [n_containers], rg_ctype */
    const uint32_t *card;      /* [n_containers], 1..65536 */
    const uint32_t *size;      /* [n_containers], array: c, bitset: 1024, run: r */
    const uint64_t *off;       /* [n_containers], byte offset into payload, multiple of 16 */
    const uint8_t *payload;    /* [payload_bytes] */
    const uint64_t *bm_card;   /* [n_bitmaps], total cardinality of each bitmap */
    const uint64_t *bm_wbytes; /* [n_bitmaps], sum over its containers of
                                  roundup16(min(8192, 2 * card)): bounds result payloads */
    const uint32_t *meta;      /* optional, may be NULL: [4 * n_containers], the packed
                                  records rg_pool_pack_meta writes. When set, key matching
                                  reads one record per matched container instead of the
                                  separate arrays; it must match the arrays. */
    const uint8_t *key_index;  /* optional, may be NULL: [RG_KEY_INDEX_BYTES * n_bitmaps], the
                                  key-presence index rg_pool_key_index writes. When set, key
                                  matching finds a key of this pool's bitmaps with a bit test and
                                  a popcount instead of a binary search, and k-way queries take
                                  their key sets from the presence words; it must match keys. */
} rg_pool;

/* Bytes of the key-presence index per bitmap: 1024 uint64 words with bit
 * (key & 63) of word (key >> 6) set for every key of the bitmap, then 1024
 * uint16 ranks (keys of the bitmap in the words before each word). */
#define RG_KEY_INDEX_BYTES 10240

/* Caller-provided output arena (device pointers) for materialised results:
 * result bitmap p (one per pair) occupies containers [bm_begin[p],
 * bm_begin[p+1]). Container payloads are written at 16-byte-aligned offsets
 * inside per-container slots, so payload may contain unused gaps. */
typedef struct rg_out {
    uint64_t cap_containers;       /* in: entries available in keys/types/card/size/off */
    uint64_t cap_payload_bytes;    /* in: bytes available in payload */
    uint64_t *bm_begin;            /* [n_pairs + 1] */
    uint16_t *keys;
    uint8_t *types;
    uint32_t *card;
    uint32_t *size;
    uint64_t *off;
    uint8_t *payload;
    uint64_t *bm_card;             /* [n_pairs] */
    uint64_t *bm_wbytes;           /* [n_pairs], may be NULL; makes the output usable as a pool */
    uint64_t needed_containers;    /* out (host): upper bound the call requires */
    uint64_t needed_payload_bytes; /* out (host): payload bytes the call requires */
    uint64_t n_containers;         /* out (host): containers written */
    uint64_t payload_used;         /* out (host): end of the last written slot */
} rg_out;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device`. The context owns a growable device
 * workspace and pinned host staging; it is not thread-safe (one per thread).
 * Calls that use the workspace may be issued on different streams: each waits,
 * on the device, for the previous one to finish with it. */
rg_status rg_create(rg_ctx **ctx, int device);
void rg_destroy(rg_ctx *ctx);
const char *rg_last_error(const rg_ctx *ctx);

/* Waits for `stream` and reports what asynchronous calls of the context found
 * on the device since the last rg_sync: RG_EINVAL if a pair index was outside
 * its pool (the flag is then cleared), else RG_OK. */
rg_status rg_sync(rg_ctx *ctx, void *stream);

/* Caller-owned workspace. d_ws: device memory, 256-byte aligned, owned by the
 * caller, which must keep it valid while calls that use it may run; NULL
 * returns to the context's own growable workspace. Waits for the last call
 * that used the previous workspace. With a workspace set, calls allocate no
 * device memory and never call hipDeviceSynchronize: pair calls, batches,
 * roaring_multi and rg_mlp_grad take their scratch from it (plans, servers
 * and the dispatcher's sampling and training keep their own memory, made at
 * creation). Calls on different streams that share it are ordered on the
 * device, as with the context's own workspace. */
rg_status rg_set_workspace(rg_ctx *ctx, void *d_ws, uint64_t bytes);
/* Bytes of workspace that a roaring_batch (or pair call: n_pairs = 1) with
 * this op, flags and pools needs. Count-only: exact (per-pair arrays, plus the
 * pools' packed metadata records when the call would pack them). Materialising:
 * the least that runs the call (per-pair arrays and one wave of the largest
 * pair's candidate slots); more lets it run in fewer waves. No device work. */
rg_status rg_workspace_size(rg_ctx *ctx, int op, uint32_t flags, const rg_pool *A, const rg_pool *B,
                            uint64_t n_pairs, uint64_t *bytes);

/* ---- two-bitmap operations (Section 1 operations; Section 5.7: inputs are
 * left unchanged and the result is built as a new bitmap) ----------------- */

/* Result of A[ia] op B[ib] into `out` (one result bitmap). Returns
 * RG_ECAPACITY with out->needed_* filled if the arena is too small.
 * Intersections are built per matched key pair by the binned kernels; union,
 * symmetric difference and difference per result key by the k-way kernels
 * (two bitmaps per query; see roaring_multi). */
rg_status roaring_and(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib, rg_out *out,
                      void *stream);
rg_status roaring_or(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib, rg_out *out,
                     void *stream);
rg_status roaring_xor(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib, rg_out *out,
                      void *stream);
rg_status roaring_andnot(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib, rg_out *out,
                         void *stream);

/* |A[ia] op B[ib]| into device uint64 *d_card, without building the result
 * (Section 4.1.2 fused operation + population count; Section 5.9). */
rg_status roaring_and_cardinality(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib,
                                  uint64_t *d_card, void *stream);
rg_status roaring_or_cardinality(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib,
                                 uint64_t *d_card, void *stream);
rg_status roaring_xor_cardinality(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib,
                                  uint64_t *d_card, void *stream);
rg_status roaring_andnot_cardinality(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib,
                                     uint64_t *d_card, void *stream);

/* Jaccard index |A n B| / |A u B| (Section 5.9) into device double *d_j:
 * exact integer counts, then one IEEE binary64 round-to-nearest division;
 * two empty sets give 1.0. */
rg_status roaring_jaccard(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib, double *d_j,
                          void *stream);
/* The same index into host double *h_j; synchronises `stream`. */
rg_status roaring_jaccard_host(rg_ctx *ctx, const rg_pool *A, uint32_t ia, const rg_pool *B, uint32_t ib, double *h_j,
                               void *stream);

/* Batched: for p < n_pairs, A[d_ia[p]] op B[d_ib[p]] (d_ia, d_ib device
 * uint32 arrays). flags: RG_FLAG_MATERIALIZE (results into out, result
 * bitmap p = pair p), RG_FLAG_CARD (|result| into d_cards[p]),
 * RG_FLAG_JACCARD (Jaccard of the two inputs into d_jacc[p]; derived from
 * the same count through the Section 5.9 identities). Without
 * RG_FLAG_MATERIALIZE the call is asynchronous: one kernel matches the keys of
 * all pairs and counts every matched container pair, and the number of
 * candidate keys never goes to the host; an index outside its pool is
 * reported by rg_sync. With it, the call synchronises (arena sizing) and
 * reports a bad index as RG_EINVAL. */
rg_status roaring_batch(rg_ctx *ctx, int op, const rg_pool *A, const rg_pool *B, const uint32_t *d_ia,
                        const uint32_t *d_ib, uint64_t n_pairs, uint32_t flags, rg_out *out, uint64_t *d_cards,
                        double *d_jacc, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * roaring_batch's count-only form (flags RG_FLAG_CARD and/or RG_FLAG_JACCARD;
 * RG_FLAG_MATERIALIZE is RG_ENOTSUP) with every byte of its scratch taken
 * from a fixed device array of RG_STATIC_SCRATCH_BYTES that the library holds
 * on each GPU it runs on until the process ends (its address is looked up by
 * rg_create). The call allocates nothing (no hipMalloc / hipFree, no events,
 * no pinned memory), never waits for the device, and gives the same counts
 * and Jaccard values as roaring_batch. At most RG_STATIC_MAX_PAIRS pairs per
 * call (more: RG_ECAPACITY before any device work). The pools' packed
 * metadata records are built in the same array when they fit beside the
 * per-pair scratch, else the call reads the pool arrays. Every call on a GPU
 * shares that GPU's array and overwrites what the last call left there: calls
 * of one context are ordered on the device (as calls sharing a workspace
 * are), but calls from two contexts that overlap on one GPU race and give
 * wrong results. Kernel timing (rg_profile_*) does not cover these calls. */
#define RG_STATIC_SCRATCH_BYTES (32ull << 20)
#define RG_STATIC_MAX_PAIRS (1ull << 20)
rg_status roaring_batch_static(rg_ctx *ctx, int op, const rg_pool *A, const rg_pool *B, const uint32_t *d_ia,
                               const uint32_t *d_ib, uint64_t n_pairs, uint32_t flags, uint64_t *d_cards,
                               double *d_jacc, void *stream);

/* ---- batched count-only plans (pointer-stable, graph-capturable) --------
 * A plan fixes the pools, the pairs (d_ia/d_ib, device uint32), the op and the
 * outputs (d_cards uint64 and/or d_jacc binary64, one per pair). Creating it
 * checks the pair indices and reads the per-pair key-candidate counts back
 * once (synchronising) and allocates its own device memory. rg_plan_execute
 * then enqueues the whole batch on `stream` - per-pair seeds, a device scan of
 * the candidate counts, one persistent work-stealing kernel that matches the
 * keys of every pair and counts every matched container pair (workgroups take
 * blocks of candidate keys from a counter), count finishing - with no host
 * synchronisation and no allocation. rg_plan_capture records that
 * sequence into a hipGraph on a non-default stream; later executes replay it.
 * rg_plan_tune times the plan on its own data and keeps the fastest setting of
 * the thread-size threshold, the persistent grid size and the galloping ratio,
 * one after the other (results never change). The pools, pair arrays and
 * outputs must stay valid and unmoved for the plan's life. The pools' contents
 * must not change either: the plan keeps a packed copy of their container
 * metadata (16 bytes per container) and, for pools with many keys per bitmap,
 * their key-presence indexes (RG_KEY_INDEX_BYTES per bitmap), made at creation
 * unless the pools carry them; without the memory for them the plan reads the
 * pool arrays and searches the keys. The pair arrays' contents may change
 * between executions as long as every pair's candidate count (number of keys
 * of its smaller bitmap) does not. */
typedef struct rg_plan rg_plan;
/* A materialising plan (Section 5.7: a new result bitmap for every pair):
 * the same, with flags holding RG_FLAG_MATERIALIZE (plus optional
 * RG_FLAG_CARD / RG_FLAG_JACCARD) and the results built into `out`, result
 * bitmap p = pair p. Creation reads every pair's result bounds back once and
 * fails with RG_ECAPACITY (out->needed_* filled) when the arena is smaller than
 * their sum; each execution is then sync-free and graph-capturable: result
 * keys, payload bounds, one workgroup per result key, scan and compaction of
 * the non-empty results, every wave's arena offsets carried on the device.
 * All four operations go through the k-way kernels (two bitmaps per query,
 * as roaring_or does). After an execution has completed, the arena holds the
 * results; rg_plan_result synchronises `stream` and reads the container count
 * and the end of the last payload slot; rg_plan_totals gives the device
 * address of the same two values (uint64 [payload end, containers]) for
 * callers that stay on the device. The arena and pools must stay valid and
 * unmoved for the plan's life. rg_plan_tune leaves materialising plans as
 * they are (nothing to tune). */
rg_status rg_plan_create_mat(rg_ctx *ctx, int op, const rg_pool *A, const rg_pool *B, const uint32_t *d_ia,
                             const uint32_t *d_ib, uint64_t n_pairs, uint32_t flags, rg_out *out, uint64_t *d_cards,
                             double *d_jacc, rg_plan **plan, void *stream);
rg_status rg_plan_result(rg_plan *plan, uint64_t *n_containers, uint64_t *payload_used, void *stream);
rg_status rg_plan_totals(const rg_plan *plan, const uint64_t **d_totals);
/* Largest number of candidate slots per wave of a batched call or plan
 * (default 2^24, at most 2^30): smaller waves need less workspace and more
 * launches. A wave always holds whole pairs. Results never change. */
rg_status rg_set_wave_slots(rg_ctx *ctx, uint64_t max_slots);
rg_status rg_plan_create(rg_ctx *ctx, int op, const rg_pool *A, const rg_pool *B, const uint32_t *d_ia,
                         const uint32_t *d_ib, uint64_t n_pairs, uint32_t flags, uint64_t *d_cards, double *d_jacc,
                         rg_plan **plan, void *stream);
rg_status rg_plan_execute(rg_plan *plan, void *stream);
rg_status rg_plan_capture(rg_plan *plan, void *stream);
rg_status rg_plan_tune(rg_plan *plan, void *stream, int reps);
/* Sets the persistent grid, galloping ratio and thread-size threshold (see
 * rg_set_thresholds); drops a captured graph (returns RG_ENOTSUP if one
 * existed: capture again). RG_EINVAL for grid 0, ratio 0, threshold > 4096. */
rg_status rg_plan_set(rg_plan *plan, uint32_t grid, uint32_t gallop_ratio, uint32_t thread_max);
/* Any output pointer may be NULL. */
rg_status rg_plan_info(const rg_plan *plan, uint32_t *grid, uint32_t *gallop_ratio, uint32_t *thread_max,
                       uint64_t *slots, uint32_t *waves, int *graph);
void rg_plan_destroy(rg_plan *plan);

/* Kernel-variant selection for matched container pairs. Every variant
 * computes the same result; they differ only in speed.
 *   mode RG_DISPATCH_HEURISTIC (default): size-ratio / type heuristic;
 *   mode RG_DISPATCH_MLP: the learned dispatcher (count-only pairs; needs a
 *   network installed with rg_dispatch_set_mlp, else RG_EINVAL);
 *   mode RG_DISPATCH_FIXED: use `variant` wherever it applies to the pair's
 *   container types, the generic variant elsewhere (bitset-bitset pairs
 *   always use their own kernel). */
#define RG_DISPATCH_HEURISTIC 0
#define RG_DISPATCH_MLP 1 /* learned: the table installed by rg_dispatch_set_mlp */
#define RG_DISPATCH_FIXED 2
#define RG_V_GENERIC 2   /* both sides expanded to LDS bitsets, any types */
#define RG_V_MERGE 3     /* array-array merge */
#define RG_V_GALLOP 4    /* array-array galloping search (Section 2.2) */
#define RG_V_PROBE 5     /* array-bitset probe / set / clear / flip (Section 3.2) */
#define RG_V_RUNMERGE 6  /* run-run and run-array interval merge */
#define RG_V_THREAD 7    /* one thread per pair: array-side values looked up in the other container */
rg_status rg_set_dispatch(rg_ctx *ctx, int mode, int variant);

/* Heuristic thresholds of a context (inherited by plans made from it):
 * galloping when max(c_A, c_B) >= gallop_ratio * min(c_A, c_B) for two arrays
 * (the paper gives no value, Section 2.2; default 64), and one thread per pair
 * when an array side holds at most thread_max values (default 8; 0 disables).
 * RG_EINVAL for gallop_ratio 0 or thread_max > 4096. Results never change. */
rg_status rg_set_thresholds(rg_ctx *ctx, uint32_t gallop_ratio, uint32_t thread_max);

/* ---- learned dispatcher --------------------------------------------------
 * Not from the paper (its variant rule is fixed, Section 2.2): a 12 -> 64 ->
 * 64 -> 6 ReLU network, fp32, that predicts the log2 cost of each count
 * variant (outputs v = 0..5 are RG_V_GENERIC + v) of one matched container
 * pair from 12 features: one-hot type of each side (3 + 3), log2(1 + c)/16 of
 * each side, log2(1 + r)/16 of each side (r = run count of a run container,
 * else 0), log2(max c / max(1, min c))/16, op/3 (0: count-only pairs always
 * compute the intersection). Parameters: flat fp32 [RG_MLP_PARAMS], W1[12][64],
 * b1[64], W2[64][64], b2[64], W3[64][6], b3[6], row-major, device memory. */
#define RG_MLP_PARAMS 5382
#define RG_MLP_TABLE 374544
/* y[n][6] = network(x[n][12]) (device arrays). */
rg_status rg_mlp_forward(rg_ctx *ctx, const float *d_params, const float *d_x, uint64_t n, float *d_y, void *stream);
/* Gradient of the masked mean squared error sum(m (y - t)^2) / sum(m) over
 * the n samples (t, m: [n][6]; m bytes 0/1) into d_grad[RG_MLP_PARAMS], the
 * loss into d_loss[0] (may be NULL). Sums in a fixed order of 256-sample
 * blocks; within a block the order of fp32 additions is not fixed. */
rg_status rg_mlp_grad(rg_ctx *ctx, const float *d_params, const float *d_x, const float *d_t, const uint8_t *d_m,
                      uint64_t n, float *d_grad, float *d_loss, void *stream);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected for step >= 1) on
 * d_params with moment buffers d_m, d_v [RG_MLP_PARAMS]. */
rg_status rg_mlp_adam(rg_ctx *ctx, float *d_params, const float *d_grad, float *d_m, float *d_v, uint32_t step,
                      float lr, void *stream);
/* Training samples measured by the count kernels themselves: runs the
 * count-only intersection of the pairs with `variant` (RG_V_GENERIC ..
 * RG_V_THREAD) forced where it applies and records each slot's cost in
 * wave-cycles (s_memtime; a workgroup task counts four waves, a thread task
 * its wave's time shared by the active lanes). Writes, per slot s < *n_slots,
 * the features d_x[s][12] (zeros for an unmatched slot), and column
 * variant - RG_V_GENERIC of d_t[s][6] (log2 cost) and d_m[s][6] (1 when the
 * slot is a matched pair that ran with `variant`). Calling it once per variant
 * fills all columns. All pairs must fit one wave of slots; RG_ECAPACITY (with
 * *n_slots set) when *n_slots > cap_slots. Synchronises. */
rg_status rg_dispatch_sample(rg_ctx *ctx, const rg_pool *A, const rg_pool *B, const uint32_t *d_ia,
                             const uint32_t *d_ib, uint64_t n_pairs, int variant, float *d_x, float *d_t,
                             uint8_t *d_m, uint64_t cap_slots, uint64_t *n_slots, void *stream);
/* Adam training on (x[n][12], t[n][6], m[n][6]) for `epochs` passes in
 * shuffled batches of `batch`; seed != 0 initialises d_params first (He
 * normal weights, zero biases, counter-based generator). d_epoch_loss[epochs]
 * receives the mean batch loss of each epoch. Synchronises. */
rg_status rg_dispatch_train(rg_ctx *ctx, const float *d_x, const float *d_t, const uint8_t *d_m, uint64_t n,
                            uint32_t epochs, uint32_t batch, float lr, uint64_t seed, float *d_params,
                            float *d_epoch_loss, void *stream);
/* Installs a trained network: evaluates it on the quantised feature grid
 * (type x type x 17 log2-cardinality buckets x 17 x 12 log2-run buckets x 12,
 * bucket centres), keeps the cheapest applicable variant of each cell, and
 * switches the context to RG_DISPATCH_MLP. Results never change. */
rg_status rg_dispatch_set_mlp(rg_ctx *ctx, const float *d_params, void *stream);
/* Copies the installed table (RG_MLP_TABLE bytes of variant numbers) to host memory. */
rg_status rg_dispatch_table(rg_ctx *ctx, uint8_t *h_table, uint64_t cap);

/* Kernel timing. When enabled, every compute-kernel launch of a call is
 * bracketed by two HIP events recorded on the call's stream; rg_profile_read
 * waits for them and returns the accumulated time, launch count and number of
 * container pairs processed for one variant (RG_V_* or 0 for the
 * bitset-bitset kernel, 8 for the bitset pairs redone
 * by the generic kernel, 9 for the small-array pairs of count-only calls that
 * key matching counts itself: items only, their time is part of key matching,
 * 10 for the fused match-and-count kernel of count-only calls (items: matched
 * container pairs, counted by the kernel while timing is on),
 * 11 for the k-way evaluation of materialised unions, symmetric differences
 * and differences (items: result slots), 12 for the one-wave kernel that
 * builds those of their results with an array side, 13 for the one-wave
 * kernel that builds their bitset results of bitset containers, 14 for the
 * one-wave fold of k-way unions and symmetric differences of up to 64 bitmaps
 * (items: result slots scanned); variant 3 (RG_V_MERGE) in materialising form is the one-wave
 * array kernel on the intersections that have an array side) in count-only
 * (materialize = 0) or materialising form. Synchronises on the
 * recorded events; costs two events per launch. */
rg_status rg_profile_enable(rg_ctx *ctx, int on);
rg_status rg_profile_reset(rg_ctx *ctx);
rg_status rg_profile_read(rg_ctx *ctx, int variant, int materialize, double *total_ms, uint64_t *launches,
                          uint64_t *items);

/* ---- k-way queries and the serving loop ---------------------------------
 * roaring_multi: the intersection (op RG_AND), union (RG_OR), symmetric
 * difference (RG_XOR: the values held by an odd number of the k bitmaps) or
 * difference (RG_ANDNOT: the first bitmap minus all the others) of k bitmaps
 * of one pool, d_ids[0..k) (device uint32, 1 <= k <= 256, ids may repeat).
 * The paper builds wide unions and intersections by folding pairwise or by
 * lazy aggregation (Section 2.2, Section 5.9); here each result container is
 * built directly from the k input containers of its key. flags:
 * RG_FLAG_MATERIALIZE (result bitmap 0 of `out`, which needs bm_wbytes) and/or
 * RG_FLAG_CARD (cardinality into d_card[0], device uint64). Output sizing as
 * for the pairwise calls (RG_ECAPACITY with needed_*), from each bitmap's key
 * count K_i and first and last key: at most min_i K_i and the keys between
 * the largest first key and the smallest last key (AND; none when that range
 * is empty), min(sum_i K_i, the keys between the smallest first key and the
 * largest last key) (OR, XOR) or K_1 (ANDNOT) containers, and payload bytes
 * at most the matching min / sum / first of the bm_wbytes and 8192 per
 * container. Synchronises on `stream` (one small readback of the ids' key
 * counts, payload bounds and key spans). */
rg_status roaring_multi(rg_ctx *ctx, int op, const rg_pool *pool, const uint32_t *d_ids, uint32_t k, uint32_t flags,
                        rg_out *out, uint64_t *d_card, void *stream);

/* A query of the serving loop: op RG_AND, RG_OR, RG_XOR or RG_ANDNOT (as for
 * roaring_multi) over k bitmap ids (host
 * array, copied at submission) of the server's pool; flags RG_FLAG_CARD
 * (count only) or RG_FLAG_MATERIALIZE (the result containers are built and
 * stay readable through rg_result.view until the query is released), plus
 * RG_FLAG_DIGEST for the result's fingerprint in rg_result.digest (one more
 * kernel in the query's step; without it digest is 0). */
typedef struct rg_query {
    int op;
    uint32_t k;
    const uint32_t *ids;
    uint32_t flags;
} rg_query;

typedef struct rg_result {
    int done;              /* 0: not finished yet (the other fields are unset) */
    int status;            /* RG_OK, or the failure of the step that ran it */
    uint64_t card;         /* |result| */
    uint64_t digest;       /* fingerprint of the result's container form (RG_FLAG_DIGEST; 0 for
                              count-only queries and queries without the flag) */
    uint64_t n_containers;
    uint64_t latency_ns;   /* arrival (or submission) to result-ready */
    rg_pool view;          /* materialised result as a one-bitmap window into the
                              server's arena (bm_begin[0..1] are absolute container
                              indices); valid until rg_serve_release */
} rg_result;

typedef struct rg_serve_stats {
    uint64_t queries;      /* finished */
    uint64_t steps;        /* device steps run */
    double mean_batch;     /* queries per step */
    uint64_t arena_peak_bytes;
    uint64_t deferred;     /* times the queue head waited for arena memory */
} rg_serve_stats;

typedef struct rg_server rg_server;

/* Starts a server thread over a device-resident pool. Queries are admitted in
 * arrival order into device steps of at most max_batch queries (1..4096) whose
 * result bound fits the arena (arena_bytes of device memory, allocated here):
 * queries arriving while steps run join the next step, and up to max_inflight
 * (1 or 2) steps are on the GPU at once, on two streams. max_batch = 1 and
 * max_inflight = 1 serve one query at a time. The pool must stay valid and
 * unchanged while the server runs; its per-bitmap key counts, payload bounds
 * and first and last keys are read back here (query bounds as for
 * roaring_multi), and a key_index on it is used as in roaring_multi. The
 * server thread uses its own buffers,
 * streams and error record, never the context's, so the caller may go on
 * using ctx for other calls meanwhile (a failed step is reported by
 * rg_serve_poll and rg_serve_stop). */
rg_status rg_serve_start(rg_ctx *ctx, const rg_pool *pool, uint64_t arena_bytes, uint32_t max_batch,
                         uint32_t max_inflight, rg_server **server);
/* Non-blocking. arrival_ns: the query's arrival time on the steady clock in
 * ns (latency is measured from it), or 0 for "now". RG_EINVAL for a bad query,
 * RG_ECAPACITY if its result bound alone exceeds the arena. Thread-safe. */
rg_status rg_serve_submit(rg_server *server, const rg_query *query, uint64_t arrival_ns, uint64_t *ticket);
/* wait = 0: returns at once (result->done says whether it finished);
 * wait = 1: blocks until it has. Thread-safe. */
rg_status rg_serve_poll(rg_server *server, uint64_t ticket, int wait, rg_result *result);
/* Frees a finished query's result memory and its ticket. */
rg_status rg_serve_release(rg_server *server, uint64_t ticket);
/* Open-loop replay: submits qs[i] at arrival_ns[i] (ns after the call starts,
 * non-decreasing), waits for all, and returns each query's latency, card and
 * digest (any output array may be NULL). Results are released as they finish. */
rg_status rg_serve_replay(rg_server *server, uint64_t n, const rg_query *qs, const uint64_t *arrival_ns,
                          uint64_t *latency_ns, uint64_t *cards, uint64_t *digests);
/* Drains, stops the thread, frees everything; stats may be NULL. */
rg_status rg_serve_stop(rg_server *server, rg_serve_stats *stats);

/* ---- access to values ----------------------------------------------------
 * Membership (Section 1: the value's 16 high bits are found among the sorted
 * keys by binary search, then the container is searched - binary search in an
 * array, bit test in a bitset (Section 3.2), search of the run starts in a run
 * container; Section 5.6 times such queries): for i < n, d_out[i] (device
 * uint8) = 1 if d_values[i] is in bitmap d_ids[i] of P, else 0 (d_ids,
 * d_values device uint32). Asynchronous, no allocation; an id outside the pool
 * gives 0 and is reported by rg_sync. */
rg_status roaring_contains(rg_ctx *ctx, const rg_pool *P, const uint32_t *d_ids, const uint32_t *d_values, uint64_t n,
                           uint8_t *d_out, void *stream);

/* Export to sorted uint32 values (Section 3.1: a bitset's set bits are turned
 * into values by counting each word's bits and extracting their positions;
 * Section 5.5 iterates over every value): the values of bitmaps b0 .. b0+n-1
 * of P, each ascending, concatenated in bitmap order into d_values (device
 * uint32, room for cap_values); d_offsets[j] (device uint64, n + 1 entries)
 * receives the index of bitmap b0 + j's first value and d_offsets[n] the total.
 * *needed_values (host, may be NULL) receives the total (the sum of the
 * bitmaps' bm_card); RG_ECAPACITY when it exceeds cap_values (nothing
 * written). RG_EINVAL when b0 + n > n_bitmaps. Synchronises once (the
 * total). */
rg_status roaring_to_uint32(rg_ctx *ctx, const rg_pool *P, uint32_t b0, uint32_t n, uint64_t *d_offsets,
                            uint32_t *d_values, uint64_t cap_values, uint64_t *needed_values, void *stream);

/* ---- mutable bitmaps: in-place operations ---------------------------------
 * The paper updates containers in place: values of an array are set, cleared
 * or flipped in a bitset while its cardinality is kept (Section 3.2), and wide
 * unions are built partly in place (Section 5.9). A mutable pool holds
 * n_bitmaps bitmaps that change in place: every bitmap has a directory of all
 * 65536 keys, and containers live in fixed 8 KiB slots (any P1 container fits,
 * so a result is written back where its input was) taken from and returned to
 * a device free list of n_slots slots. Memory: 256 KiB per bitmap plus
 * 8 KiB + 25 B per slot, allocated by rg_mpool_create. Every bitmap starts
 * empty; containers always stay in P1 form and each bitmap's cardinality is
 * maintained by every operation (no recount).
 *
 * rg_mpool_op: M[b] op= P[src] (P an ordinary pool; union, intersection,
 * symmetric difference, difference A \ B), asynchronous on `stream`. Only
 * the keys of P[src] are visited (intersection also drops M[b]'s keys that
 * P[src] lacks): a key in both is recomputed in M[b]'s slot, a key only in
 * P[src] takes a free slot (union, symmetric difference), an empty result
 * frees its slot. When the keys to insert outnumber the free slots the whole
 * operation is skipped on the device (M[b] unchanged) and rg_mpool_status
 * reports RG_ECAPACITY. rg_mpool_assign: M[b] = P[src]; rg_mpool_clear:
 * M[b] = {}. rg_mpool_cards: copies the n_bitmaps maintained cardinalities
 * (uint64) into d_cards (device, caller-owned), enqueued on `stream`.
 * rg_mpool_status: synchronises `stream`, gives the free
 * slots, and returns RG_ECAPACITY once if an operation was skipped since the
 * last call. rg_mpool_export: bitmaps b0 .. b0+n-1 as an ordinary pool in
 * `out` (P1, ascending keys; sizing as for roaring_batch with needed_*);
 * synchronises. Calls on one mutable pool must be ordered (one stream, or
 * the caller's synchronisation): they share its work lists. */
typedef struct rg_mpool rg_mpool;
rg_status rg_mpool_create(rg_ctx *ctx, uint32_t n_bitmaps, uint32_t n_slots, rg_mpool **mp);
void rg_mpool_destroy(rg_mpool *mp);
rg_status rg_mpool_op(rg_mpool *mp, int op, uint32_t b, const rg_pool *P, uint32_t src, void *stream);
/* n operations at once: M[bitmaps[i]] ops[i]= P[srcs[i]] (host arrays, the
 * bitmaps distinct: RG_EINVAL otherwise), run as device batches of up to 64
 * operations, each in the same six launches whatever its size. The keys the
 * batch's unions and symmetric differences insert are checked against the
 * free slots for the batch as a whole: when they do not fit, the whole batch
 * is skipped (its bitmaps unchanged) and rg_mpool_status reports
 * RG_ECAPACITY. Results equal the operations applied one by one. */
rg_status rg_mpool_op_batch(rg_mpool *mp, uint32_t n, const int *ops, const uint32_t *bitmaps, const rg_pool *P,
                            const uint32_t *srcs, void *stream);
rg_status rg_mpool_assign(rg_mpool *mp, uint32_t b, const rg_pool *P, uint32_t src, void *stream);
rg_status rg_mpool_clear(rg_mpool *mp, uint32_t b, void *stream);
rg_status rg_mpool_cards(rg_mpool *mp, uint64_t *d_cards, void *stream);
rg_status rg_mpool_status(rg_mpool *mp, uint32_t *free_slots, void *stream);
rg_status rg_mpool_export(rg_mpool *mp, uint32_t b0, uint32_t n, rg_out *out, void *stream);

/* ---- pools -------------------------------------------------------------- */

/* Host-side pool construction from sorted values. Bitmap b holds
 * values[offsets[b] .. offsets[b+1]) (strictly increasing uint32).
 * rg_pool_measure_host gives the sizes; rg_pool_build_host fills host arrays
 * of those sizes (payload zero-padded to 16-byte units) in the format above.
 * Returns RG_EINVAL if a bitmap's values are not strictly increasing. */
rg_status rg_pool_measure_host(const uint32_t *values, const uint64_t *offsets, uint32_t n_bitmaps,
                               uint64_t *n_containers, uint64_t *payload_bytes);
rg_status rg_pool_build_host(const uint32_t *values, const uint64_t *offsets, uint32_t n_bitmaps, uint64_t *bm_begin,
                             uint16_t *keys, uint8_t *types, uint32_t *card, uint32_t *size, uint64_t *off,
                             uint8_t *payload, uint64_t *bm_card, uint64_t *bm_wbytes);

/* Recompute card (from payload), bm_card and bm_wbytes of a device pool whose
 * bm_begin/keys/types/size/off/payload are set. The card/bm_card/bm_wbytes
 * pointers of `pool` are written through (they must be writable). */
rg_status rg_pool_recount(rg_ctx *ctx, const rg_pool *pool, void *stream);

/* Fills the metadata of a pool of dense bitsets: `pool` points at writable
 * device arrays for n_bitmaps bitmaps of n_keys containers each
 * (n_containers = n_bitmaps * n_keys) and at a payload of n_containers x 1024
 * uint64 words laid out [bitmap][key][word] (Section 3.2 bit addressing).
 * Writes bm_begin, keys (0..n_keys-1 in every bitmap), types (bitset), size,
 * off, then card, bm_card and bm_wbytes as rg_pool_recount does. The bitsets
 * must be in P1 form (more than 4096 values, more than 2047 runs) for the pool
 * to validate. Enqueued on `stream`, no synchronisation. */
rg_status rg_pool_init_dense(rg_ctx *ctx, const rg_pool *pool, uint32_t n_keys, void *stream);

/* Packs every container's type, cardinality, size and payload offset into one
 * 16-byte record: d_meta (device, caller-owned, 16 * n_containers bytes, 16-byte
 * aligned) receives {data low, data high, card, size | inline << 21 | type << 24}
 * per container, data being the payload offset or, for an array of at most 4
 * values (inline = 1), the values (value i in bits 16i..16i+15). Setting
 * pool.meta = d_meta afterwards lets key matching read one record per side of
 * each matched container pair (and no payload for the smallest arrays); the
 * pool must then not change while meta is set. Not from the paper: a layout
 * choice for gathers on this GPU. Enqueued on `stream`, no synchronisation. */
rg_status rg_pool_pack_meta(rg_ctx *ctx, const rg_pool *pool, uint32_t *d_meta, void *stream);

/* Key-presence index of every bitmap of a pool (layout at RG_KEY_INDEX_BYTES)
 * into d_index (device, caller-owned, RG_KEY_INDEX_BYTES * n_bitmaps bytes,
 * 16-byte aligned). Setting pool.key_index = d_index lets key matching find a
 * key in O(1) - the key-matching step turned into a bitset operation: the
 * presence bit, then the container's index from the word's rank plus the
 * popcount of the bits below. Count-only calls and plans build it in their own
 * memory when the pools have many keys per bitmap; a pool that carries it is
 * never indexed again. Enqueued on `stream`, no synchronisation. */
rg_status rg_pool_key_index(rg_ctx *ctx, const rg_pool *pool, uint8_t *d_index, void *stream);

/* Check every container of a device pool against the format rules above;
 * *n_bad (host) receives the number of offending containers. Synchronises.
 * rg_pool_validate checks everything, including the P1 form (Section 1 size
 * rules) and maximal runs: the form every call but rg_pool_canonicalize
 * requires. rg_pool_check with rules 0 checks only that the pool is
 * well-formed Roaring data: keys ascending; arrays of 1..65536 strictly
 * increasing values; bitsets with at least one bit; runs sorted and disjoint
 * (they may touch), at most 65536; card, bm_card and bm_wbytes consistent
 * with the payload - what rg_pool_canonicalize accepts. RG_RULES_P1 adds the
 * P1 rules (rg_pool_validate). */
#define RG_RULES_P1 1u
rg_status rg_pool_validate(rg_ctx *ctx, const rg_pool *pool, uint64_t *n_bad, void *stream);
rg_status rg_pool_check(rg_ctx *ctx, const rg_pool *pool, uint32_t rules, uint64_t *n_bad, void *stream);

/* Canonicalisation (the paper's inputs are run-optimised before any timing,
 * Section 5.1; the Section 1 size rules pick each container's type for least
 * memory): rebuilds every bitmap of a well-formed pool `in` (rg_pool_check
 * with rules 0; card, bm_card and bm_wbytes must be right, which
 * rg_pool_recount ensures) into `out` in P1 form - arrays longer than 4096
 * values become bitsets or runs, sparse bitsets arrays or runs, touching runs
 * merge, and every container takes the least-memory type. Result bitmap b =
 * input bitmap b. Output sizing as for roaring_batch (RG_ECAPACITY with
 * needed_*: at most n_containers containers and the sum of bm_wbytes payload
 * bytes). Synchronises (arena sizing). */
rg_status rg_pool_canonicalize(rg_ctx *ctx, const rg_pool *in, rg_out *out, void *stream);

/* Per-bitmap fingerprint of the container form into device uint64
 * d_digest[n_bitmaps]: the sum, over containers and their serialised 64-bit
 * words w_i (w0 = key | type << 16 | card << 32, w1 = size, then the payload
 * packed little-endian into 64-bit words, zero padded), of
 * mix64(w_i + (key * 2^20 + i + 1) * 0x9E3779B97F4A7C15) mod 2^64, with mix64
 * the SplitMix64 finalizer. */
rg_status rg_pool_digest(rg_ctx *ctx, const rg_pool *pool, uint64_t *d_digest, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ROARING_GPU_H */
