// rg_finalize.h - device routines shared by the workgroup (256-thread)
// kernels: expansion of any container into an LDS bitset, and the output
// step that turns a result bitset held in registers into a P1 container.
#pragma once
#include "rg_internal.h"

namespace rg {

// LDS scratch of one 256-thread workgroup
struct WgShared {
    uint64_t sa[1024];   // 8 KiB
    uint64_t sb[1024];   // 8 KiB
    uint32_t tmp[8];
    uint64_t tmp64[4];
    uint32_t xchg[8];
};

// Expand container `idx` of pool P into the LDS bitset s (1024 words).
// Array: set one bit per value (Section 3.2: value x is bit x & 63 of word
// x >> 6). Run: mark a toggle at each run start and one past each run end,
// then a prefix XOR over all 65536 bits (in-word shift-xor ladder, across
// words a ballot-based parity scan) leaves exactly the run bits set.
// Bitset: copied. Ends with a barrier. idx == NONE gives the empty set.
__device__ inline void expand_container(uint64_t* s, const PoolView& P, uint32_t idx, WgShared& sh) {
    const uint32_t tid = threadIdx.x;
    // type, size and offset are the same for the whole workgroup; as scalars
    // they keep every branch below (each holds barriers) uniform control flow
    const uint8_t type = idx == NONE ? 0 : (uint8_t)uniform(P.types[idx]);
    const uint32_t size = idx == NONE ? 0 : uniform(P.size[idx]);
    const uint8_t* pl = idx == NONE ? nullptr : P.payload + uniform64(P.off[idx]);
    if (type == RG_BITSET) {
        const u32x4* src = reinterpret_cast<const u32x4*>(pl);
        for (uint32_t i = tid; i < 512; i += 256) {
            u32x4 v = src[i];
            s[2 * i] = (uint64_t)v.x | ((uint64_t)v.y << 32);
            s[2 * i + 1] = (uint64_t)v.z | ((uint64_t)v.w << 32);
        }
        __syncthreads();
        return;
    }
    for (uint32_t i = tid; i < 1024; i += 256) s[i] = 0;
    __syncthreads();
    if (type == RG_ARRAY) {
        const uint16_t* v = reinterpret_cast<const uint16_t*>(pl);
        const uint32_t c = size;
        for (uint32_t i = tid; i < c; i += 256) {
            uint32_t x = v[i];
            atomicOr(reinterpret_cast<unsigned long long*>(&s[x >> 6]), 1ull << (x & 63));
        }
        __syncthreads();
    } else if (type == RG_RUN) {
        const uint32_t* rp = reinterpret_cast<const uint32_t*>(pl);
        const uint32_t r = size;
        for (uint32_t i = tid; i < r; i += 256) {
            uint32_t pr = rp[i];
            uint32_t st = pr & 0xFFFFu, e = st + (pr >> 16) + 1;
            atomicXor(reinterpret_cast<unsigned long long*>(&s[st >> 6]), 1ull << (st & 63));
            if (e < 65536u) atomicXor(reinterpret_cast<unsigned long long*>(&s[e >> 6]), 1ull << (e & 63));
        }
        __syncthreads();
        uint64_t w[4];
        uint32_t par = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w[j] = s[4 * tid + j];
            par ^= __popcll(w[j]) & 1u;
        }
        // exclusive XOR-scan of thread parities: ballot within the wave, LDS across waves
        const uint32_t lane = lane_id(), wid = tid >> 6;
        uint64_t bal = __ballot(par);
        uint32_t excl = __popcll(bal & ((1ull << lane) - 1ull)) & 1u;
        if (lane == 0) sh.xchg[wid] = __popcll(bal) & 1u;
        __syncthreads();
        for (uint32_t q = 0; q < wid; ++q) excl ^= sh.xchg[q];
        uint32_t carry = excl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint64_t x = w[j];
            uint32_t pj = __popcll(x) & 1u;
            x ^= x << 1;
            x ^= x << 2;
            x ^= x << 4;
            x ^= x << 8;
            x ^= x << 16;
            x ^= x << 32;
            s[4 * tid + j] = x ^ (carry ? ~0ull : 0ull);
            carry ^= pj;
        }
        __syncthreads();
    } else {
        __syncthreads();
    }
}

// Output step. Thread t holds result words 4t..4t+3 in w. Computes the
// cardinality c (population count) and the number of runs r, chooses the P1
// type, and writes the container into its slot: bitset words as they are;
// array by extracting set-bit positions (Section 3.1, count-then-extract with
// a workgroup prefix sum for the write positions); runs as (start, len-1)
// pairs from the run-start and run-end masks. `stage` (>= 8 KiB of LDS, free
// for reuse) collects starts and ends. Returns c to all threads.
__device__ inline uint32_t finalize_words(const uint64_t (&w)[4], uint32_t slot, const SlotOut& so, uint64_t* stage_s,
                                          uint64_t* stage_e, WgShared& sh) {
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    uint32_t ct = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) ct += __popcll(w[j]);
    // neighbour words: MSB of the previous word and LSB of the next word
    uint64_t prev = __shfl_up(w[3], 1);
    uint64_t next = __shfl_down(w[0], 1);
    if (lane == 63) sh.xchg[wid] = (uint32_t)(w[3] >> 63);
    if (lane == 0) sh.xchg[4 + wid] = (uint32_t)(w[0] & 1u);
    __syncthreads();
    uint32_t pmsb = (uint32_t)(prev >> 63), nlsb = (uint32_t)(next & 1u);
    if (lane == 0) pmsb = wid > 0 ? sh.xchg[wid - 1] : 0u;
    if (lane == 63) nlsb = wid < 3 ? sh.xchg[4 + wid + 1] : 0u;
    uint64_t st[4], en[4];
    uint32_t rs = 0, re = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint64_t below = j == 0 ? (uint64_t)pmsb : (w[j - 1] >> 63);
        uint64_t above = j == 3 ? (uint64_t)nlsb : (w[j + 1] & 1u);
        st[j] = w[j] & ~((w[j] << 1) | below);
        en[j] = w[j] & ~((w[j] >> 1) | (above << 63));
        rs += __popcll(st[j]);
        re += __popcll(en[j]);
    }
    uint64_t cr = block_sum_u64((uint64_t)ct | ((uint64_t)rs << 32), sh.tmp64);
    const uint32_t c = (uint32_t)cr, r = (uint32_t)(cr >> 32);
    if (c == 0) return 0;
    const uint8_t type = p1_type(c, r);
    const uint64_t nbytes = type == RG_ARRAY ? 2ull * c : type == RG_BITSET ? 8192ull : 4ull * r;
    if (so.slot_off[slot] + nbytes > so.cap) {  // the same decision in every thread
        if (tid == 0 && so.err) atomicOr(so.err, 2u);
        return c;
    }
    uint8_t* dst = so.payload + so.slot_off[slot];
    if (type == RG_BITSET) {
        u32x4* d4 = reinterpret_cast<u32x4*>(dst);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            u32x4 v;
            v.x = (uint32_t)w[2 * j];
            v.y = (uint32_t)(w[2 * j] >> 32);
            v.z = (uint32_t)w[2 * j + 1];
            v.w = (uint32_t)(w[2 * j + 1] >> 32);
            d4[2 * tid + j] = v;
        }
    } else if (type == RG_ARRAY) {
        uint32_t tot;
        uint32_t pos = block_excl_scan_u32(ct, sh.tmp, &tot);
        uint16_t* d16 = reinterpret_cast<uint16_t*>(dst);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint64_t x = w[j];
            const uint32_t base = (4 * tid + j) * 64;
            while (x) {
                d16[pos++] = (uint16_t)(base + __builtin_ctzll(x));
                x &= x - 1;
            }
        }
    } else {
        uint32_t tot;
        uint32_t ps = block_excl_scan_u32(rs, sh.tmp, &tot);
        uint32_t pe = block_excl_scan_u32(re, sh.tmp, &tot);
        uint16_t* ss = reinterpret_cast<uint16_t*>(stage_s);
        uint16_t* ee = reinterpret_cast<uint16_t*>(stage_e);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t base = (4 * tid + j) * 64;
            uint64_t x = st[j];
            while (x) {
                ss[ps++] = (uint16_t)(base + __builtin_ctzll(x));
                x &= x - 1;
            }
            x = en[j];
            while (x) {
                ee[pe++] = (uint16_t)(base + __builtin_ctzll(x));
                x &= x - 1;
            }
        }
        __syncthreads();
        uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
        for (uint32_t i = tid; i < r; i += 256) {
            uint32_t s0 = ss[i], e0 = ee[i];
            d32[i] = s0 | ((e0 - s0) << 16);
        }
    }
    if (tid == 0) {
        so.res_card[slot] = c;
        so.res_type[slot] = type;
        so.res_size[slot] = type == RG_ARRAY ? c : type == RG_BITSET ? 1024u : r;
    }
    return c;
}

// count-only variant: population count of the result words, summed over the workgroup
__device__ inline uint32_t count_words(const uint64_t (&w)[4], WgShared& sh) {
    uint32_t ct = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) ct += __popcll(w[j]);
    return (uint32_t)block_sum_u64(ct, sh.tmp64);
}

}  // namespace rg
