// rg_pool.hip - device-side pool utilities: recount (cardinalities and
// payload bounds from the payload), validation against the container rules
// of Section 1 (P1 form, sorted keys, maximal runs), and the per-bitmap
// fingerprint used to compare large results.
#include "rg_internal.h"

namespace rg {

__device__ __forceinline__ uint32_t bitmap_of(const uint64_t* bm_begin, uint32_t n_bitmaps, uint64_t c) {
    uint32_t lo = 0, hi = n_bitmaps;  // largest b with bm_begin[b] <= c
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (bm_begin[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ recount
__global__ void __launch_bounds__(256) k_recount(rg_pool p) {
    const uint32_t lane = lane_id();
    const uint64_t i = wave_index();
    if (i >= p.n_containers || i < uniform64(p.bm_begin[0])) return;  // a window may start past 0
    const uint8_t type = (uint8_t)uniform(p.types[i]);
    const uint32_t size = uniform(p.size[i]);
    const uint8_t* pl = p.payload + uniform64(p.off[i]);
    uint32_t c = 0;
    if (type == RG_ARRAY) {
        c = size;
    } else if (type == RG_BITSET) {
        const uint64_t* w = reinterpret_cast<const uint64_t*>(pl);
        for (uint32_t k = lane; k < 1024; k += 64) c += __popcll(w[k]);
        c = wave_sum_u32(c);
    } else {
        const uint32_t* rp = reinterpret_cast<const uint32_t*>(pl);
        for (uint32_t k = lane; k < size; k += 64) c += (rp[k] >> 16) + 1;
        c = wave_sum_u32(c);
    }
    if (lane == 0) {
        const_cast<uint32_t*>(p.card)[i] = c;
        uint32_t b = bitmap_of(p.bm_begin, p.n_bitmaps, i);
        atomicAdd(reinterpret_cast<unsigned long long*>(const_cast<uint64_t*>(p.bm_card) + b),
                  (unsigned long long)c);
        atomicAdd(reinterpret_cast<unsigned long long*>(const_cast<uint64_t*>(p.bm_wbytes) + b),
                  (unsigned long long)wbytes_of(c));
    }
}

void launch_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t st);

void launch_pool_recount(const rg_pool& p, hipStream_t st) {
    launch_fill_u64(const_cast<uint64_t*>(p.bm_card), 0, p.n_bitmaps, st);
    launch_fill_u64(const_cast<uint64_t*>(p.bm_wbytes), 0, p.n_bitmaps, st);
    if (!p.n_containers) return;
    hipLaunchKernelGGL(k_recount, dim3((uint32_t)((p.n_containers + 3) / 4)), dim3(256), 0, st, p);
}

// ------------------------------------------------------------------ dense pools
// Metadata of a pool whose payload is n_bitmaps x n_keys bitset containers laid
// out [bitmap][key][1024 words]: bitmap b holds keys 0..n_keys-1, container
// i = b * n_keys + k at byte offset 8192 i. Cardinalities come from the recount.
__global__ void k_dense_init(rg_pool p, uint32_t n_keys) {
    const uint64_t n = p.n_containers;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (i % n_keys == 0) const_cast<uint64_t*>(p.bm_begin)[i / n_keys] = i;
        if (i == n) break;
        const_cast<uint16_t*>(p.keys)[i] = (uint16_t)(i % n_keys);
        const_cast<uint8_t*>(p.types)[i] = RG_BITSET;
        const_cast<uint32_t*>(p.size)[i] = 1024;
        const_cast<uint64_t*>(p.off)[i] = i * 8192ull;
    }
}

void launch_pool_dense_init(const rg_pool& p, uint32_t n_keys, hipStream_t st) {
    uint64_t g = (p.n_containers + 1 + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_dense_init, dim3((uint32_t)g), dim3(256), 0, st, p, n_keys);
    launch_pool_recount(p, st);
}

// ------------------------------------------------------------------ validate
// p1 = 0 checks only that every container is a well-formed set (arrays of
// any length strictly increasing, runs sorted and disjoint but possibly
// touching, cardinalities right); p1 = 1 also requires the P1 form.
__global__ void __launch_bounds__(256) k_validate(rg_pool p, unsigned long long* bad, int p1) {
    const uint32_t lane = lane_id();
    const uint64_t i = wave_index();
    if (i >= p.n_containers || i < uniform64(p.bm_begin[0])) return;  // a window may start past 0
    const uint8_t type = (uint8_t)uniform(p.types[i]);
    const uint32_t size = uniform(p.size[i]), card = uniform(p.card[i]);
    const uint64_t off = uniform64(p.off[i]);
    bool ok = type >= RG_ARRAY && type <= RG_RUN && (off & 15) == 0 && card >= 1 && card <= 65536;
    if (ok) {
        uint64_t bytes = payload_bytes_of(type, size);
        if (type == RG_ARRAY) ok = size >= 1 && size <= (p1 ? 4096u : 65536u) && size == card;
        if (type == RG_BITSET) ok = size == 1024;
        if (type == RG_RUN) ok = size >= 1 && size <= (p1 ? 32768u : 65536u);
        ok = ok && off + ((bytes + 15) & ~15ull) <= p.payload_bytes;
    }
    const uint32_t b = bitmap_of(p.bm_begin, p.n_bitmaps, i);
    if (ok && i > p.bm_begin[b]) ok = p.keys[i - 1] < p.keys[i];
    uint32_t c = 0, r = 0;
    bool lok = true;
    if (ok) {
        const uint8_t* pl = p.payload + off;
        if (type == RG_ARRAY) {
            const uint16_t* v = reinterpret_cast<const uint16_t*>(pl);
            for (uint32_t k = lane; k < size; k += 64) {
                if (k > 0 && !(v[k - 1] < v[k])) lok = false;
                if (k == 0 || v[k] != v[k - 1] + 1) r++;
            }
            c = lane == 0 ? size : 0;  // summed over the wave below
        } else if (type == RG_BITSET) {
            const uint64_t* w = reinterpret_cast<const uint64_t*>(pl);
            for (uint32_t k = lane; k < 1024; k += 64) {
                uint64_t x = w[k];
                uint64_t below = k > 0 ? (w[k - 1] >> 63) : 0;
                c += __popcll(x);
                r += __popcll(x & ~((x << 1) | below));
            }
        } else {
            const uint32_t* rp = reinterpret_cast<const uint32_t*>(pl);
            for (uint32_t k = lane; k < size; k += 64) {
                uint32_t s = rp[k] & 0xFFFFu, l = rp[k] >> 16;
                if (s + l > 65535u) lok = false;
                if (k > 0) {
                    uint32_t ps = rp[k - 1] & 0xFFFFu, pl2 = rp[k - 1] >> 16;
                    // sorted and disjoint; P1 also forbids touching runs
                    if (!(s > ps + pl2 + (p1 ? 1u : 0u))) lok = false;
                }
                c += l + 1;
            }
            r = size;
        }
    }
    c = wave_sum_u32(c);
    uint32_t rr = wave_sum_u32(r);
    bool all_ok = __ballot(!lok) == 0;
    if (lane == 0) {
        if (type == RG_RUN) rr = size;
        bool good = ok && all_ok && c == card && (!p1 || p1_type(c, rr) == type);
        if (!good) atomicAdd(bad, 1ull);
    }
}

__global__ void k_validate_bitmaps(rg_pool p, unsigned long long* bad) {
    uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > p.n_bitmaps) return;
    if (b == p.n_bitmaps) {
        if (p.bm_begin[0] != 0 || p.bm_begin[p.n_bitmaps] != p.n_containers) atomicAdd(bad, 1ull);
        return;
    }
    uint64_t s = p.bm_begin[b], e = p.bm_begin[b + 1];
    if (e < s || e > p.n_containers) {
        atomicAdd(bad, 1ull);
        return;
    }
    uint64_t tc = 0, tw = 0;
    for (uint64_t i = s; i < e; ++i) {
        tc += p.card[i];
        tw += wbytes_of(p.card[i]);
    }
    if (tc != p.bm_card[b] || tw != p.bm_wbytes[b]) atomicAdd(bad, 1ull);
}

void launch_pool_validate(const rg_pool& p, uint64_t* d_bad, bool p1, hipStream_t st) {
    launch_fill_u64(d_bad, 0, 1, st);
    hipLaunchKernelGGL(k_validate_bitmaps, dim3((p.n_bitmaps + 1 + 255) / 256), dim3(256), 0, st, p,
                       reinterpret_cast<unsigned long long*>(d_bad));
    if (p.n_containers)
        hipLaunchKernelGGL(k_validate, dim3((uint32_t)((p.n_containers + 3) / 4)), dim3(256), 0, st, p,
                           reinterpret_cast<unsigned long long*>(d_bad), (int)p1);
}

// ------------------------------------------------------------------ digest
__device__ __forceinline__ uint64_t dmix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_digest(rg_pool p, const uint64_t* d_n, uint64_t* digest) {
    const uint32_t lane = lane_id();
    const uint64_t i = wave_index();
    const uint64_t n = d_n ? uniform64(*d_n) : p.n_containers;  // d_n: live count (<= p.n_containers)
    if (i >= n || i >= p.n_containers || i < uniform64(p.bm_begin[0])) return;
    const uint8_t type = (uint8_t)uniform(p.types[i]);
    const uint32_t size = uniform(p.size[i]), card = uniform(p.card[i]);
    const uint32_t key = uniform(p.keys[i]);
    const uint8_t* pl = p.payload + uniform64(p.off[i]);
    uint32_t npl = type == RG_ARRAY ? (size + 3) / 4 : type == RG_BITSET ? 1024 : (size + 1) / 2;
    uint64_t sum = 0;
    for (uint32_t k = lane; k < npl + 2; k += 64) {
        uint64_t w;
        if (k == 0) {
            w = (uint64_t)key | ((uint64_t)type << 16) | ((uint64_t)card << 32);
        } else if (k == 1) {
            w = size;
        } else {
            uint32_t j = k - 2;
            if (type == RG_ARRAY) {
                const uint16_t* v = reinterpret_cast<const uint16_t*>(pl);
                w = 0;
                for (uint32_t q = 0; q < 4; ++q)
                    if (4 * j + q < size) w |= (uint64_t)v[4 * j + q] << (16 * q);
            } else if (type == RG_BITSET) {
                w = reinterpret_cast<const uint64_t*>(pl)[j];
            } else {
                const uint32_t* rp = reinterpret_cast<const uint32_t*>(pl);
                w = rp[2 * j];
                if (2 * j + 1 < size) w |= (uint64_t)rp[2 * j + 1] << 32;
            }
        }
        sum += dmix64(w + ((uint64_t)key * (1ull << 20) + k + 1) * 0x9E3779B97F4A7C15ULL);
    }
    sum = wave_sum_u64(sum);
    if (lane == 0) {
        uint32_t b = bitmap_of(p.bm_begin, p.n_bitmaps, i);
        atomicAdd(reinterpret_cast<unsigned long long*>(digest + b), (unsigned long long)sum);
    }
}

void launch_pool_digest(const rg_pool& p, uint64_t* d_digest, hipStream_t st) {
    launch_pool_digest_n(p, nullptr, d_digest, st);
}

void launch_pool_digest_n(const rg_pool& p, const uint64_t* d_n, uint64_t* d_digest, hipStream_t st) {
    launch_fill_u64(d_digest, 0, p.n_bitmaps, st);
    if (!p.n_containers) return;
    hipLaunchKernelGGL(k_digest, dim3((uint32_t)((p.n_containers + 3) / 4)), dim3(256), 0, st, p, d_n, d_digest);
}

// ------------------------------------------------------------------ packed metadata
__global__ void k_pack_meta(PoolView P, uint64_t n, u32x4* out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t off = P.off[i];
    const uint8_t type = P.types[i];
    const uint32_t card = P.card[i], size = P.size[i];
    uint64_t data = off;
    uint32_t inl = 0;
    if (type == RG_ARRAY && card <= META_INLINE_MAX) {
        const uint16_t* v = reinterpret_cast<const uint16_t*>(P.payload + off);
        data = 0;
        for (uint32_t k = 0; k < card; ++k) data |= (uint64_t)v[k] << (16 * k);
        inl = 1;
    }
    u32x4 r;
    r.x = (uint32_t)data;
    r.y = (uint32_t)(data >> 32);
    r.z = card;
    r.w = (size & 0x1FFFFFu) | (inl << 21) | ((uint32_t)type << 24);
    out[i] = r;
}

void launch_pack_meta(const PoolView& P, uint64_t n, u32x4* out, hipStream_t st) {
    if (n) hipLaunchKernelGGL(k_pack_meta, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, P, n, out);
}

// ------------------------------------------------------------------ key index
// One workgroup per bitmap: the presence bit of every key, then each word's
// rank (keys in the words before it) by a workgroup prefix sum of popcounts.
__global__ void __launch_bounds__(256) k_key_index(PoolView P, uint8_t* out) {
    __shared__ uint64_t w[KIDX_WORDS];
    __shared__ uint32_t tmp[8];
    const uint32_t b = blockIdx.x, tid = threadIdx.x;
    for (uint32_t i = tid; i < KIDX_WORDS; i += 256) w[i] = 0;
    __syncthreads();
    const uint64_t s = P.bm_begin[b], e = P.bm_begin[b + 1];
    for (uint64_t i = s + tid; i < e; i += 256) {
        const uint32_t k = P.keys[i];
        atomicOr(reinterpret_cast<unsigned long long*>(&w[k >> 6]), 1ull << (k & 63));
    }
    __syncthreads();
    uint64_t x[4];
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        x[j] = w[4 * tid + j];
        c += __popcll(x[j]);
    }
    uint32_t tot;
    uint32_t r = block_excl_scan_u32(c, tmp, &tot);
    uint8_t* o = out + (uint64_t)b * RG_KEY_INDEX_BYTES;
    uint64_t* ow = reinterpret_cast<uint64_t*>(o);
    uint16_t* orank = reinterpret_cast<uint16_t*>(o + 8 * KIDX_WORDS);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        ow[4 * tid + j] = x[j];
        orank[4 * tid + j] = (uint16_t)r;
        r += __popcll(x[j]);
    }
}

void launch_key_index(const PoolView& P, uint32_t n_bitmaps, uint8_t* out, hipStream_t st) {
    if (n_bitmaps) hipLaunchKernelGGL(k_key_index, dim3(n_bitmaps), dim3(256), 0, st, P, out);
}

}  // namespace rg
