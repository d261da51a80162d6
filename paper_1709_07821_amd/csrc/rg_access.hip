// rg_access.hip - access to single values of device-resident bitmaps.
//
// Membership (Section 1: a value's 16 high bits select the container by a
// binary search over the sorted keys; then the container is searched: a
// binary search in an array, a bit test in a bitset (Section 3.2 addressing),
// a search of the run starts in a run container).
//
// Export to sorted uint32 values (Section 3.1: a bitset's set bits become an
// array by counting the bits of each word and extracting their positions;
// Section 5.5 iterates over all values this way). One wave per container:
// bitsets are read 64 words per round (one per lane), each lane's bit count
// is scanned across the wave so that a round's values land in one contiguous
// range; arrays are widened; runs are expanded 64 runs at a time with the
// wave's prefix sum of their lengths in LDS.
#include "rg_access.h"

namespace rg {

// ------------------------------------------------------------------ membership

__device__ __forceinline__ bool contains_one(const rg_pool& P, uint32_t b, uint32_t v) {
    const uint64_t c0 = P.bm_begin[b], c1 = P.bm_begin[b + 1];
    const uint16_t key = (uint16_t)(v >> 16), low = (uint16_t)(v & 0xFFFFu);
    // lower bound of the key among the bitmap's keys
    uint64_t lo = c0, hi = c1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (P.keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    if (lo == c1 || P.keys[lo] != key) return false;
    uint8_t type;
    uint32_t size;
    uint64_t off;
    if (P.meta) {
        // one packed record: {data lo, data hi, card, size | inline << 21 | type << 24}
        const u32x4 r = reinterpret_cast<const u32x4*>(P.meta)[lo];
        type = (uint8_t)(r.w >> 24);
        size = r.w & 0x1FFFFFu;
        if ((r.w >> 21) & 1u) {  // an array of at most four values held in the record
            const uint64_t d = (uint64_t)r.x | ((uint64_t)r.y << 32);
            for (uint32_t i = 0; i < size; ++i)
                if ((uint16_t)(d >> (16 * i)) == low) return true;
            return false;
        }
        off = (uint64_t)r.x | ((uint64_t)r.y << 32);
    } else {
        type = P.types[lo];
        size = P.size[lo];
        off = P.off[lo];
    }
    const uint8_t* pl = P.payload + off;
    if (type == RG_BITSET) {
        const uint64_t w = reinterpret_cast<const uint64_t*>(pl)[low >> 6];
        return (w >> (low & 63)) & 1ull;
    }
    if (type == RG_ARRAY) {
        const uint16_t* a = reinterpret_cast<const uint16_t*>(pl);
        uint32_t l = 0, h = size;
        while (l < h) {
            const uint32_t m = (l + h) >> 1;
            if (a[m] < low) l = m + 1;
            else h = m;
        }
        return l < size && a[l] == low;
    }
    // run: the last run starting at or below low covers it if low <= start + length - 1
    const uint32_t* r = reinterpret_cast<const uint32_t*>(pl);
    uint32_t l = 0, h = size;  // first run whose start is above low
    while (l < h) {
        const uint32_t m = (l + h) >> 1;
        if ((r[m] & 0xFFFFu) <= low) l = m + 1;
        else h = m;
    }
    if (l == 0) return false;
    const uint32_t run = r[l - 1];
    return (uint32_t)low <= (run & 0xFFFFu) + (run >> 16);
}

__global__ void __launch_bounds__(256) k_contains(rg_pool P, const uint32_t* ids, const uint32_t* values, uint64_t n,
                                                  uint8_t* out, uint32_t* err) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = ids[i];
        if (b >= P.n_bitmaps) {
            atomicOr(err, 1u);
            out[i] = 0;
            continue;
        }
        out[i] = contains_one(P, b, values[i]) ? 1 : 0;
    }
}

void launch_contains(const rg_pool& P, const uint32_t* ids, const uint32_t* values, uint64_t n, uint8_t* out,
                     uint32_t* err, hipStream_t st) {
    if (!n) return;
    uint64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_contains, dim3((uint32_t)g), dim3(256), 0, st, P, ids, values, n, out, err);
}

// ------------------------------------------------------------------ export

__global__ void __launch_bounds__(256) k_export_range(rg_pool P, uint32_t b0, uint32_t n, uint64_t* range) {
    __shared__ uint64_t tmp[4];
    uint64_t s = 0;
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) s += P.bm_card[b0 + j];
    s = block_sum_u64(s, tmp);
    if (threadIdx.x == 0) {
        range[0] = P.bm_begin[b0];
        range[1] = P.bm_begin[b0 + n];
        range[2] = s;
    }
}

void launch_export_range(const rg_pool& P, uint32_t b0, uint32_t n, uint64_t* range, hipStream_t st) {
    hipLaunchKernelGGL(k_export_range, dim3(1), dim3(256), 0, st, P, b0, n, range);
}

__global__ void k_export_offsets(rg_pool P, uint32_t b0, uint32_t n, uint64_t c0, const uint64_t* val_off,
                                 uint64_t total, uint64_t* offsets) {
    const uint64_t nc = P.bm_begin[b0 + n] - c0;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= n; j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t idx = P.bm_begin[b0 + j] - c0;
        offsets[j] = idx < nc ? val_off[idx] : total;
    }
}

void launch_export_offsets(const rg_pool& P, uint32_t b0, uint32_t n, uint64_t c0, const uint64_t* val_off,
                           uint64_t total, uint64_t* offsets, hipStream_t st) {
    uint64_t g = ((uint64_t)n + 1 + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_export_offsets, dim3((uint32_t)g), dim3(256), 0, st, P, b0, n, c0, val_off, total, offsets);
}

__global__ void __launch_bounds__(256) k_export_values(rg_pool P, uint64_t c0, uint64_t c1, const uint64_t* val_off,
                                                       uint32_t* values, uint64_t cap) {
    __shared__ uint32_t run_end[4][64];    // inclusive prefix sum of run lengths, per wave
    __shared__ uint32_t run_start[4][64];  // run starts
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
    const uint64_t nwaves = (uint64_t)gridDim.x * 4;
    for (uint64_t i = c0 + wave_index(); i < c1; i += nwaves) {
        const uint8_t type = (uint8_t)uniform(P.types[i]);
        const uint32_t size = uniform(P.size[i]);
        const uint32_t hi = (uint32_t)uniform(P.keys[i]) << 16;
        const uint8_t* pl = P.payload + uniform64(P.off[i]);
        const uint64_t o = uniform64(val_off[i - c0]);
        uint32_t* out = values + o;
        // the container's range of the output is card[i] values, and the
        // output holds cap values: a pool inconsistent with its cardinalities
        // gives wrong values but no write outside the output
        const uint32_t cd = uniform(P.card[i]);
        const uint32_t lim = o >= cap ? 0u : (cap - o < cd ? (uint32_t)(cap - o) : cd);
        if (type == RG_ARRAY) {
            const uint16_t* a = reinterpret_cast<const uint16_t*>(pl);
            const uint32_t n = size < lim ? size : lim;
            for (uint32_t k = lane; k < n; k += 64) out[k] = hi | a[k];
        } else if (type == RG_BITSET) {
            const uint64_t* w = reinterpret_cast<const uint64_t*>(pl);
            uint32_t base = 0;
            for (uint32_t r = 0; r < 1024; r += 64) {
                uint64_t x = w[r + lane];
                const uint32_t pc = (uint32_t)__popcll(x);
                const uint32_t incl = wave_incl_scan_u32(pc);
                uint32_t pos = base + incl - pc;
                const uint32_t bit0 = (r + lane) << 6;
                while (x && pos < lim) {
                    out[pos++] = hi | (bit0 + (uint32_t)__builtin_ctzll(x));
                    x &= x - 1;
                }
                base += uniform(__shfl(incl, 63));
            }
        } else {
            const uint32_t* rp = reinterpret_cast<const uint32_t*>(pl);
            uint32_t base = 0;
            for (uint32_t r0 = 0; r0 < size; r0 += 64) {
                const uint32_t nr = size - r0 < 64 ? size - r0 : 64;
                const uint32_t pr = lane < nr ? rp[r0 + lane] : 0u;
                const uint32_t len = lane < nr ? (pr >> 16) + 1 : 0u;
                const uint32_t incl = wave_incl_scan_u32(len);
                run_end[wid][lane] = incl;
                run_start[wid][lane] = pr & 0xFFFFu;
                const uint32_t total = uniform(__shfl(incl, 63));
                __builtin_amdgcn_wave_barrier();
                for (uint32_t p = lane; p < total; p += 64) {
                    // the run holding position p: the first whose inclusive end exceeds p
                    uint32_t l = 0, h = nr - 1;
                    while (l < h) {
                        const uint32_t m = (l + h) >> 1;
                        if (run_end[wid][m] <= p) l = m + 1;
                        else h = m;
                    }
                    const uint32_t before = l ? run_end[wid][l - 1] : 0u;
                    if (base + p < lim) out[base + p] = hi | (run_start[wid][l] + (p - before));
                }
                __builtin_amdgcn_wave_barrier();
                base += total;
            }
        }
    }
}

void launch_export_values(const rg_pool& P, uint64_t c0, uint64_t c1, const uint64_t* val_off, uint32_t* values,
                          uint64_t cap, hipStream_t st) {
    if (c1 <= c0) return;
    uint64_t g = (c1 - c0 + 3) / 4;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_export_values, dim3((uint32_t)g), dim3(256), 0, st, P, c0, c1, val_off, values, cap);
}

}  // namespace rg
