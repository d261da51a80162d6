// rg_build_host.cpp - host-side construction of a pool from sorted values:
// values are cut into 2^16-value chunks by their high 16 bits (Section 1),
// each non-empty chunk becomes one container in its P1 form (least memory
// under the Section 1 size rules), payloads 16-byte aligned and zero padded.
#include <string.h>

#include <vector>

#include "rg_internal.h"

using namespace rg;

namespace {

struct ChunkInfo {
    uint32_t key, c, r;
    uint64_t first;
};

// visits the chunks of one bitmap; returns false if values are not strictly increasing
template <class F>
bool for_each_chunk(const uint32_t* v, uint64_t n, F&& f) {
    uint64_t i = 0;
    while (i < n) {
        uint32_t key = v[i] >> 16;
        uint64_t j = i;
        uint32_t r = 0;
        while (j < n && (v[j] >> 16) == key) {
            if (j > i && v[j] <= v[j - 1]) return false;
            if (j == i || v[j] != v[j - 1] + 1) r++;
            j++;
        }
        if (j < n && v[j] <= v[j - 1]) return false;
        f(ChunkInfo{key, (uint32_t)(j - i), r, i});
        i = j;
    }
    return true;
}

}  // namespace

extern "C" rg_status rg_pool_measure_host(const uint32_t* values, const uint64_t* offsets, uint32_t n_bitmaps,
                                          uint64_t* n_containers, uint64_t* payload_bytes) {
    if (!offsets || !n_containers || !payload_bytes || (!values && n_bitmaps && offsets[n_bitmaps]))
        return RG_EINVAL;
    uint64_t nc = 0, pb = 0;
    for (uint32_t b = 0; b < n_bitmaps; ++b) {
        if (offsets[b + 1] < offsets[b]) return RG_EINVAL;
        bool ok = for_each_chunk(values + offsets[b], offsets[b + 1] - offsets[b], [&](const ChunkInfo& ci) {
            uint8_t t = p1_type(ci.c, ci.r);
            uint32_t size = t == RG_ARRAY ? ci.c : t == RG_BITSET ? 1024 : ci.r;
            nc++;
            pb += (payload_bytes_of(t, size) + 15) & ~15u;
        });
        if (!ok) return RG_EINVAL;
    }
    *n_containers = nc;
    *payload_bytes = pb;
    return RG_OK;
}

extern "C" rg_status rg_pool_build_host(const uint32_t* values, const uint64_t* offsets, uint32_t n_bitmaps,
                                        uint64_t* bm_begin, uint16_t* keys, uint8_t* types, uint32_t* card,
                                        uint32_t* size, uint64_t* off, uint8_t* payload, uint64_t* bm_card,
                                        uint64_t* bm_wbytes) {
    if (!offsets || !bm_begin) return RG_EINVAL;
    uint64_t k = 0, pb = 0;
    for (uint32_t b = 0; b < n_bitmaps; ++b) {
        bm_begin[b] = k;
        uint64_t tc = 0, tw = 0;
        const uint32_t* v = values + offsets[b];
        bool ok = for_each_chunk(v, offsets[b + 1] - offsets[b], [&](const ChunkInfo& ci) {
            uint8_t t = p1_type(ci.c, ci.r);
            uint32_t sz = t == RG_ARRAY ? ci.c : t == RG_BITSET ? 1024 : ci.r;
            uint32_t bytes = payload_bytes_of(t, sz), padded = (bytes + 15) & ~15u;
            uint8_t* dst = payload + pb;
            memset(dst, 0, padded);
            const uint32_t* cv = v + ci.first;
            if (t == RG_ARRAY) {
                uint16_t* d = reinterpret_cast<uint16_t*>(dst);
                for (uint32_t q = 0; q < ci.c; ++q) d[q] = (uint16_t)(cv[q] & 0xFFFFu);
            } else if (t == RG_BITSET) {
                uint64_t* d = reinterpret_cast<uint64_t*>(dst);
                for (uint32_t q = 0; q < ci.c; ++q) {
                    uint32_t x = cv[q] & 0xFFFFu;
                    d[x >> 6] |= 1ull << (x & 63);
                }
            } else {
                uint32_t* d = reinterpret_cast<uint32_t*>(dst);
                uint32_t q = 0, ri = 0;
                while (q < ci.c) {
                    uint32_t e = q;
                    while (e + 1 < ci.c && cv[e + 1] == cv[e] + 1) e++;
                    uint32_t s = cv[q] & 0xFFFFu;
                    d[ri++] = s | ((e - q) << 16);
                    q = e + 1;
                }
            }
            keys[k] = (uint16_t)ci.key;
            types[k] = t;
            card[k] = ci.c;
            size[k] = sz;
            off[k] = pb;
            k++;
            pb += padded;
            tc += ci.c;
            tw += wbytes_of(ci.c);
        });
        if (!ok) return RG_EINVAL;
        bm_card[b] = tc;
        if (bm_wbytes) bm_wbytes[b] = tw;
    }
    bm_begin[n_bitmaps] = k;
    return RG_OK;
}
