// Host pool builder under AddressSanitizer / UndefinedBehaviorSanitizer:
// builds pools from many sets (type boundaries, chunk edges, random
// mixtures), decodes every container back with a reader written here, and
// checks values, cardinalities, sizes, 16-byte alignment and the
// per-bitmap totals. Exit status 0 when every check holds.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <set>
#include <vector>

#include "../../include/roaring_gpu.h"

static uint64_t state = 0x1709078215ull;
static uint64_t next_u64() {  // xorshift64*, only to vary the test sets
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return state * 2685821657736338717ull;
}

static std::vector<uint32_t> decode(const std::vector<uint8_t>& pl, uint8_t type, uint32_t size, uint64_t off,
                                    uint16_t key) {
    std::vector<uint32_t> v;
    const uint32_t hi = (uint32_t)key << 16;
    if (type == RG_ARRAY) {
        for (uint32_t i = 0; i < size; ++i) {
            uint16_t x;
            memcpy(&x, &pl[off + 2 * i], 2);
            v.push_back(hi | x);
        }
    } else if (type == RG_BITSET) {
        for (uint32_t w = 0; w < 1024; ++w) {
            uint64_t x;
            memcpy(&x, &pl[off + 8 * w], 8);
            for (int b = 0; b < 64; ++b)
                if ((x >> b) & 1) v.push_back(hi | (w * 64 + b));
        }
    } else {
        for (uint32_t i = 0; i < size; ++i) {
            uint16_t s, l;
            memcpy(&s, &pl[off + 4 * i], 2);
            memcpy(&l, &pl[off + 4 * i + 2], 2);
            for (uint32_t x = s; x <= (uint32_t)s + l; ++x) v.push_back(hi | x);
        }
    }
    return v;
}

int main() {
    std::vector<std::vector<uint32_t>> sets;
    sets.push_back({});
    std::vector<uint32_t> full;
    for (uint32_t x = 0; x < 65536; ++x) full.push_back(x);
    sets.push_back(full);
    sets.push_back({0, 65535, 65536, 131071, 0xFFFFFFFFu});
    for (int n : {1, 2, 3, 4095, 4096, 4097}) {
        std::vector<uint32_t> v;
        for (int i = 0; i < n; ++i) v.push_back(5 * 65536 + 2 * i);
        sets.push_back(v);
    }
    for (int rep = 0; rep < 40; ++rep) {
        std::set<uint32_t> s;
        const int kind = rep % 4;
        const uint32_t n = (uint32_t)(next_u64() % 60000);
        for (uint32_t i = 0; i < n; ++i) {
            uint32_t x = (uint32_t)next_u64();
            if (kind == 1) x &= 0x3FFFFu;                               // dense in 4 chunks
            if (kind == 2) x = (x & 0xFFF00000u) | (i * 3 % 4000);      // short runs of values
            s.insert(x);
        }
        if (kind == 3) {
            const uint32_t base = (uint32_t)(next_u64() & 0xFFFF0000u);
            const uint32_t start = (uint32_t)(next_u64() % 30000), len = (uint32_t)(next_u64() % 30000);
            for (uint32_t x = start; x < start + len; ++x) s.insert(base | x);
        }
        sets.emplace_back(s.begin(), s.end());
    }
    std::vector<uint32_t> values;
    std::vector<uint64_t> offsets{0};
    for (auto& s : sets) {
        values.insert(values.end(), s.begin(), s.end());
        offsets.push_back(values.size());
    }
    const uint32_t nb = (uint32_t)sets.size();
    uint64_t nc = 0, pb = 0;
    if (rg_pool_measure_host(values.data(), offsets.data(), nb, &nc, &pb) != RG_OK) return 10;
    std::vector<uint64_t> bm_begin(nb + 1), off(nc), bm_card(nb), bm_wbytes(nb);
    std::vector<uint16_t> keys(nc);
    std::vector<uint8_t> types(nc), payload(pb);
    std::vector<uint32_t> card(nc), size(nc);
    if (rg_pool_build_host(values.data(), offsets.data(), nb, bm_begin.data(), keys.data(), types.data(), card.data(),
                           size.data(), off.data(), payload.data(), bm_card.data(), bm_wbytes.data()) != RG_OK)
        return 11;
    if (bm_begin[0] != 0 || bm_begin[nb] != nc) return 12;
    for (uint32_t b = 0; b < nb; ++b) {
        std::vector<uint32_t> got;
        uint64_t tc = 0, tw = 0;
        for (uint64_t i = bm_begin[b]; i < bm_begin[b + 1]; ++i) {
            if (off[i] % 16) return 13;
            if (i > bm_begin[b] && keys[i] <= keys[i - 1]) return 14;
            std::vector<uint32_t> v = decode(payload, types[i], size[i], off[i], keys[i]);
            if (v.size() != card[i] || v.empty()) return 15;
            got.insert(got.end(), v.begin(), v.end());
            tc += card[i];
            const uint64_t w = std::min<uint64_t>(8192, 2ull * card[i]);
            tw += (w + 15) & ~15ull;
        }
        if (got != sets[b]) return 16;
        if (tc != bm_card[b] || tw != bm_wbytes[b]) return 17;
    }
    // unsorted and repeated values are refused
    std::vector<uint32_t> bad{5, 3};
    std::vector<uint64_t> bo{0, 2};
    if (rg_pool_measure_host(bad.data(), bo.data(), 1, &nc, &pb) == RG_OK) return 18;
    printf("pool builder: %u bitmaps, all checks passed\n", nb);
    return 0;
}
