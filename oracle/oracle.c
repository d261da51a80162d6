/*
 * oracle.c - TEST INFRASTRUCTURE ONLY. The plain, slow, obviously correct CPU
 * definition of what the GPU library computes. Only tests/, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the GPU library never
 * does, and this file shares no code with it.
 *
 * Paper: Lemire et al., "Roaring Bitmaps: Implementation of an Optimized
 * Software Library" (arXiv:1709.07821).
 *
 * Representation: a set is a strictly increasing list of uint32 values
 * (the universe [0, 2^32) of Section 1). Every operation here is the
 * textbook two-pointer merge over two sorted lists - the same computation
 * as the C++ standard set algorithms that Section 5.1 (Software) uses for
 * its sorted-vector baseline. Nothing is blocked, fused or reordered.
 *
 * Container view (Section 1: the 32-bit universe cut into 2^16-value chunks,
 * and the container-size rules): values are grouped by their 16 most significant
 * bits (the key); each non-empty group is one container holding the 16
 * least significant bits. Empty groups have no container (Section 2.2,
 * where Roaring is said to omit empty containers).
 *
 * Container type (Section 1 size rules; the type is chosen for least memory):
 * policy P1 - run if (c <= 4096 ? 2r < c : r <= 2047); else array if
 * c <= 4096; else bitset. Here c is the number of values in the chunk and
 * r the number of maximal runs of consecutive values.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORA_AND = 0, ORA_OR = 1, ORA_XOR = 2, ORA_ANDNOT = 3 };
enum { ORA_ARRAY = 1, ORA_BITSET = 2, ORA_RUN = 3 };

/* ---------------------------------------------------------------------------
 * Two-way set operations (Section 1: intersection, union, difference
 * A \ B, symmetric difference (A \ B) u (B \ A)). `out` may be NULL, in which
 * case only the size of the result is returned (Section 5.9, Fast Counts).
 * ------------------------------------------------------------------------- */

uint64_t ora_and(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out) {
    uint64_t i = 0, j = 0, n = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) {
            i++;
        } else if (b[j] < a[i]) {
            j++;
        } else {
            if (out) out[n] = a[i];
            n++;
            i++;
            j++;
        }
    }
    return n;
}

uint64_t ora_or(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out) {
    uint64_t i = 0, j = 0, n = 0;
    while (i < na || j < nb) {
        uint32_t v;
        if (j >= nb || (i < na && a[i] < b[j])) {
            v = a[i++];
        } else if (i >= na || b[j] < a[i]) {
            v = b[j++];
        } else {
            v = a[i];
            i++;
            j++;
        }
        if (out) out[n] = v;
        n++;
    }
    return n;
}

uint64_t ora_xor(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out) {
    uint64_t i = 0, j = 0, n = 0;
    while (i < na || j < nb) {
        if (j >= nb || (i < na && a[i] < b[j])) {
            if (out) out[n] = a[i];
            n++;
            i++;
        } else if (i >= na || b[j] < a[i]) {
            if (out) out[n] = b[j];
            n++;
            j++;
        } else { /* present in both: in neither A \ B nor B \ A */
            i++;
            j++;
        }
    }
    return n;
}

uint64_t ora_andnot(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out) {
    uint64_t i = 0, j = 0, n = 0;
    while (i < na) {
        if (j >= nb || a[i] < b[j]) {
            if (out) out[n] = a[i];
            n++;
            i++;
        } else if (b[j] < a[i]) {
            j++;
        } else {
            i++;
            j++;
        }
    }
    return n;
}

uint64_t ora_op(int op, const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out) {
    switch (op) {
    case ORA_AND: return ora_and(a, na, b, nb, out);
    case ORA_OR: return ora_or(a, na, b, nb, out);
    case ORA_XOR: return ora_xor(a, na, b, nb, out);
    case ORA_ANDNOT: return ora_andnot(a, na, b, nb, out);
    default: return UINT64_MAX;
    }
}

/* Jaccard index |A n B| / |A u B| (Section 5.9, Fast Counts), as one
 * binary64 division of the two exact counts. Both sets empty: 1.0. */
double ora_jaccard(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb) {
    uint64_t inter = ora_and(a, na, b, nb, NULL);
    uint64_t uni = ora_or(a, na, b, nb, NULL);
    if (uni == 0) return 1.0;
    return (double)inter / (double)uni;
}

/* k-way AND/OR: left fold of the two-way operation over lists[0..k-1]
 * in the given order. `out` and `tmp` must each hold the largest possible
 * result (the sum of the list lengths for OR, the first length for AND). */
uint64_t ora_kway(int op, const uint32_t *const *lists, const uint64_t *lens, uint32_t k, uint32_t *out,
                  uint32_t *tmp) {
    if (k == 0) return 0;
    memcpy(out, lists[0], sizeof(uint32_t) * lens[0]);
    uint64_t n = lens[0];
    for (uint32_t i = 1; i < k; ++i) {
        uint64_t m = ora_op(op, out, n, lists[i], lens[i], tmp);
        memcpy(out, tmp, sizeof(uint32_t) * m);
        n = m;
    }
    return n;
}

/* ---------------------------------------------------------------------------
 * Container view
 * ------------------------------------------------------------------------- */

/* P1 container type for a chunk with c values forming r maximal runs */
int ora_type_of(uint32_t c, uint32_t r) {
    int run_ok = (c <= 4096) ? (2ull * r < c) : (r <= 2047);
    if (run_ok) return ORA_RUN;
    if (c <= 4096) return ORA_ARRAY;
    return ORA_BITSET;
}

uint64_t ora_container_count(const uint32_t *v, uint64_t n) {
    uint64_t k = 0;
    for (uint64_t i = 0; i < n; ++i)
        if (i == 0 || (v[i] >> 16) != (v[i - 1] >> 16)) k++;
    return k;
}

/* One entry per non-empty chunk, ascending key: key, P1 type, cardinality c,
 * number of maximal runs r, and the index of the chunk's first value in v. */
void ora_containers(const uint32_t *v, uint64_t n, uint16_t *keys, uint8_t *types, uint32_t *card,
                    uint32_t *runs, uint64_t *first) {
    uint64_t k = 0, i = 0;
    while (i < n) {
        uint32_t key = v[i] >> 16;
        uint64_t j = i;
        uint32_t r = 0;
        while (j < n && (v[j] >> 16) == key) {
            if (j == i || v[j] != v[j - 1] + 1) r++; /* a new maximal run starts here */
            j++;
        }
        uint32_t c = (uint32_t)(j - i);
        keys[k] = (uint16_t)key;
        types[k] = (uint8_t)ora_type_of(c, r);
        card[k] = c;
        runs[k] = r;
        if (first) first[k] = i;
        k++;
        i = j;
    }
}

/* ---------------------------------------------------------------------------
 * Canonical digest of a set's container form (a fingerprint used to compare
 * large results; it is not part of the method).
 *
 * Container serialised as 64-bit words:
 *   w0 = key | type << 16 | card << 32;  w1 = size (array: c, bitset: 1024,
 *   run: r); then the payload: array - the low 16 bits of each value, four per
 *   word, little-endian, zero padded; bitset - 1024 words, value x at bit
 *   (x & 63) of word (x >> 6); run - (start, length - 1) 16-bit pairs, two
 *   runs per word, zero padded.
 * digest = sum over containers and their words i of
 *   mix64(w_i + (key * 2^20 + i + 1) * 0x9E3779B97F4A7C15)  (mod 2^64),
 * mix64 being the SplitMix64 finalizer.
 * ------------------------------------------------------------------------- */

static uint64_t ora_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t term(uint32_t key, uint64_t i, uint64_t w) {
    return ora_mix64(w + ((uint64_t)key * (1ull << 20) + i + 1) * 0x9E3779B97F4A7C15ULL);
}

/* serialise the container whose values are v[0..c-1] (all sharing `key`)
 * into words; returns the number of words */
static uint64_t serialise(const uint32_t *v, uint32_t c, uint32_t r, int type, uint32_t key,
                          uint64_t *words) {
    uint64_t size = type == ORA_ARRAY ? c : type == ORA_BITSET ? 1024 : r;
    uint64_t nw = 2;
    words[0] = (uint64_t)key | ((uint64_t)type << 16) | ((uint64_t)c << 32);
    words[1] = size;
    if (type == ORA_ARRAY) {
        uint64_t np = (c + 3) / 4;
        memset(words + 2, 0, np * 8);
        for (uint32_t i = 0; i < c; ++i) words[2 + i / 4] |= (uint64_t)(v[i] & 0xFFFF) << (16 * (i % 4));
        nw += np;
    } else if (type == ORA_BITSET) {
        memset(words + 2, 0, 1024 * 8);
        for (uint32_t i = 0; i < c; ++i) {
            uint32_t x = v[i] & 0xFFFF;
            words[2 + (x >> 6)] |= 1ull << (x & 63);
        }
        nw += 1024;
    } else {
        uint64_t np = (r + 1) / 2;
        memset(words + 2, 0, np * 8);
        uint32_t ri = 0, i = 0;
        while (i < c) {
            uint32_t j = i;
            while (j + 1 < c && v[j + 1] == v[j] + 1) j++;
            uint64_t s = v[i] & 0xFFFF, l = (uint64_t)(j - i); /* run [s, s + l] */
            uint64_t pair = s | (l << 16);
            words[2 + ri / 2] |= pair << (32 * (ri % 2));
            ri++;
            i = j + 1;
        }
        nw += np;
    }
    return nw;
}

uint64_t ora_digest(const uint32_t *v, uint64_t n) {
    uint64_t *words = (uint64_t *)malloc(sizeof(uint64_t) * 2048);
    uint64_t d = 0, i = 0;
    while (i < n) {
        uint32_t key = v[i] >> 16;
        uint64_t j = i;
        uint32_t r = 0;
        while (j < n && (v[j] >> 16) == key) {
            if (j == i || v[j] != v[j - 1] + 1) r++;
            j++;
        }
        uint32_t c = (uint32_t)(j - i);
        int type = ora_type_of(c, r);
        uint64_t nw = serialise(v + i, c, r, type, key, words);
        for (uint64_t t = 0; t < nw; ++t) d += term(key, t, words[t]);
        i = j;
    }
    free(words);
    return d;
}

/* Per-pair loop over a collection: for each pair p, op(A[ia[p]], B[ib[p]]).
 * Writes the result size to card[p] (if card != NULL), the digest of the
 * result to digest[p] (if digest != NULL) and the Jaccard index to jac[p] (if
 * jac != NULL). Scratch `tmp` must hold the largest possible result. */
void ora_pairs(int op, const uint32_t *va, const uint64_t *oa, const uint32_t *vb, const uint64_t *ob,
               const uint32_t *ia, const uint32_t *ib, uint64_t n_pairs, uint64_t *card, uint64_t *digest,
               double *jac, uint32_t *tmp) {
    for (uint64_t p = 0; p < n_pairs; ++p) {
        const uint32_t *a = va + oa[ia[p]];
        uint64_t na = oa[ia[p] + 1] - oa[ia[p]];
        const uint32_t *b = vb + ob[ib[p]];
        uint64_t nb = ob[ib[p] + 1] - ob[ib[p]];
        if (card || digest) {
            uint64_t n = ora_op(op, a, na, b, nb, digest ? tmp : NULL);
            if (card) card[p] = n;
            if (digest) digest[p] = ora_digest(tmp, n);
        }
        if (jac) jac[p] = ora_jaccard(a, na, b, nb);
    }
}

/* Membership (Section 1: random access to one value of a set): 1 if x is in
 * the strictly increasing list v of n values, else 0. A plain binary search
 * over the whole list; the two-level search the library does (key, then
 * container) reaches the same answer. */
int ora_contains(const uint32_t *v, uint64_t n, uint32_t x) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (v[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && v[lo] == x;
}

/* Batched membership over a collection (values va, offsets oa):
 * out[i] = contains(set ids[i], xs[i]). */
void ora_contains_many(const uint32_t *va, const uint64_t *oa, const uint32_t *ids, const uint32_t *xs, uint64_t n,
                       uint8_t *out) {
    for (uint64_t i = 0; i < n; ++i) {
        const uint64_t s = oa[ids[i]], e = oa[ids[i] + 1];
        out[i] = (uint8_t)ora_contains(va + s, e - s, xs[i]);
    }
}

/* Serialised words (the digest's layout above) of container number `idx` of
 * the set v; returns the number of words (at most 1026), 0 if idx is out of
 * range. */
uint64_t ora_serialise(const uint32_t *v, uint64_t n, uint64_t idx, uint64_t *words) {
    uint64_t k = 0, i = 0;
    while (i < n) {
        uint32_t key = v[i] >> 16;
        uint64_t j = i;
        uint32_t r = 0;
        while (j < n && (v[j] >> 16) == key) {
            if (j == i || v[j] != v[j - 1] + 1) r++;
            j++;
        }
        if (k == idx) {
            uint32_t c = (uint32_t)(j - i);
            return serialise(v + i, c, r, ora_type_of(c, r), key, words);
        }
        k++;
        i = j;
    }
    return 0;
}
