/*
 * synth.c - seeded synthetic inputs (host side).
 *
 * This module generates integer sets only. It holds none of the set-operation
 * arithmetic, container typing or layout of either the GPU library or the
 * oracle; both of those consume its outputs (sorted uint32 value lists, or
 * raw 1024-word bitsets for the dense-bitset workload).
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), used as a counter-based
 * generator:
 *     key(seed, stream) = mix64(seed + (stream + 1) * GAMMA)
 *     rand(seed, stream, ctr) = mix64(key + (ctr + 1) * GAMMA)
 * i.e. output number ctr of the SplitMix64 sequence whose state starts at
 * key(seed, stream). mix64 is the SplitMix64 output finalizer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

uint64_t synth_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_stream_key(uint64_t seed, uint64_t stream) {
    return synth_mix64(seed + (stream + 1) * GAMMA);
}

uint64_t synth_rand(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return synth_mix64(synth_stream_key(seed, stream) + (ctr + 1) * GAMMA);
}

typedef struct {
    uint64_t key;
    uint64_t ctr;
} rng_t;

static rng_t rng_make(uint64_t seed, uint64_t stream) {
    rng_t r;
    r.key = synth_stream_key(seed, stream);
    r.ctr = 0;
    return r;
}

static uint64_t rng_next(rng_t *r) {
    r->ctr += 1;
    return synth_mix64(r->key + r->ctr * GAMMA);
}

/* uniform double in [0, 1) */
static double rng_unit(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform double in (0, 1] */
static double rng_unit_open0(rng_t *r) { return (double)((rng_next(r) >> 11) + 1) * 0x1.0p-53; }

/* geometric on {1, 2, ...} with success probability p (mean 1/p) */
static uint64_t rng_geom(rng_t *r, double p) {
    double u = rng_unit_open0(r);
    double g = floor(log(u) / log1p(-p));
    if (g > 1e9) g = 1e9;
    return 1 + (uint64_t)g;
}

static uint64_t rng_below(rng_t *r, uint64_t n) { return n ? rng_next(r) % n : 0; }

/* ---- sorting: LSD radix sort of uint32 (two 16-bit passes), then dedup ---- */

static void radix_sort_u32(uint32_t *v, uint64_t n, uint32_t *tmp) {
    static const int B = 16;
    uint64_t *cnt = (uint64_t *)calloc((size_t)1 << B, sizeof(uint64_t));
    uint32_t *src = v, *dst = tmp;
    for (int pass = 0; pass < 2; ++pass) {
        int sh = pass * B;
        memset(cnt, 0, sizeof(uint64_t) << B);
        for (uint64_t i = 0; i < n; ++i) cnt[(src[i] >> sh) & 0xFFFF]++;
        uint64_t s = 0;
        for (uint64_t d = 0; d < ((uint64_t)1 << B); ++d) {
            uint64_t c = cnt[d];
            cnt[d] = s;
            s += c;
        }
        for (uint64_t i = 0; i < n; ++i) dst[cnt[(src[i] >> sh) & 0xFFFF]++] = src[i];
        uint32_t *t = src;
        src = dst;
        dst = t;
    }
    /* after an even number of passes the data is back in v */
    free(cnt);
}

static uint64_t sort_unique(uint32_t *v, uint64_t n) {
    if (n == 0) return 0;
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * n);
    radix_sort_u32(v, n, tmp);
    free(tmp);
    uint64_t w = 1;
    for (uint64_t i = 1; i < n; ++i)
        if (v[i] != v[w - 1]) v[w++] = v[i];
    return w;
}

uint64_t synth_sort_unique(uint32_t *v, uint64_t n) { return sort_unique(v, n); }

/* ---- distinct hot chunk keys ---- */

void synth_hot_keys(uint64_t seed, uint64_t stream, uint32_t n_hot, uint32_t n_chunks,
                    uint32_t *out) {
    rng_t r = rng_make(seed, stream);
    uint32_t k = 0;
    while (k < n_hot) {
        uint32_t c = (uint32_t)rng_below(&r, n_chunks);
        int dup = 0;
        for (uint32_t i = 0; i < k; ++i)
            if (out[i] == c) dup = 1;
        if (!dup) out[k++] = c;
    }
}

/*
 * Mixed bitmap: n_target values split 40% uniform sparse over [0, 2^ulog2),
 * 30% one dense window (density d ~ U(0.3, 0.9), Bernoulli(d) per position,
 * window length ceil(n_dense / d), placed in a chunk drawn from the hot set),
 * 30% clustered runs (lengths and gaps Geom(mean 64), starting at a uniform
 * position of a hot chunk). The union is sorted and deduplicated.
 * out must hold n_target values. Returns the number of distinct values.
 */
uint64_t synth_mixed_bitmap(uint64_t seed, uint64_t index, uint64_t n_target, uint32_t ulog2,
                            const uint32_t *hot, uint32_t n_hot, uint32_t *out) {
    const uint64_t U = (uint64_t)1 << ulog2;
    const uint64_t n_sparse = n_target * 4 / 10;
    const uint64_t n_dense = n_target * 3 / 10;
    const uint64_t n_run = n_target - n_sparse - n_dense;
    uint64_t w = 0;

    rng_t rs = rng_make(seed, index * 4 + 0);
    for (uint64_t i = 0; i < n_sparse; ++i) out[w++] = (uint32_t)(rng_next(&rs) & (U - 1));

    rng_t rd = rng_make(seed, index * 4 + 1);
    if (n_dense > 0) {
        double d = 0.3 + 0.6 * rng_unit(&rd);
        uint64_t L = (uint64_t)ceil((double)n_dense / d);
        uint64_t chunk = hot[rng_below(&rd, n_hot)];
        uint64_t start = chunk << 16;
        if (L <= 65536) start += rng_below(&rd, 65536 - L + 1);
        uint64_t placed = 0;
        for (uint64_t p = 0; p < L && placed < n_dense; ++p) {
            if (start + p >= U) break;
            if (rng_unit(&rd) < d) {
                out[w++] = (uint32_t)(start + p);
                placed++;
            }
        }
    }

    rng_t rr = rng_make(seed, index * 4 + 2);
    if (n_run > 0) {
        uint64_t pos = ((uint64_t)hot[rng_below(&rr, n_hot)] << 16) + rng_below(&rr, 65536);
        uint64_t placed = 0;
        while (placed < n_run && pos < U) {
            uint64_t len = rng_geom(&rr, 1.0 / 64.0);
            uint64_t gap = rng_geom(&rr, 1.0 / 64.0);
            for (uint64_t q = 0; q < len && placed < n_run; ++q) {
                if (pos + q < U) out[w++] = (uint32_t)(pos + q);
                placed++;
            }
            pos += len + gap;
        }
    }
    return sort_unique(out, w);
}

/* ---- lognormal cardinality, clipped ---- */
uint64_t synth_lognormal_card(uint64_t seed, uint64_t stream, uint64_t idx, double median,
                              double sigma, uint64_t lo, uint64_t hi) {
    rng_t r = rng_make(seed, stream);
    r.ctr = idx * 2;
    double u1 = rng_unit_open0(&r), u2 = rng_unit(&r);
    double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2); /* Box-Muller */
    double c = exp(log(median) + sigma * z);
    if (c < (double)lo) c = (double)lo;
    if (c > (double)hi) c = (double)hi;
    return (uint64_t)c;
}

/* ---- array-array stress sizes: truncated Zipf(s) on [1, kmax], ratio <= rmax ---- */
void synth_zipf_pair_sizes(uint64_t seed, uint64_t stream, uint64_t n_pairs, double s,
                           uint32_t kmax, uint32_t rmax, uint32_t *ca, uint32_t *cb) {
    double *cdf = (double *)malloc(sizeof(double) * kmax);
    double acc = 0;
    for (uint32_t k = 1; k <= kmax; ++k) {
        acc += pow((double)k, -s);
        cdf[k - 1] = acc;
    }
    for (uint32_t k = 0; k < kmax; ++k) cdf[k] /= acc;
    for (uint64_t p = 0; p < n_pairs; ++p) {
        rng_t r = rng_make(seed, stream + p);
        for (;;) {
            uint32_t v[2];
            for (int t = 0; t < 2; ++t) {
                double u = rng_unit(&r);
                uint32_t lo = 0, hi = kmax - 1;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) / 2;
                    if (cdf[mid] < u)
                        lo = mid + 1;
                    else
                        hi = mid;
                }
                v[t] = lo + 1;
            }
            uint32_t mx = v[0] > v[1] ? v[0] : v[1], mn = v[0] < v[1] ? v[0] : v[1];
            if (mx <= (uint64_t)mn * rmax) {
                ca[p] = v[0];
                cb[p] = v[1];
                break;
            }
        }
    }
    free(cdf);
}

/* c distinct uniform values of [0, 65536), sorted ascending, plus an offset */
void synth_distinct_u16(uint64_t seed, uint64_t stream, uint32_t c, uint32_t base, uint32_t *out) {
    uint64_t mark[1024];
    memset(mark, 0, sizeof(mark));
    rng_t r = rng_make(seed, stream);
    uint32_t k = 0;
    if (c > 65536) c = 65536;
    while (k < c) {
        uint32_t v = (uint32_t)(rng_next(&r) & 0xFFFF);
        if (!(mark[v >> 6] >> (v & 63) & 1)) {
            mark[v >> 6] |= 1ULL << (v & 63);
            k++;
        }
    }
    k = 0;
    for (uint32_t wi = 0; wi < 1024; ++wi) {
        uint64_t x = mark[wi];
        while (x) {
            out[k++] = base + wi * 64 + (uint32_t)__builtin_ctzll(x);
            x &= x - 1;
        }
    }
}

/* ---- dense-bitset workload (CPU twin of the device generator) ----
 * Container (b, k): threshold t = 13107 + rand(seed, b, k) % 39322, so the bit
 * density t / 65536 lies in [0.2, 0.8). Word w, bit 4i+j (i < 16, j < 4) is set
 * iff 16-bit lane j of rand(seed, 2^40 + b * 2^16 + k, w * 16 + i) is < t.
 */
uint32_t synth_dense_threshold(uint64_t seed, uint64_t b, uint64_t k) {
    return 13107u + (uint32_t)(synth_rand(seed, b, k) % 39322u);
}

void synth_dense_container(uint64_t seed, uint64_t b, uint64_t k, uint64_t *words) {
    uint32_t t = synth_dense_threshold(seed, b, k);
    uint64_t key = synth_stream_key(seed, ((uint64_t)1 << 40) + (b << 16) + k);
    for (uint64_t w = 0; w < 1024; ++w) {
        uint64_t x = 0;
        for (uint64_t i = 0; i < 16; ++i) {
            uint64_t h = synth_mix64(key + (w * 16 + i + 1) * GAMMA);
            for (uint64_t j = 0; j < 4; ++j) {
                uint32_t u = (uint32_t)(h >> (16 * j)) & 0xFFFF;
                if (u < t) x |= 1ULL << (4 * i + j);
            }
        }
        words[w] = x;
    }
}

/* the values of dense bitmap b (keys 0..n_keys-1); out must hold n_keys*65536 */
uint64_t synth_dense_bitmap_values(uint64_t seed, uint64_t b, uint32_t n_keys, uint32_t *out) {
    uint64_t words[1024];
    uint64_t n = 0;
    for (uint32_t k = 0; k < n_keys; ++k) {
        synth_dense_container(seed, b, k, words);
        for (uint32_t w = 0; w < 1024; ++w) {
            uint64_t x = words[w];
            for (uint32_t bit = 0; bit < 64; ++bit)
                if (x >> bit & 1) out[n++] = (k << 16) | (w << 6) | bit;
        }
    }
    return n;
}

/* n_pairs random (ia != ib) pairs over [0, n) */
void synth_random_pairs(uint64_t seed, uint64_t stream, uint64_t n, uint64_t n_pairs, uint32_t *ia,
                        uint32_t *ib) {
    rng_t r = rng_make(seed, stream);
    for (uint64_t p = 0; p < n_pairs; ++p) {
        uint32_t a = (uint32_t)rng_below(&r, n);
        uint32_t b = (uint32_t)rng_below(&r, n);
        while (n > 1 && b == a) b = (uint32_t)rng_below(&r, n);
        ia[p] = a;
        ib[p] = b;
    }
}
