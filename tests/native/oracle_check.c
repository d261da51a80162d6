/* The CPU oracle and the host input generator under AddressSanitizer /
 * UndefinedBehaviorSanitizer: every entry point the tests use, on random sets
 * of every size class, with the results checked against a brute-force
 * membership count. Exit status 0 when every check holds. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint64_t ora_op(int op, const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb, uint32_t *out);
double ora_jaccard(const uint32_t *a, uint64_t na, const uint32_t *b, uint64_t nb);
uint64_t ora_kway(int op, const uint32_t *const *lists, const uint64_t *lens, uint32_t k, uint32_t *out,
                  uint32_t *tmp);
uint64_t ora_container_count(const uint32_t *v, uint64_t n);
void ora_containers(const uint32_t *v, uint64_t n, uint16_t *keys, uint8_t *types, uint32_t *card, uint32_t *runs,
                    uint64_t *first);
uint64_t ora_digest(const uint32_t *v, uint64_t n);
int ora_contains(const uint32_t *v, uint64_t n, uint32_t x);
uint64_t synth_mixed_bitmap(uint64_t seed, uint64_t index, uint64_t n_target, uint32_t ulog2, const uint32_t *hot,
                            uint32_t n_hot, uint32_t *out);
void synth_hot_keys(uint64_t seed, uint64_t stream, uint32_t n_hot, uint32_t n_chunks, uint32_t *out);

static int in(const uint32_t *v, uint64_t n, uint32_t x) {
    for (uint64_t i = 0; i < n; ++i)
        if (v[i] == x) return 1;
    return 0;
}

int main(void) {
    uint32_t hot[32];
    synth_hot_keys(7, 1, 32, 1024, hot);
    enum { K = 6 };
    uint32_t *sets[K];
    uint64_t lens[K];
    for (int i = 0; i < K; ++i) {
        uint64_t target = 50 + 4000 * (uint64_t)i;
        sets[i] = (uint32_t *)malloc(sizeof(uint32_t) * target);
        lens[i] = synth_mixed_bitmap(11, (uint64_t)i, target, 20, hot, 32, sets[i]);
        if (lens[i] > target) return 20;
    }
    uint32_t *out = (uint32_t *)malloc(sizeof(uint32_t) * 70000);
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * 70000);
    for (int a = 0; a < K; ++a) {
        for (int b = 0; b < K; ++b) {
            for (int op = 0; op < 4; ++op) {
                uint64_t n = ora_op(op, sets[a], lens[a], sets[b], lens[b], out);
                if (n != ora_op(op, sets[a], lens[a], sets[b], lens[b], NULL)) return 21;
                /* brute-force size of the result */
                uint64_t a_only = 0, b_only = 0, both = 0;
                for (uint64_t i = 0; i < lens[a]; ++i) {
                    if (in(sets[b], lens[b], sets[a][i])) both++;
                    else a_only++;
                }
                for (uint64_t j = 0; j < lens[b]; ++j) b_only += !in(sets[a], lens[a], sets[b][j]);
                const uint64_t e = op == 0 ? both : op == 1 ? a_only + b_only + both : op == 2 ? a_only + b_only
                                                                                                : a_only;
                if (n != e) return 22;
                for (uint64_t i = 1; i < n; ++i)
                    if (out[i] <= out[i - 1]) return 23;
                (void)ora_digest(out, n);
            }
            double j = ora_jaccard(sets[a], lens[a], sets[b], lens[b]);
            if (j < 0.0 || j > 1.0) return 24;
        }
        uint64_t nc = ora_container_count(sets[a], lens[a]);
        uint16_t *keys = (uint16_t *)malloc(2 * (nc + 1));
        uint8_t *types = (uint8_t *)malloc(nc + 1);
        uint32_t *card = (uint32_t *)malloc(4 * (nc + 1)), *runs = (uint32_t *)malloc(4 * (nc + 1));
        uint64_t *first = (uint64_t *)malloc(8 * (nc + 1));
        ora_containers(sets[a], lens[a], keys, types, card, runs, first);
        uint64_t tc = 0;
        for (uint64_t i = 0; i < nc; ++i) tc += card[i];
        if (tc != lens[a]) return 25;
        for (uint64_t i = 0; i < lens[a]; i += 17)
            if (!ora_contains(sets[a], lens[a], sets[a][i])) return 26;
        free(keys);
        free(types);
        free(card);
        free(runs);
        free(first);
    }
    const uint32_t *lists[K];
    for (int i = 0; i < K; ++i) lists[i] = sets[i];
    for (int op = 0; op < 4; ++op) (void)ora_kway(op, lists, lens, K, out, tmp);
    printf("oracle and generator: all checks passed\n");
    for (int i = 0; i < K; ++i) free(sets[i]);
    free(out);
    free(tmp);
    return 0;
}
