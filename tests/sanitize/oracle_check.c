/* Sanitizer check of the CPU oracle (oracle/imsim_oracle.c): built with
 * -fsanitize=address,undefined (without OpenMP) by tests/test_sanitizers.py
 * and run over random graphs and the edge cases (empty seed set, every node a
 * seed, self-loops, repeated arcs, probabilities 0 and 1, full LT weights,
 * trial ranges that start inside a word), checking that every output stays
 * consistent.  Prints "oracle_check ok" on success. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_validate(int model, int64_t n, const int64_t* offsets, const uint32_t* indices, const uint64_t* w64);
int orc_simulate(int model, int64_t n, const int64_t* offsets, const uint32_t* indices, const void* param,
                 const uint32_t* seeds, int64_t n_seeds, int64_t t_begin, int64_t t_end, uint64_t rng_seed, int n_threads,
                 uint32_t* trial_counts, uint64_t* exams, uint32_t* node_counts, uint64_t* active_bits, int32_t* levels);

static uint64_t st = 0x243F6A8885A308D3ull;
static uint64_t rnd(void)
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return st;
}

#define CHECK(c)                                                     \
    do {                                                             \
        if (!(c)) {                                                  \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            exit(1);                                                 \
        }                                                            \
    } while (0)

static void run(int model, int64_t n, int64_t m, int seeds_mode, int64_t t0, int64_t T)
{
    int64_t* off = calloc((size_t)n + 1, sizeof(int64_t));
    uint32_t* idx = malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    uint32_t* src = malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t e = 0; e < m; ++e) src[e] = (uint32_t)(rnd() % (uint64_t)n);
    /* counting sort by source: rows in arc order */
    for (int64_t e = 0; e < m; ++e) off[src[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    int64_t* pos = malloc(sizeof(int64_t) * (size_t)n);
    memcpy(pos, off, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < m; ++e) idx[pos[src[e]]++] = (uint32_t)(rnd() % (uint64_t)n);
    void* param;
    if (model == 0) {
        uint32_t* thr = malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
        for (int64_t e = 0; e < m; ++e) {
            const uint64_t r = rnd() % 4;
            thr[e] = r == 0 ? 0u : (r == 1 ? 0xFFFFFFFFu : (uint32_t)(rnd() >> 40));
        }
        param = thr;
    } else {
        int64_t* indeg = calloc((size_t)n, sizeof(int64_t));
        for (int64_t e = 0; e < m; ++e) indeg[idx[e]]++;
        uint64_t* w = malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
        for (int64_t e = 0; e < m; ++e) w[e] = (1ull << 32) / (uint64_t)indeg[idx[e]];
        param = w;
        CHECK(orc_validate(1, n, off, idx, w) == 0);
        free(indeg);
    }
    int64_t ns = seeds_mode == 0 ? 0 : (seeds_mode == 1 ? n : 1 + (int64_t)(rnd() % 5));
    uint32_t* seeds = malloc(sizeof(uint32_t) * (size_t)(ns > 0 ? ns : 1));
    for (int64_t i = 0; i < ns; ++i) seeds[i] = seeds_mode == 1 ? (uint32_t)i : (uint32_t)(rnd() % (uint64_t)n);
    const int64_t W = (T + 63) / 64;
    uint32_t* tc = malloc(sizeof(uint32_t) * (size_t)T);
    uint64_t* ex = malloc(sizeof(uint64_t) * (size_t)T);
    uint32_t* nc = malloc(sizeof(uint32_t) * (size_t)n);
    uint64_t* bits = malloc(sizeof(uint64_t) * (size_t)(W * n));
    int32_t* lv = malloc(sizeof(int32_t) * (size_t)(T * n));
    CHECK(orc_simulate(model, n, off, idx, param, seeds, ns, t0, t0 + T, rnd(), 1, tc, ex, nc, bits, lv) == 0);
    uint64_t sum_tc = 0, sum_nc = 0, pop = 0;
    for (int64_t t = 0; t < T; ++t) sum_tc += tc[t];
    for (int64_t v = 0; v < n; ++v) sum_nc += nc[v];
    for (int64_t i = 0; i < W * n; ++i) pop += (uint64_t)__builtin_popcountll(bits[i]);
    CHECK(sum_tc == sum_nc && sum_nc == pop);
    for (int64_t t = 0; t < T; ++t) {
        int64_t active = 0;
        for (int64_t v = 0; v < n; ++v) active += lv[t * n + v] >= 0;
        CHECK(active == (int64_t)tc[t]);
        if (seeds_mode == 1) CHECK(tc[t] == (uint32_t)n);
    }
    free(off); free(idx); free(src); free(pos); free(param); free(seeds);
    free(tc); free(ex); free(nc); free(bits); free(lv);
}

int main(void)
{
    for (int rep = 0; rep < 60; ++rep) {
        const int64_t n = 1 + (int64_t)(rnd() % 120);
        const int64_t m = (int64_t)(rnd() % 600);
        const int64_t T = 1 + (int64_t)(rnd() % 150);
        const int64_t t0 = (int64_t)(rnd() % 100);
        run(rep & 1, n, m, rep % 3, t0, T);
    }
    printf("oracle_check ok\n");
    return 0;
}
