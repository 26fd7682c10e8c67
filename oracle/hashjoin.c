/*
 * Plain C hash join of two key columns (test infrastructure only: the
 * oracle's second, independently written witness of the equi-join that
 * Algorithm 1 of the MapSQ paper computes, and its multi-core host timing).
 * Nothing in the GPU product links or loads this file.
 *
 * The build side is chained through a power-of-two bucket array; the probe
 * side is split over OpenMP threads.  Two passes: count the matches of every
 * probe row, prefix-sum the counts, then write the (probe row, build row)
 * index pairs.  Output order: probe rows ascending, then build rows in chain
 * order (the join's row order is not part of its result).
 */
#include <stdint.h>
#include <stdlib.h>
#include <omp.h>

static uint64_t mix(uint32_t k) {
    uint64_t x = (uint64_t)k * 0x9E3779B97F4A7C15ull;
    return x ^ (x >> 29);
}

typedef struct { int64_t* head; int64_t* next; uint64_t mask; } chains;

static int build(const int32_t* bk, int64_t nb, chains* c) {
    uint64_t size = 1;
    while (size < (uint64_t)(2 * nb + 1)) size <<= 1;
    c->mask = size - 1;
    c->head = (int64_t*)malloc(size * sizeof(int64_t));
    c->next = (int64_t*)malloc((nb > 0 ? nb : 1) * sizeof(int64_t));
    if (!c->head || !c->next) return -1;
    for (uint64_t i = 0; i < size; i++) c->head[i] = -1;
    /* insert in descending order so each chain lists build rows ascending */
    for (int64_t j = nb - 1; j >= 0; j--) {
        uint64_t h = mix((uint32_t)bk[j]) & c->mask;
        c->next[j] = c->head[h];
        c->head[h] = j;
    }
    return 0;
}

/* Number of pairs (i, j) with pk[i] == bk[j]; -1 on allocation failure. */
int64_t oracle_hj_count(const int32_t* pk, int64_t np_, const int32_t* bk, int64_t nb, int nthreads) {
    chains c;
    if (build(bk, nb, &c)) return -1;
    int64_t total = 0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for reduction(+ : total) schedule(static)
    for (int64_t i = 0; i < np_; i++) {
        for (int64_t j = c.head[mix((uint32_t)pk[i]) & c.mask]; j >= 0; j = c.next[j])
            if (bk[j] == pk[i]) total++;
    }
    free(c.head);
    free(c.next);
    return total;
}

/* Writes up to cap pairs into out_p/out_b; returns the pair count, or -1 on
 * allocation failure, or -2 when cap is too small (nothing meaningful written). */
int64_t oracle_hj_pairs(const int32_t* pk, int64_t np_, const int32_t* bk, int64_t nb,
                        int64_t* out_p, int64_t* out_b, int64_t cap, int nthreads) {
    chains c;
    if (build(bk, nb, &c)) return -1;
    int64_t* cnt = (int64_t*)malloc((np_ + 1) * sizeof(int64_t));
    if (!cnt) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np_; i++) {
        int64_t m = 0;
        for (int64_t j = c.head[mix((uint32_t)pk[i]) & c.mask]; j >= 0; j = c.next[j])
            if (bk[j] == pk[i]) m++;
        cnt[i] = m;
    }
    int64_t run = 0;
    for (int64_t i = 0; i < np_; i++) { int64_t m = cnt[i]; cnt[i] = run; run += m; }
    cnt[np_] = run;
    if (run > cap) { free(cnt); free(c.head); free(c.next); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np_; i++) {
        int64_t w = cnt[i];
        for (int64_t j = c.head[mix((uint32_t)pk[i]) & c.mask]; j >= 0; j = c.next[j])
            if (bk[j] == pk[i]) { out_p[w] = i; out_b[w] = j; w++; }
    }
    free(cnt);
    free(c.head);
    free(c.next);
    return run;
}
