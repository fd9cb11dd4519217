/*
 * Host memory-safety check of the CPU oracle: built with the address and
 * undefined-behaviour sanitizers and run by tests/test_oracle_sanitize.py.
 * Exercises every oracle routine on seeded random inputs (empty arrays,
 * n < p, heavy ties, all three key types) and checks that the three merge
 * forms agree and the sort is ordered.  Exit status 0 = no failure.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_rank_low(const void *XA, int64_t xi, const void *X, int64_t len, int dtype);
int64_t orc_rank_high(const void *XA, int64_t xi, const void *X, int64_t len, int dtype);
void orc_merge(const void *A, const uint32_t *pa, int64_t n, const void *B, const uint32_t *pb,
               int64_t m, void *C, uint32_t *pc, int dtype);
int orc_merge_scatter(const void *A, const uint32_t *pa, int64_t n, const void *B,
                      const uint32_t *pb, int64_t m, void *C, uint32_t *pc, int dtype);
void orc_cross_ranks(const void *A, int64_t n, const void *B, int64_t m, int64_t p_a,
                     int64_t p_b, int dtype, int64_t *xbar, int64_t *ybar);
void orc_pieces(int64_t n, int64_t m, int64_t p_a, int64_t p_b, const int64_t *xbar,
                const int64_t *ybar, int64_t *out);
void orc_pieces_two_select(int64_t n, int64_t m, int64_t p_a, int64_t p_b, const int64_t *xbar,
                           const int64_t *ybar, int64_t *out);
int orc_merge_by_pieces(const void *A, const uint32_t *pa, int64_t n, const void *B,
                        const uint32_t *pb, int64_t m, int64_t p_a, int64_t p_b, void *C,
                        uint32_t *pc, int dtype);
void orc_sort(void *keys, uint32_t *pay, int64_t N, int64_t run_len, void *tmp_keys,
              uint32_t *tmp_pay, int dtype);
int64_t orc_gallop(const void *XA, int64_t xi, const void *X, int64_t len, int dtype, int is_high,
                   int64_t g, int64_t step0, int64_t window, int64_t *probes, int *fallback);

static uint64_t state = 0x12026575ull;
static uint64_t next_u64(void)
{
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

static size_t ksize(int dtype) { return dtype == 2 ? 8 : 4; }

static int cmp_key(const void *X, int64_t i, int64_t j, int dtype)
{
    if (dtype == 0) {
        int32_t a = ((const int32_t *)X)[i], b = ((const int32_t *)X)[j];
        return (a > b) - (a < b);
    }
    if (dtype == 1) {
        uint32_t a = ((const uint32_t *)X)[i], b = ((const uint32_t *)X)[j];
        return (a > b) - (a < b);
    }
    uint64_t a = ((const uint64_t *)X)[i], b = ((const uint64_t *)X)[j];
    return (a > b) - (a < b);
}

/* n random keys over `alpha` symbols, sorted by insertion (small n) */
static void *rand_sorted(int64_t n, uint64_t alpha, int dtype, int sorted)
{
    void *X = malloc((size_t)(n > 0 ? n : 1) * ksize(dtype));
    for (int64_t i = 0; i < n; i++) {
        uint64_t v = next_u64() % alpha;
        if (dtype == 0) ((int32_t *)X)[i] = (int32_t)(v - alpha / 2);
        else if (dtype == 1) ((uint32_t *)X)[i] = (uint32_t)(v * (0xffffffffull / alpha));
        else ((uint64_t *)X)[i] = v * (0xffffffffffffffffull / alpha);
    }
    if (sorted)
        for (int64_t i = 1; i < n; i++)
            for (int64_t j = i; j > 0 && cmp_key(X, j - 1, j, dtype) > 0; j--) {
                char tmp[8];
                size_t s = ksize(dtype);
                memcpy(tmp, (char *)X + (size_t)(j - 1) * s, s);
                memcpy((char *)X + (size_t)(j - 1) * s, (char *)X + (size_t)j * s, s);
                memcpy((char *)X + (size_t)j * s, tmp, s);
            }
    return X;
}

int main(void)
{
    int failures = 0;
    for (int trial = 0; trial < 3000; trial++) {
        int dtype = trial % 3;
        int64_t n = (int64_t)(next_u64() % 60), m = (int64_t)(next_u64() % 60);
        uint64_t alpha = 1 + next_u64() % 40;
        int64_t pa = 1 + (int64_t)(next_u64() % 12), pb = 1 + (int64_t)(next_u64() % 12);
        size_t s = ksize(dtype);
        void *A = rand_sorted(n, alpha, dtype, 1), *B = rand_sorted(m, alpha, dtype, 1);
        uint32_t *qa = malloc((size_t)(n + 1) * 4), *qb = malloc((size_t)(m + 1) * 4);
        for (int64_t i = 0; i < n; i++) qa[i] = (uint32_t)i;
        for (int64_t j = 0; j < m; j++) qb[j] = (uint32_t)(n + j);
        size_t cb = (size_t)(n + m + 1);
        void *C1 = malloc(cb * s), *C2 = malloc(cb * s), *C3 = malloc(cb * s);
        uint32_t *q1 = malloc(cb * 4), *q2 = malloc(cb * 4), *q3 = malloc(cb * 4);
        orc_merge(A, qa, n, B, qb, m, C1, q1, dtype);
        if (orc_merge_scatter(A, qa, n, B, qb, m, C2, q2, dtype) != 0) failures++;
        if (orc_merge_by_pieces(A, qa, n, B, qb, m, pa, pb, C3, q3, dtype) != 0) failures++;
        if (memcmp(C1, C2, (size_t)(n + m) * s) || memcmp(C1, C3, (size_t)(n + m) * s) ||
            memcmp(q1, q2, (size_t)(n + m) * 4) || memcmp(q1, q3, (size_t)(n + m) * 4))
            failures++;
        int64_t *xbar = malloc((size_t)(pa + 1) * 8), *ybar = malloc((size_t)(pb + 1) * 8);
        int64_t *pc1 = malloc((size_t)(pa + pb) * 6 * 8), *pc2 = malloc((size_t)(pa + pb) * 6 * 8);
        orc_cross_ranks(A, n, B, m, pa, pb, dtype, xbar, ybar);
        orc_pieces(n, m, pa, pb, xbar, ybar, pc1);
        orc_pieces_two_select(n, m, pa, pb, xbar, ybar, pc2);
        for (int64_t w = 0; w < pa + pb; w++)
            for (int f = 0; f < 5; f++)
                if (pc1[6 * w + f] != pc2[6 * w + f]) failures++;
        /* the bounded search returns the exact rank from any guess */
        for (int64_t i = 0; i < n; i++) {
            int64_t probes;
            int fb;
            int64_t g = (int64_t)(next_u64() % (uint64_t)(m + 3)) - 1;
            int64_t r = orc_gallop(A, i, B, m, dtype, 0, g, 1 + (int64_t)(next_u64() % 4),
                                   (int64_t)(next_u64() % 16), &probes, &fb);
            if (r != orc_rank_low(A, i, B, m, dtype)) failures++;
        }
        /* sort of an unsorted array with payloads, ragged run lengths */
        int64_t N = n + m;
        void *K = rand_sorted(N, alpha, dtype, 0);
        uint32_t *P = malloc((size_t)(N + 1) * 4);
        for (int64_t i = 0; i < N; i++) P[i] = (uint32_t)i;
        void *TK = malloc((size_t)(N + 1) * s);
        uint32_t *TP = malloc((size_t)(N + 1) * 4);
        orc_sort(K, P, N, 1 + (int64_t)(next_u64() % 9), TK, TP, dtype);
        for (int64_t i = 1; i < N; i++) {
            int c = cmp_key(K, i - 1, i, dtype);
            if (c > 0 || (c == 0 && P[i - 1] > P[i])) failures++;
        }
        free(A); free(B); free(qa); free(qb); free(C1); free(C2); free(C3); free(q1); free(q2);
        free(q3); free(xbar); free(ybar); free(pc1); free(pc2); free(K); free(P); free(TK); free(TP);
    }
    printf("failures %d\n", failures);
    return failures ? 1 : 0;
}
