/*
 * oracle.c -- plain CPU oracle for the simplified stable parallel merge
 * (J. L. Traeff, "Simplified, stable parallel merging", arXiv:1202.6575).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the tests, the
 * package smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product path never calls it and shares no code with it.
 *
 * Every routine is written for readability, not speed: plain loops, one
 * comparison function per key type, no blocking and no fusion.
 *
 * Key types (the order relation of Section 2, problem statement):
 *   0 = int32  (signed compare), 1 = uint32, 2 = uint64 (unsigned compare),
 *   3 = int64, 4 = float32, 5 = float64 (IEEE 754 totalOrder).
 * Adding ORC_DESCENDING (8) to a key type reverses its order: "smaller" then
 * means "later in non-increasing order", and every routine below (ranks,
 * merges, sort) runs unchanged on that reversed relation.  Ties still keep
 * A before B and each source's own order.
 * Payloads are uint32 values that travel with their key; NULL means none.
 *
 * Pinned by tests/test_oracle_*.py against: the Figure 1 worked example,
 * brute-force stable sorting of (key, source, index)-tagged inputs, the
 * closed-form output positions, counting definitions of the two ranks,
 * special cases and invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_INT32 = 0, ORC_UINT32 = 1, ORC_UINT64 = 2, ORC_INT64 = 3, ORC_FLOAT32 = 4,
       ORC_FLOAT64 = 5, ORC_DESCENDING = 8 };

/* ------------------------------------------------------------------ */
/* Element access                                                      */
/* ------------------------------------------------------------------ */

static size_t key_size(int dtype)
{
    dtype &= 7;
    return dtype == ORC_UINT64 || dtype == ORC_INT64 || dtype == ORC_FLOAT64 ? 8 : 4;
}

/*
 * IEEE 754 totalOrder of two binary32 / binary64 values given as bit
 * patterns of `bits` bits: a negative sign orders before a positive one
 * (so -0 < +0 and -NaN < -inf); with equal signs, the magnitude (exponent
 * and significand read together as one unsigned number, which orders
 * numbers, infinities and NaN payloads as totalOrder does) decides,
 * ascending for positive values and descending for negative ones.
 */
static int total_order_lt(uint64_t a, uint64_t b, int bits)
{
    const uint64_t sign = (uint64_t)1 << (bits - 1);
    const uint64_t mag = sign - 1;
    const int na = (a & sign) != 0, nb = (b & sign) != 0;
    if (na != nb) return na;
    return na ? (a & mag) > (b & mag) : (a & mag) < (b & mag);
}

/* X[i] < Y[j] under the ascending order of the key type. */
static int key_lt_asc(const void *X, int64_t i, const void *Y, int64_t j, int dtype)
{
    switch (dtype) {
    case ORC_INT32:  return ((const int32_t *)X)[i]  < ((const int32_t *)Y)[j];
    case ORC_UINT32: return ((const uint32_t *)X)[i] < ((const uint32_t *)Y)[j];
    case ORC_INT64:  return ((const int64_t *)X)[i]  < ((const int64_t *)Y)[j];
    case ORC_FLOAT32:
        return total_order_lt(((const uint32_t *)X)[i], ((const uint32_t *)Y)[j], 32);
    case ORC_FLOAT64:
        return total_order_lt(((const uint64_t *)X)[i], ((const uint64_t *)Y)[j], 64);
    default:         return ((const uint64_t *)X)[i] < ((const uint64_t *)Y)[j];
    }
}

/* X[i] < Y[j] under the requested order: with ORC_DESCENDING, X[i] comes
 * before Y[j] exactly when Y[j] < X[i] ascending. */
static int key_lt(const void *X, int64_t i, const void *Y, int64_t j, int dtype)
{
    if (dtype & ORC_DESCENDING) return key_lt_asc(Y, j, X, i, dtype & 7);
    return key_lt_asc(X, i, Y, j, dtype);
}

static void key_copy(void *dst, int64_t di, const void *src, int64_t si, int dtype)
{
    size_t s = key_size(dtype);
    memcpy((char *)dst + (size_t)di * s, (const char *)src + (size_t)si * s, s);
}

/* ------------------------------------------------------------------ */
/* Ranks (Section 2, definitions of low and high rank)                 */
/* ------------------------------------------------------------------ */

/*
 * rank_low(x, X): the unique i in [0, len] with X[i-1] < x <= X[i], using the
 * sentinels X[-1] = -inf and X[len] = +inf.  It equals the number of
 * elements of X strictly smaller than x.  Binary search over [0, len].
 * x is element xi of array XA.
 */
int64_t orc_rank_low(const void *XA, int64_t xi, const void *X, int64_t len, int dtype)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (key_lt(X, mid, XA, xi, dtype))   /* X[mid] < x */
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/*
 * rank_high(x, X): the unique j in [0, len] with X[j-1] <= x < X[j]; the
 * number of elements of X smaller than or equal to x.
 */
int64_t orc_rank_high(const void *XA, int64_t xi, const void *X, int64_t len, int dtype)
{
    int64_t lo = 0, hi = len;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (!key_lt(XA, xi, X, mid, dtype))  /* X[mid] <= x */
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------ */
/* O1: the stable sequential merge the method assumes (Section 2,      */
/* stability paragraph; the abstract's "stable sequential merge")     */
/* ------------------------------------------------------------------ */

/*
 * Two-pointer merge of A (n) and B (m) into C (n+m).  An element of B is
 * taken only when it is strictly smaller than the current element of A, so
 * equal keys keep A before B and each source keeps its own order.
 */
void orc_merge(const void *A, const uint32_t *pa, int64_t n,
               const void *B, const uint32_t *pb, int64_t m,
               void *C, uint32_t *pc, int dtype)
{
    int64_t i = 0, j = 0, k = 0;
    while (i < n && j < m) {
        if (key_lt(B, j, A, i, dtype)) {          /* B[j] < A[i]: take B */
            key_copy(C, k, B, j, dtype);
            if (pc) pc[k] = pb[j];
            j++;
        } else {                                   /* A[i] <= B[j]: take A */
            key_copy(C, k, A, i, dtype);
            if (pc) pc[k] = pa[i];
            i++;
        }
        k++;
    }
    for (; i < n; i++, k++) {
        key_copy(C, k, A, i, dtype);
        if (pc) pc[k] = pa[i];
    }
    for (; j < m; j++, k++) {
        key_copy(C, k, B, j, dtype);
        if (pc) pc[k] = pb[j];
    }
}

/*
 * O5: many independent merges (Section 3, the merge applied to many pairs).
 * Pair k occupies keys[offsets[k], offsets[k+1]) with its first n_a[k]
 * elements as A and the rest as B; its merge lands in the same range of
 * out.  Pairs [k0, k1) only, so that callers can split a batch.
 */
void orc_merge_batched(const void *keys, const uint32_t *pay, const int64_t *offsets,
                       const int64_t *n_a, int64_t k0, int64_t k1,
                       void *out, uint32_t *out_pay, int dtype)
{
    size_t s = key_size(dtype);
    int64_t k;
    for (k = k0; k < k1; k++) {
        int64_t o = offsets[k], n = n_a[k], m = offsets[k + 1] - o - n_a[k];
        const char *A = (const char *)keys + (size_t)o * s;
        const char *B = A + (size_t)n * s;
        orc_merge(A, pay ? pay + o : NULL, n, B, pay ? pay + o + n : NULL, m,
                  (char *)out + (size_t)o * s, out_pay ? out_pay + o : NULL, dtype);
    }
}

/* ------------------------------------------------------------------ */
/* O2: closed-form output positions (Section 2, the paragraph after    */
/* Observation 1: A[i] lands at i + rank_low(A[i], B), B[j] at         */
/* j + rank_high(B[j], A))                                             */
/* ------------------------------------------------------------------ */

/*
 * Scatter every element to its closed-form position.  Returns 0 when the
 * positions form a permutation of [0, n+m), -1 otherwise.
 */
int orc_merge_scatter(const void *A, const uint32_t *pa, int64_t n,
                      const void *B, const uint32_t *pb, int64_t m,
                      void *C, uint32_t *pc, int dtype)
{
    int64_t total = n + m;
    unsigned char *hit = (unsigned char *)calloc((size_t)(total > 0 ? total : 1), 1);
    int ok = 0;
    if (!hit) return -1;
    for (int64_t i = 0; i < n; i++) {
        int64_t pos = i + orc_rank_low(A, i, B, m, dtype);
        if (pos < 0 || pos >= total || hit[pos]) { ok = -1; continue; }
        hit[pos] = 1;
        key_copy(C, pos, A, i, dtype);
        if (pc) pc[pos] = pa[i];
    }
    for (int64_t j = 0; j < m; j++) {
        int64_t pos = j + orc_rank_high(B, j, A, n, dtype);
        if (pos < 0 || pos >= total || hit[pos]) { ok = -1; continue; }
        hit[pos] = 1;
        key_copy(C, pos, B, j, dtype);
        if (pc) pc[pos] = pb[j];
    }
    for (int64_t k = 0; k < total; k++)
        if (!hit[k]) ok = -1;
    free(hit);
    return ok;
}

/* ------------------------------------------------------------------ */
/* Blocks (Section 2, block decomposition and block membership)        */
/* ------------------------------------------------------------------ */

/*
 * Start of block i of an array of length len split into p >= 1 blocks: the
 * first r = len mod p blocks have ceil(len/p) elements, the rest floor(len/p).
 * x_i = i*ceil(len/p) for i < r, else i*floor(len/p) + r; x_p = len.
 */
int64_t orc_block_start(int64_t len, int64_t p, int64_t i)
{
    int64_t q = len / p, r = len % p, c = (len + p - 1) / p;
    if (i >= p) return len;
    return i < r ? i * c : i * q + r;
}

/*
 * The block an index k belongs to.  For k < r*ceil(len/p) it is
 * floor(k / ceil(len/p)); otherwise floor((k - r*ceil(len/p)) / floor(len/p)) + r.
 * Reading for the cases the printed formula leaves open: an index k >= len
 * (the position of the +inf sentinel) belongs to the virtual block p; when
 * len < p every k < len falls in the first branch (r = len, ceil = 1), so
 * the division by floor(len/p) = 0 never happens.
 */
int64_t orc_block_of(int64_t len, int64_t p, int64_t k)
{
    int64_t q = len / p, r = len % p, c = (len + p - 1) / p;
    if (k >= len) return p;
    if (k < r * c) return k / c;
    return (k - r * c) / q + r;
}

/* ------------------------------------------------------------------ */
/* Steps 1 and 2: cross ranks of the block starts (Section 2, Steps)    */
/* ------------------------------------------------------------------ */

/*
 * xbar[i] = rank_low(A[x_i], B) for 0 <= i < p_a and xbar[p_a] = m;
 * ybar[j] = rank_high(B[y_j], A) for 0 <= j < p_b and ybar[p_b] = n.
 * A block that is empty (len < p) starts at the sentinel +inf, whose low
 * rank in B is m and whose high rank in A is n.
 * A and B may use different block counts (p_a != p_b); the correctness
 * argument of Section 2 does not depend on the counts being equal.
 */
void orc_cross_ranks(const void *A, int64_t n, const void *B, int64_t m,
                     int64_t p_a, int64_t p_b, int dtype,
                     int64_t *xbar, int64_t *ybar)
{
    for (int64_t i = 0; i < p_a; i++) {
        int64_t xi = orc_block_start(n, p_a, i);
        xbar[i] = xi < n ? orc_rank_low(A, xi, B, m, dtype) : m;
    }
    xbar[p_a] = m;
    for (int64_t j = 0; j < p_b; j++) {
        int64_t yj = orc_block_start(m, p_b, j);
        ybar[j] = yj < m ? orc_rank_high(B, yj, A, n, dtype) : n;
    }
    ybar[p_b] = n;
}

/* ------------------------------------------------------------------ */
/* Steps 3 and 4: the five cases (Section 2, Step 3 (a)-(e); Step 4     */
/* "in the same fashion"; Figure 2)                                     */
/* ------------------------------------------------------------------ */

/*
 * One subproblem: merge A[a_lo, a_hi) with B[b_lo, b_hi) stably (A before B
 * on equal keys) into C starting at c_off.  kase is the case letter: 'a'..'e'
 * for the processing element of A block i (Step 3), 'A'..'E' for the mirrored
 * cases of B block j (Step 4).
 */
typedef struct {
    int64_t a_lo, a_hi, b_lo, b_hi, c_off, kase;
} orc_piece;

/*
 * Step 3, the processing element of A block i (0 <= i < p_a), following the
 * printed case analysis.  Reading of case (d): its A range ends at x_{i+1}
 * (the whole A block); the printed index x_{j+1} is taken as a typo, since
 * the A range of a processing element never leaves its own block and only
 * x_{i+1} reproduces the Figure 1 subproblems and tiles C.
 */
static orc_piece step3_piece(int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                             const int64_t *xbar, const int64_t *ybar, int64_t i)
{
    orc_piece s;
    int64_t xi = orc_block_start(n, p_a, i), xi1 = orc_block_start(n, p_a, i + 1);
    int64_t xb = xbar[i], xb1 = xbar[i + 1];
    s.a_lo = xi;
    s.b_lo = xb;
    s.c_off = xi + xb;
    if (xb == xb1) {                               /* (a) copy the A block */
        s.a_hi = xi1; s.b_hi = xb; s.kase = 'a';
        return s;
    }
    int64_t j = orc_block_of(m, p_b, xb);          /* xb < m here */
    int64_t yj = orc_block_start(m, p_b, j), yj1 = orc_block_start(m, p_b, j + 1);
    if (xb == yj) {                                /* (e) A[x_i, ybar_j) alone */
        s.a_hi = ybar[j]; s.b_hi = xb; s.kase = 'e';
    } else if (orc_block_of(m, p_b, xb1) == j) {   /* (b) same B block */
        s.a_hi = xi1; s.b_hi = xb1; s.kase = 'b';
    } else if (xb1 != yj1) {                       /* (c) */
        s.a_hi = ybar[j + 1]; s.b_hi = yj1; s.kase = 'c';
    } else {                                       /* (d) */
        s.a_hi = xi1; s.b_hi = yj1; s.kase = 'd';
    }
    return s;
}

/*
 * Step 4, the processing element of B block j (0 <= j < p_b): Step 3 with
 * the roles of A and B exchanged (rank_low <-> rank_high, x <-> y).  The
 * tie rule stays with the sources: every merge keeps A before B.
 */
static orc_piece step4_piece(int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                             const int64_t *xbar, const int64_t *ybar, int64_t j)
{
    orc_piece s;
    int64_t yj = orc_block_start(m, p_b, j), yj1 = orc_block_start(m, p_b, j + 1);
    int64_t yb = ybar[j], yb1 = ybar[j + 1];
    s.b_lo = yj;
    s.a_lo = yb;
    s.c_off = yj + yb;
    if (yb == yb1) {                               /* (a') copy the B block */
        s.b_hi = yj1; s.a_hi = yb; s.kase = 'A';
        return s;
    }
    int64_t i = orc_block_of(n, p_a, yb);          /* yb < n here */
    int64_t xi = orc_block_start(n, p_a, i), xi1 = orc_block_start(n, p_a, i + 1);
    if (yb == xi) {                                /* (e') B[y_j, xbar_i) alone */
        s.b_hi = xbar[i]; s.a_hi = yb; s.kase = 'E';
    } else if (orc_block_of(n, p_a, yb1) == i) {   /* (b') same A block */
        s.b_hi = yj1; s.a_hi = yb1; s.kase = 'B';
    } else if (yb1 != xi1) {                       /* (c') */
        s.b_hi = xbar[i + 1]; s.a_hi = xi1; s.kase = 'C';
    } else {                                       /* (d') */
        s.b_hi = yj1; s.a_hi = xi1; s.kase = 'D';
    }
    return s;
}

/*
 * All 2p subproblems: p_a from Step 3 (indices 0..p_a-1), then p_b from
 * Step 4.  out must hold p_a + p_b records of 6 int64 each.
 */
void orc_pieces(int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                const int64_t *xbar, const int64_t *ybar, int64_t *out)
{
    for (int64_t i = 0; i < p_a; i++) {
        orc_piece s = step3_piece(n, m, p_a, p_b, xbar, ybar, i);
        memcpy(out + 6 * i, &s, sizeof s);
    }
    for (int64_t j = 0; j < p_b; j++) {
        orc_piece s = step4_piece(n, m, p_a, p_b, xbar, ybar, j);
        memcpy(out + 6 * (p_a + j), &s, sizeof s);
    }
}

/*
 * The same subproblems in a two-select form: outside case (e), the B range
 * of A block i ends at min(xbar_{i+1}, y_{j+1}) and its A range ends at
 * ybar_{j+1} when xbar_{i+1} > y_{j+1}, else at x_{i+1}; this covers (a)-(d)
 * at once.  Mirrored for Step 4.  kase is set to 0.  The tests require this
 * form to agree with orc_pieces on every input.
 */
void orc_pieces_two_select(int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                           const int64_t *xbar, const int64_t *ybar, int64_t *out)
{
    for (int64_t i = 0; i < p_a; i++) {
        int64_t xi = orc_block_start(n, p_a, i), xi1 = orc_block_start(n, p_a, i + 1);
        int64_t xb = xbar[i], xb1 = xbar[i + 1];
        int64_t j = orc_block_of(m, p_b, xb);      /* p_b when xb == m */
        int64_t yj = orc_block_start(m, p_b, j), yj1 = orc_block_start(m, p_b, j + 1);
        int64_t *s = out + 6 * i;
        s[0] = xi; s[2] = xb; s[4] = xi + xb; s[5] = 0;
        if (xb != xb1 && xb == yj) {
            s[1] = ybar[j]; s[3] = xb;
        } else {
            s[3] = xb1 < yj1 ? xb1 : yj1;
            s[1] = xb1 > yj1 ? ybar[j + 1] : xi1;
        }
    }
    for (int64_t j = 0; j < p_b; j++) {
        int64_t yj = orc_block_start(m, p_b, j), yj1 = orc_block_start(m, p_b, j + 1);
        int64_t yb = ybar[j], yb1 = ybar[j + 1];
        int64_t i = orc_block_of(n, p_a, yb);      /* p_a when yb == n */
        int64_t xi = orc_block_start(n, p_a, i), xi1 = orc_block_start(n, p_a, i + 1);
        int64_t *s = out + 6 * (p_a + j);
        s[2] = yj; s[0] = yb; s[4] = yj + yb; s[5] = 0;
        if (yb != yb1 && yb == xi) {
            s[3] = xbar[i]; s[1] = yb;
        } else {
            s[1] = yb1 < xi1 ? yb1 : xi1;
            s[3] = yb1 > xi1 ? xbar[i + 1] : yj1;
        }
    }
}

/*
 * The parallel merge of Section 2 executed sequentially: Steps 1-2, then each
 * of the 2p subproblems of Steps 3-4 merged with O1 into its own range of C.
 * Returns 0, or -1 if a subproblem would write outside C.
 */
int orc_merge_by_pieces(const void *A, const uint32_t *pa, int64_t n,
                        const void *B, const uint32_t *pb, int64_t m,
                        int64_t p_a, int64_t p_b,
                        void *C, uint32_t *pc, int dtype)
{
    int64_t *xbar = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p_a + 1));
    int64_t *ybar = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p_b + 1));
    int64_t *pcs = (int64_t *)malloc(sizeof(int64_t) * 6 * (size_t)(p_a + p_b));
    size_t ks = key_size(dtype);
    int rc = 0;
    if (!xbar || !ybar || !pcs) { free(xbar); free(ybar); free(pcs); return -1; }
    orc_cross_ranks(A, n, B, m, p_a, p_b, dtype, xbar, ybar);
    orc_pieces(n, m, p_a, p_b, xbar, ybar, pcs);
    for (int64_t s = 0; s < p_a + p_b; s++) {
        const int64_t *d = pcs + 6 * s;
        int64_t la = d[1] - d[0], lb = d[3] - d[2];
        if (la < 0 || lb < 0 || d[4] < 0 || d[4] + la + lb > n + m) { rc = -1; break; }
        orc_merge((const char *)A + (size_t)d[0] * ks, pa ? pa + d[0] : NULL, la,
                  (const char *)B + (size_t)d[2] * ks, pb ? pb + d[2] : NULL, lb,
                  (char *)C + (size_t)d[4] * ks, pc ? pc + d[4] : NULL, dtype);
    }
    free(xbar); free(ybar); free(pcs);
    return rc;
}

/* ------------------------------------------------------------------ */
/* O4: stable merge sort (Section 3): sort consecutive blocks          */
/* sequentially, then ceil(log2(#runs)) rounds of pairwise merges; a   */
/* run without a partner is copied; the two arrays are used in turn.   */
/* ------------------------------------------------------------------ */

/* Stable insertion sort of keys[lo, hi) with payloads. */
static void insertion_sort(void *keys, uint32_t *pay, int64_t lo, int64_t hi, int dtype)
{
    size_t ks = key_size(dtype);
    unsigned char tmp[8];
    for (int64_t i = lo + 1; i < hi; i++) {
        uint32_t tp = pay ? pay[i] : 0;
        memcpy(tmp, (char *)keys + (size_t)i * ks, ks);
        int64_t k = i;
        /* move left only past strictly larger keys: equal keys keep order */
        while (k > lo && key_lt(tmp, 0, keys, k - 1, dtype)) {
            key_copy(keys, k, keys, k - 1, dtype);
            if (pay) pay[k] = pay[k - 1];
            k--;
        }
        memcpy((char *)keys + (size_t)k * ks, tmp, ks);
        if (pay) pay[k] = tp;
    }
}

/*
 * Sorts keys[0, N) (payloads travel along).  run_len >= 1 is the length of
 * the sequentially sorted blocks.  The result ends in keys/pay; tmp_keys and
 * tmp_pay (N elements each, tmp_pay may be NULL when pay is NULL) are the
 * second array of the ping-pong.
 */
void orc_sort(void *keys, uint32_t *pay, int64_t N, int64_t run_len,
              void *tmp_keys, uint32_t *tmp_pay, int dtype)
{
    size_t ks = key_size(dtype);
    void *src = keys, *dst = tmp_keys;
    uint32_t *sp = pay, *dp = tmp_pay;
    for (int64_t lo = 0; lo < N; lo += run_len)
        insertion_sort(keys, pay, lo, lo + run_len < N ? lo + run_len : N, dtype);
    for (int64_t w = run_len; w < N; w *= 2) {
        for (int64_t lo = 0; lo < N; lo += 2 * w) {
            int64_t mid = lo + w < N ? lo + w : N;
            int64_t hi = lo + 2 * w < N ? lo + 2 * w : N;
            /* runs [lo, mid) and [mid, hi); mid == hi copies a lone run */
            orc_merge((char *)src + (size_t)lo * ks, sp ? sp + lo : NULL, mid - lo,
                      (char *)src + (size_t)mid * ks, sp ? sp + mid : NULL, hi - mid,
                      (char *)dst + (size_t)lo * ks, dp ? dp + lo : NULL, dtype);
        }
        void *t = src; src = dst; dst = t;
        uint32_t *tp = sp; sp = dp; dp = tp;
    }
    if (src != keys) {
        memcpy(keys, src, (size_t)N * ks);
        if (pay) memcpy(pay, sp, (size_t)N * sizeof(uint32_t));
    }
}

/* ------------------------------------------------------------------ */
/* O6: bounded exponential search from a guess (learned cross rank;    */
/* an addition to the paper's plain binary search of Steps 1-2)        */
/* ------------------------------------------------------------------ */

/*
 * Returns the exact rank_low (is_high = 0) or rank_high (is_high = 1) of
 * x = XA[xi] in X[0, len), starting from the guess g (clamped to [0, len]).
 * Let pred(t) be "X[t] < x" (low) or "X[t] <= x" (high); the rank is the
 * number of t with pred(t) true.  The search probes g, then moves away from
 * g in steps of step0, 2 step0, 4 step0, ... until the rank is bracketed,
 * then binary searches the bracket, splitting it at aligned points (below).
 * If a step larger than window would be needed, it gives up and binary
 * searches all of [0, len] instead (*fallback = 1).  *probes counts every
 * element of X that is read.
 * step0 >= 1 (the initial step is a free choice of the search: a predictor
 * whose typical error is e starts near e instead of 1).
 */
int64_t orc_gallop(const void *XA, int64_t xi, const void *X, int64_t len, int dtype,
                   int is_high, int64_t g, int64_t step0, int64_t window,
                   int64_t *probes, int *fallback)
{
    int64_t lo, hi, np = 0;
#define PRED(t) (np++, is_high ? !key_lt(XA, xi, X, (t), dtype) : key_lt(X, (t), XA, xi, dtype))
    *fallback = 0;
    if (g < 0) g = 0;
    if (g > len) g = len;
    if (g < len && PRED(g)) {
        /* rank > g: move right */
        int64_t d = step0 < 1 ? 1 : step0;
        lo = g + 1;
        for (;;) {
            if (d > window) goto full;
            int64_t t = g + d;
            if (t >= len) { hi = len; break; }
            if (!PRED(t)) { hi = t; break; }
            lo = t + 1;
            d *= 2;
        }
    } else {
        /* rank <= g: move left */
        int64_t d = step0 < 1 ? 1 : step0;
        hi = g;
        for (;;) {
            if (d > window) goto full;
            int64_t t = g - d;
            if (t < 0) { lo = 0; break; }
            if (PRED(t)) { lo = t + 1; break; }
            hi = t;
            d *= 2;
        }
    }
    goto bisect;
full:
    *fallback = 1;
    lo = 0;
    hi = len;
bisect:
    /* The rank lies in [lo, hi].  Each probe splits the bracket at the
     * number m in (lo, hi] with the most trailing zero bits (the top bit in
     * which lo and hi differ set, the bits below it clear): the rank is >= m
     * exactly when X[m - 1] satisfies the predicate.  Split points are
     * aligned, so searches with nearby brackets probe the same elements. */
    while (lo < hi) {
        int h = 63;
        while (!(((uint64_t)lo ^ (uint64_t)hi) >> h & 1)) h--;
        int64_t m = (int64_t)(((uint64_t)hi >> h) << h);
        if (PRED(m - 1)) lo = m;
        else hi = m - 1;
    }
#undef PRED
    *probes = np;
    return lo;
}
