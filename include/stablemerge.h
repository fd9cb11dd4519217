/*
 * stablemerge.h -- C ABI of libstablemerge.so, a stable parallel merge for
 * AMD Instinct MI355X (gfx950), after J. L. Traeff, "Simplified, stable
 * parallel merging" (arXiv:1202.6575).
 *
 * The method (Section 2): split the non-decreasing arrays A (n elements) and
 * B (m elements) into blocks; compute the cross rank of every block's first
 * element -- rank_low of an A element in B (Step 1), rank_high of a B
 * element in A (Step 2); after one synchronisation, every block's processing
 * element picks one of five cases and merges a disjoint pair of segments
 * into its own range of C (Steps 3 and 4, Figure 2).  Equal keys keep A
 * before B and each source keeps its own order (stability, Section 2).
 *
 * Conventions shared by every entry point:
 *  - Every data pointer is a DEVICE pointer (HIP global memory) owned by the
 *    caller.  The library never allocates, frees or retains caller memory.
 *  - Keys of A and B are stored contiguously in one buffer: A = keys[0, n),
 *    B = keys[n, n + m).  Payloads (optional, uint32) use the same layout.
 *  - Key type (dtype): SM_INT32 and SM_INT64 compare as signed integers,
 *    SM_UINT32 and SM_UINT64 as unsigned; SM_FLOAT32 and SM_FLOAT64 follow
 *    IEEE 754 totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN,
 *    NaNs ordered by payload), so every bit pattern is a key and -0 comes
 *    strictly before +0.  Key, payload and output arrays passed to
 *    the merge entry points must start on a 16-byte boundary (the kernels
 *    move 16-byte chunks); the partition entry point needs element
 *    alignment only.
 *  - Every call that launches work is asynchronous on `stream` (a
 *    hipStream_t, NULL = the default stream); host-side argument checks are
 *    synchronous and return before anything is launched.
 *  - Return value: SM_OK (0) or a negative sm_status; sm_last_error() gives
 *    a message for the last failing call of the calling thread.  No C++
 *    exception crosses this interface.
 *  - Inputs must be non-decreasing under the key order (Section 2, problem
 *    statement).  This is checked only when options.validate is set.
 */
#ifndef STABLEMERGE_H
#define STABLEMERGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef SM_API
#define SM_API __attribute__((visibility("default")))
#endif

typedef enum {
    SM_INT32 = 0,
    SM_UINT32 = 1,
    SM_UINT64 = 2,
    SM_INT64 = 3,
    SM_FLOAT32 = 4,
    SM_FLOAT64 = 5
} sm_dtype;

typedef enum {
    SM_OK = 0,
    SM_ERR_ARG = -1,        /* bad size, NULL pointer, misalignment, bad option */
    SM_ERR_DTYPE = -2,      /* unknown key type */
    SM_ERR_ALIAS = -3,      /* an output range overlaps an input range */
    SM_ERR_WORKSPACE = -4,  /* workspace missing or smaller than required */
    SM_ERR_HIP = -5,        /* a HIP runtime call or kernel launch failed */
    SM_ERR_UNSORTED = -6    /* validate was set and an input is not sorted */
} sm_status;

/*
 * Tuning and checking options; a NULL pointer or a zero field means "choose".
 *  p_a, p_b   number of blocks of A and of B (Section 2, block decomposition).
 *             0 = ceil(len / tile).  Forcing them reproduces the paper's
 *             partition for a given p; the two may differ.
 *  tile       block length in elements when p_a / p_b are 0 (1..65536; a
 *             subproblem of up to 2 * tile elements must fit one
 *             workgroup's LDS, else SM_ERR_ARG).  Forced p_a / p_b whose
 *             subproblems exceed 2 * tile are split again with this tile.
 *  validate   nonzero: first check that A and B are non-decreasing (one extra
 *             read of the keys and a synchronisation with the host).
 *  run        stable_merge_sort only: length of the runs sorted inside one
 *             workgroup before the merge passes; 256, 512, 1024, 2048, or
 *             4096 for 32-bit keys (0 = 512).
 *  descending stable_merge, stable_merge_batched and the two sorts: nonzero
 *             orders keys from largest to smallest (inputs non-increasing,
 *             ties as in ascending order: A before B, input order within a
 *             source).  Same workspace, same speed: the kernels are
 *             compiled for both orders.
 *  reserved   must be zero: calls reject anything else with SM_ERR_ARG and
 *             the workspace queries return 0.
 */
typedef struct {
    int64_t p_a;
    int64_t p_b;
    int32_t tile;
    int32_t validate;
    int32_t run;
    int32_t descending;
    int32_t reserved[4];
} sm_options;

/* Message describing the last non-OK status returned on this thread. */
SM_API const char *sm_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
SM_API int sm_version(void);

/*
 * Bytes of device workspace stable_merge needs for these arguments: the two
 * cross-rank arrays of p_a + 1 and p_b + 1 int64 entries (Section 2, the
 * synchronisation remark), a status word, one 32-byte descriptor per
 * subproblem and, when forced block counts make subproblems larger than one
 * workgroup stages, the state of their second-level split.  Returns 0 on
 * bad arguments.
 */
SM_API size_t stable_merge_workspace_bytes(int64_t n, int64_t m, int dtype, int has_payload,
                                    const sm_options *opt);

/*
 * Stable merge of A = keys[0, n) and B = keys[n, n + m) into out_keys[0, n + m)
 * (Section 2, Steps 1-4).  If payloads is not NULL, payloads[k] travels with
 * keys[k] into out_payloads; payloads and out_payloads are both NULL or both
 * non-NULL.  On equal keys every A element precedes every B element, and
 * each source keeps its order.  n = 0 or m = 0 is valid; m > n is valid (the
 * arrays are never swapped, which would change the tie order).
 * Outputs must not overlap inputs (SM_ERR_ALIAS).  ws must hold at least
 * stable_merge_workspace_bytes() bytes of device memory (SM_ERR_WORKSPACE).
 * The result does not depend on p_a, p_b or tile: a stable merge is unique.
 */
SM_API int stable_merge(const void *keys, const uint32_t *payloads, int64_t n, int64_t m,
                 void *out_keys, uint32_t *out_payloads, int dtype,
                 void *ws, size_t ws_bytes, const sm_options *opt, void *stream);

/*
 * Addition for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * stable_merge without a workspace argument.  Same arguments, result and
 * errors as stable_merge, minus ws / ws_bytes.  Its cross ranks and
 * subproblem descriptors live in a fixed scratch array of
 * SM_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on, from its first call there until the process ends.  The call
 * allocates nothing (no hipMalloc, no hipFree, no allocating library call).
 *   - A merge whose stable_merge_workspace_bytes() exceeds the limit returns
 *     SM_ERR_WORKSPACE before any launch (use stable_merge, or a larger
 *     tile).  The default tile needs about 9.1 MB for n = m = 2^28.
 *   - opt->validate is rejected (SM_ERR_ARG): it needs a host read-back.
 *   - Every call on one device shares that device's scratch array, and the
 *     array keeps the last call's contents (nothing in it has to start at
 *     zero).  Calls that overlap on one device -- on two streams, or from
 *     two host threads without ordering -- race on it and give undefined
 *     results; calls ordered on one stream are safe.
 *   - The device is the current HIP device; stream must belong to it.
 */
#define SM_NOALLOC_SCRATCH_BYTES (16u << 20)
SM_API int stable_merge_noalloc(const void *keys, const uint32_t *payloads, int64_t n, int64_t m,
                 void *out_keys, uint32_t *out_payloads, int dtype,
                 const sm_options *opt, void *stream);

/*
 * Steps 1 and 2 alone (Section 2): xbar[i] = rank_low(A[x_i], B) for
 * 0 <= i < p_a with xbar[p_a] = m, and ybar[j] = rank_high(B[y_j], A) for
 * 0 <= j < p_b with ybar[p_b] = n, where x_i and y_j are the block starts of
 * the paper's block decomposition.  A block that is empty (len < p) starts at
 * the +inf sentinel: its cross rank is m (resp. n).  xbar holds p_a + 1 and
 * ybar p_b + 1 device int64 entries.  p_a, p_b >= 1.
 */
SM_API int stable_merge_partition(const void *keys, int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                           int dtype, int64_t *xbar, int64_t *ybar, void *stream);

/*
 * Steps 3 and 4 alone (Section 2): given the cross ranks xbar[0..p_a] and
 * ybar[0..p_b] that stable_merge_partition wrote for the same keys, n, m,
 * p_a, p_b and dtype, every block's processing element picks its case
 * (a)-(e) and merges its subproblem into out_keys (and out_payloads).
 * stable_merge_partition followed by this call on one stream is exactly
 * stable_merge with forced p_a, p_b; the stream order is the method's single
 * synchronisation.  Subproblems larger than one workgroup stages (few
 * blocks) are split again by the same method.  Same aliasing, alignment and
 * payload rules as stable_merge.  ws (device, 16-byte aligned) receives the
 * p_a + p_b subproblem descriptors (and the state of the second-level split)
 * and must hold stable_merge_pieces_workspace_bytes() bytes
 * (SM_ERR_WORKSPACE otherwise).
 */
SM_API int stable_merge_pieces(const void *keys, const uint32_t *payloads, int64_t n, int64_t m,
                               int64_t p_a, int64_t p_b, const int64_t *xbar, const int64_t *ybar,
                               void *out_keys, uint32_t *out_payloads, int dtype,
                               void *ws, size_t ws_bytes, void *stream);

/* Device workspace bytes of stable_merge_pieces (0 on bad arguments). */
SM_API size_t stable_merge_pieces_workspace_bytes(int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                                                  int dtype, int has_payload);

/*
 * Many independent stable merges in one launch sequence (Section 3: the
 * merge running on many pairs at once).  Pair k occupies
 * keys[offsets[k], offsets[k + 1]); its first n_a[k] elements are its A and
 * the rest its B, and its merge is written to out_keys[offsets[k],
 * offsets[k + 1]) (payloads alike).  offsets holds count + 1 and n_a count
 * device int64 entries, with 0 <= offsets[k] <= offsets[k + 1] <= total,
 * 0 <= n_a[k] <= offsets[k + 1] - offsets[k] and pairs of fewer than 2^30
 * elements.  A pair that breaks these rules is skipped (its output range is
 * left unwritten); with options.validate set the call checks the rules and
 * the sortedness of every A and B first and returns SM_ERR_ARG or
 * SM_ERR_UNSORTED.  Pairs of any sizes may be mixed: a pair that one
 * workgroup stages is merged whole, a larger pair is split by the method
 * with blocks of options.tile elements.  The host never reads offsets or
 * n_a (except to validate), so the call can be captured in a graph.  keys,
 * out_keys and payloads follow the rules of stable_merge; ws must hold
 * stable_merge_batched_workspace_bytes() bytes.
 */
SM_API int stable_merge_batched(const void *keys, const uint32_t *payloads,
                                const int64_t *offsets, const int64_t *n_a, int64_t count,
                                int64_t total, void *out_keys, uint32_t *out_payloads, int dtype,
                                void *ws, size_t ws_bytes, const sm_options *opt, void *stream);

/* Device workspace bytes of stable_merge_batched (0 on bad arguments);
 * options.tile is used, p_a and p_b are ignored. */
SM_API size_t stable_merge_batched_workspace_bytes(int64_t count, int64_t total, int dtype,
                                                   int has_payload, const sm_options *opt);

/*
 * Stable merge sort (Section 3: sorting by repeated stable merging).
 * Sorts keys[0, N) into out_keys[0, N); payloads (optional) travel with
 * their keys.  Equal keys keep their input order.  Runs of options.run
 * elements are first sorted inside one workgroup each (by cross ranks with
 * blocks of one element), then ceil(log2(N / run)) passes each merge pairs
 * of neighbouring runs with the stable merge.  out_keys may be keys itself
 * (in-place sort; likewise out_payloads and payloads), any other overlap is
 * SM_ERR_ALIAS.  0 <= N < 2^31.  ws must hold
 * stable_merge_sort_workspace_bytes() bytes: a second buffer of N keys (and
 * N payloads) for the passes to alternate with, plus the merge state.
 */
SM_API int stable_merge_sort(const void *keys, const uint32_t *payloads, int64_t N,
                             void *out_keys, uint32_t *out_payloads, int dtype,
                             void *ws, size_t ws_bytes, const sm_options *opt, void *stream);

/*
 * The merge sort's first phase alone (Section 3: the blocks are sorted
 * first, then merged): every run keys[k * run, min((k + 1) * run, N)) is
 * stably sorted on its own into the same range of out_keys, payloads
 * (optional) travelling with their keys.  run is 256, 512, 1024, 2048 or,
 * for 32-bit keys, 4096.  out_keys may be keys itself (in place; likewise
 * the payloads), any other overlap is SM_ERR_ALIAS.  0 <= N <= 2^38.  No
 * workspace; asynchronous on `stream`.
 */
SM_API int stable_merge_sort_runs(const void *keys, const uint32_t *payloads, int64_t N,
                                  void *out_keys, uint32_t *out_payloads, int dtype, int run,
                                  void *stream);

/*
 * Segmented stable sort: every segment keys[offsets[s], offsets[s + 1]) is
 * sorted on its own, payloads (optional) travelling with their keys and
 * equal keys keeping their input order, as stable_merge_sort would sort it
 * alone.  offsets holds count + 1 device int64 entries running from 0 to N
 * without decreasing; no segment may be longer than max_len (a host-side
 * bound, which fixes the number of merge passes: ceil(log2(max_len / run))).
 * Runs start at segment starts, and every merge pass pairs runs within a
 * segment.  The host never reads offsets, so the call can be captured in a
 * graph; with options.validate set it checks offsets and max_len first and
 * returns SM_ERR_ARG (otherwise a violation leaves the output undefined).
 * 1 <= count < 2^31, 0 <= max_len <= N < 2^31; buffers, aliasing and
 * options.run as for stable_merge_sort; ws must hold
 * stable_merge_segmented_sort_workspace_bytes() bytes.
 */
SM_API int stable_merge_segmented_sort(const void *keys, const uint32_t *payloads,
                                       const int64_t *offsets, int64_t count, int64_t N,
                                       int64_t max_len, void *out_keys, uint32_t *out_payloads,
                                       int dtype, void *ws, size_t ws_bytes,
                                       const sm_options *opt, void *stream);

/* Device workspace bytes of stable_merge_segmented_sort (0 on bad arguments). */
SM_API size_t stable_merge_segmented_sort_workspace_bytes(int64_t count, int64_t N,
                                                          int64_t max_len, int dtype,
                                                          int has_payload,
                                                          const sm_options *opt);

/* Device workspace bytes of stable_merge_sort (0 on bad arguments). */
SM_API size_t stable_merge_sort_workspace_bytes(int64_t N, int dtype, int has_payload,
                                                const sm_options *opt);

/* ------------------------------------------------------------------------
 * Learned cross ranks (an addition to the paper).  Steps 1-2 find every
 * cross rank by binary search.  These calls let a small network predict
 * where each rank lies and a bounded exponential search finish the job;
 * the ranks, and so every merge, stay exactly those of the paper.
 *
 * The network models the cumulative distribution of a sorted array X:
 * phi(key) = log2(u + 1) / bits (u the key's position in its order as an
 * unsigned integer: signed keys with the sign bit flipped, float keys mapped
 * through totalOrder; bits = the key width), h = ReLU(W1 phi + b1)
 * with 32 hidden units, y = w2 . h + b2 ~ rank / len(X).  Parameters are 97
 * device floats: W1[0:32], b1[32:64], w2[64:96], b2[96].  All arithmetic is
 * FP32.  A prediction is clamp(rint(y * len), 0, len).
 * ------------------------------------------------------------------------ */
#define SM_MLP_HIDDEN 32
#define SM_MLP_PARAMS 97
#define SM_HIST_BINS 65   /* error histogram: bin 32 = exact, 32 +- (1 + floor(log2 |e|)) */

/* Device workspace of sm_mlp_grad for `samples` samples (0 on bad arguments). */
SM_API size_t sm_mlp_grad_workspace_bytes(int64_t samples);

/*
 * Forward and backward pass over a sample: grad[97] = d loss / d params and
 * *loss (optional, may be NULL) for loss = mean over k of (y(keys[k]) -
 * target[k])^2, with the ReLU derivative taken as 0 at 0.  keys (dtype) and
 * target (float, normalised ranks) hold `samples` device entries.  The
 * reduction order is fixed: the same inputs give the same bits.
 */
SM_API int sm_mlp_grad(const float *params, const void *keys, const float *target,
                       int64_t samples, int dtype, float *grad, float *loss,
                       void *ws, size_t ws_bytes, void *stream);

/*
 * One Adam step (Kingma and Ba, 2015) in place: m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, params -= lr m / (1 - b1^step) /
 * (sqrt(v / (1 - b2^step)) + eps).  params, m, v, grad: 97 device floats.
 */
SM_API int sm_mlp_adam(float *params, float *m, float *v, const float *grad, int64_t step,
                       float lr, float beta1, float beta2, float eps, void *stream);

/*
 * Interpolating knot initialisation from a sorted sample of `samples` query
 * keys and their targets: hidden unit k is ReLU(phi - c_k) with c_k the
 * feature of sample i_k = floor((k + 1/2) samples / 32) (W1 = 1, b1 = -c_k),
 * and the output layer makes the network the piecewise-linear interpolant of
 * the points (c_k, target[i_k]): b2 = target[i_0], w2[k] = s_k - s_{k-1} with
 * s_k the slope between knots k and k + 1 (0 if they are closer than 1e-6;
 * s_31 = 0).  samples = 0 gives all-zero parameters.
 */
SM_API int sm_mlp_init(const void *sorted_keys, const float *target, int64_t samples, int dtype,
                       float *params, void *stream);

/* rhat[i] = clamp(rint(y(keys[i]) * len), 0, len) for q device keys. */
SM_API int sm_mlp_predict(const float *params, const void *keys, int64_t q, int dtype,
                          int64_t len, int64_t *rhat, void *stream);

/* Device workspace of sm_rank_model_train (0 on bad arguments). */
SM_API size_t sm_rank_model_workspace_bytes(int64_t samples, int dtype);

/*
 * Trains a model of the sorted X[0, len) for queries from the sorted
 * Q[0, q_len): draws `samples` queries by stratified sampling (one uniform
 * draw in each of `samples` equal slices of Q, from `seed`), computes their
 * exact ranks in X by the binary search of Steps 1-2 (rank_high if is_high,
 * else rank_low), initialises as sm_mlp_init on that sample, then runs
 * `steps` full-batch
 * Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) on the mean squared error of
 * the normalised rank, the learning rate decaying from lr to lr / 100 on a
 * cosine.  Writes params (97 device floats) and, if loss is not NULL, the
 * final loss (device float; its square root times len is the RMS rank
 * error on the sample in elements).  len, q_len >= 1.
 */
SM_API int sm_rank_model_train(const void *X, int64_t len, const void *Q, int64_t q_len, int dtype,
                               int is_high, int64_t samples, int64_t steps, float lr,
                               uint64_t seed, float *params, float *loss,
                               void *ws, size_t ws_bytes, void *stream);

/*
 * Exact ranks of q query keys in the sorted X[0, len) from given guesses
 * (device int64, clamped to [0, len]): rank_low (is_high = 0) or rank_high.
 * The search probes the guess g, then X[g +- step0], X[g +- 2 step0], ...
 * away from g until the rank is bracketed (or the array ends), then bisects
 * the bracket [lo, hi] of possible ranks, each read splitting it at the
 * number m in (lo, hi] with the most trailing zero bits (the rank is >= m
 * exactly when X[m - 1] is below x, or not above it for rank_high); a step
 * beyond `window` abandons the walk for the same bisection of [0, len].
 * ranks[i] (int64) is always exact; probes[i] (int32: reads of X) and
 * fallback[i] (int32 0/1) are optional (NULL to skip).
 * step0 >= 1, 0 <= window <= 2^40.
 */
SM_API int stable_merge_rank_search(const void *X, int64_t len, const void *queries, int64_t q,
                                    int dtype, int is_high, const int64_t *guess, int64_t step0,
                                    int64_t window, int64_t *ranks, int32_t *probes,
                                    int32_t *fallback, void *stream);

/*
 * Steps 1 and 2 with learned starting points: writes exactly what
 * stable_merge_partition writes (xbar[p_a + 1], ybar[p_b + 1]).  An A block
 * start x_i < n searches B from model_b's prediction with initial step
 * step0_a, a B block start searches A from model_a's prediction with
 * step0_b (both with the given window, as in stable_merge_rank_search).
 * For every search, hist[bin(predicted - exact)] += 1 (SM_HIST_BINS device
 * uint64), counters[0] += 1 (searches), counters[1] += fallbacks,
 * counters[2] += probes (reads of A or B); the caller zeroes them first.
 */
SM_API int stable_merge_partition_learned(const void *keys, int64_t n, int64_t m, int64_t p_a,
                                          int64_t p_b, int dtype, const float *model_b,
                                          const float *model_a, int64_t step0_a, int64_t step0_b,
                                          int64_t window, int64_t *xbar, int64_t *ybar,
                                          uint64_t *hist, uint64_t *counters, void *stream);

/*
 * The whole stable merge with learned cross ranks: the partition of
 * stable_merge_partition_learned with blocks of `block` elements per side
 * (p_a = ceil(n / block), p_b = ceil(m / block), at least 1 each), then
 * Steps 3-4 as stable_merge_pieces.  The output is the unique stable merge,
 * byte for byte what stable_merge writes, whatever the models predict.
 * keys, payloads and outputs follow the rules of stable_merge; model_b /
 * model_a, step0_a / step0_b, window, hist and counters those of
 * stable_merge_partition_learned (the caller zeroes hist and counters).
 * 1 <= block <= 2^20.  ws must hold stable_merge_learned_workspace_bytes()
 * bytes (the cross ranks, then the merge's workspace).
 */
SM_API int stable_merge_learned(const void *keys, const uint32_t *payloads, int64_t n, int64_t m,
                                void *out_keys, uint32_t *out_payloads, int dtype,
                                const float *model_b, const float *model_a, int64_t step0_a,
                                int64_t step0_b, int64_t block, int64_t window, uint64_t *hist,
                                uint64_t *counters, void *ws, size_t ws_bytes, void *stream);

/* Device workspace bytes of stable_merge_learned (0 on bad arguments). */
SM_API size_t stable_merge_learned_workspace_bytes(int64_t n, int64_t m, int64_t block, int dtype,
                                                   int has_payload);

/*
 * stable_merge_sort with learned cross ranks in every merge pass (an
 * addition to the paper; the learned partition of stable_merge_learned,
 * amortised over the passes).  The runs of every pass are drawn from the
 * same keys, so one model serves them all: `model` (97 device floats, the
 * layout of sm_mlp_grad) maps a key to its normalised rank in a sorted
 * sample of the keys.  A cross rank in a run of len elements is searched
 * from the guess model(key) * len, stepping away by the largest power of
 * two <= max(1, step_frac * len) and doubling before the bisection, so
 * step_frac is the model's relative rank error (0 <= step_frac <= 1).
 * The output is byte for byte that of stable_merge_sort whatever the model
 * predicts; only the number of probes changes.  counters (device, may be
 * NULL) accumulate [searches, probes] over all passes.  Ascending order
 * only (opt->descending is rejected); workspace and other arguments as
 * stable_merge_sort (stable_merge_sort_workspace_bytes).
 */
SM_API int stable_merge_sort_learned(const void *keys, const uint32_t *payloads, int64_t N,
                                     void *out_keys, uint32_t *out_payloads, int dtype,
                                     const float *model, float step_frac, uint64_t *counters,
                                     void *ws, size_t ws_bytes, const sm_options *opt,
                                     void *stream);

/* ------------------------------------------------------------------------
 * Rank-model handles (an addition to the paper, beside the plain 97-float
 * arrays above).  A handle keeps a network together with what it models:
 * the key type, which rank it predicts (rank_low, as for A's block starts
 * searched in B, or rank_high, as for B's block starts searched in A), its
 * feature kind and the length of the array it was trained on, so that a
 * trained model can be saved, loaded and reused as one unit.  The library owns a handle and its 98 device floats (the 97
 * parameters, then the last training loss); everything else stays the
 * caller's.  Handles are not thread-safe: one thread at a time per handle.
 * ------------------------------------------------------------------------ */
typedef struct sm_predictor sm_predictor;

/* Size of a saved model: a 40-byte header (magic "SMRM", format version 1,
 * key type, is_high, feature kind 1 = log2(u + 1) / bits, hidden width 32,
 * parameter count 97, the last loss as float, the trained array length as
 * int64), the 97 parameters as little-endian floats, and an FNV-1a checksum
 * of everything before it. */
#define SM_PREDICTOR_BLOB_BYTES 432

/*
 * Allocates a handle for keys of `dtype` that predicts rank_high (is_high
 * != 0) or rank_low positions; its parameters start at zero (a constant
 * prediction of rank 0) and its loss at 1.  Allocates device memory on the
 * current device (synchronous).  *out is NULL on failure.
 */
SM_API int sm_predictor_create(sm_predictor **out, int dtype, int is_high);

/* Frees a handle and its device memory; NULL is a no-op. */
SM_API int sm_predictor_destroy(sm_predictor *p);

/*
 * sm_rank_model_train into the handle: trains a model of the sorted
 * X[0, len) for queries from Q[0, q_len) with the handle's key type and
 * rank kind; the loss is kept in the handle.  Asynchronous on `stream`;
 * workspace as sm_rank_model_train (sm_rank_model_workspace_bytes).
 */
SM_API int sm_predictor_train(sm_predictor *p, const void *X, int64_t len, const void *Q,
                              int64_t q_len, int64_t samples, int64_t steps, float lr,
                              uint64_t seed, void *ws, size_t ws_bytes, void *stream);

/* The handle's 97 device parameters, for the calls that take a model
 * (stable_merge_learned, stable_merge_partition_learned, ...); NULL for an
 * invalid handle.  Valid until sm_predictor_destroy. */
SM_API const float *sm_predictor_params(const sm_predictor *p);

/* Key type, rank kind, trained array length and last loss of a handle (any
 * output pointer may be NULL).  Reading the loss waits for the handle's
 * last training run. */
SM_API int sm_predictor_info(const sm_predictor *p, int *dtype, int *is_high,
                             int64_t *trained_len, float *loss);

/*
 * Writes the SM_PREDICTOR_BLOB_BYTES-byte saved form of a handle into the
 * host buffer host_buf (bytes >= SM_PREDICTOR_BLOB_BYTES, else SM_ERR_ARG).
 * Waits for the handle's last training run (synchronous).
 */
SM_API int sm_predictor_save(const sm_predictor *p, void *host_buf, size_t bytes);

/*
 * Creates a handle from a saved form: checks the magic, the version, the
 * checksum and that the network shape and feature kind are the ones this
 * library evaluates (SM_ERR_ARG otherwise, SM_ERR_DTYPE for an unknown key
 * type), then uploads the parameters to the current device (synchronous).
 * A loaded handle predicts exactly what the saved one did.
 */
SM_API int sm_predictor_load(sm_predictor **out, const void *host_buf, size_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* STABLEMERGE_H */
