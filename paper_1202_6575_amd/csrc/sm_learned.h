// sm_learned.h -- host side of the learned cross ranks (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sm {

constexpr int kMlpHidden = 32;
constexpr int kMlpParams = 3 * kMlpHidden + 1;  // W1[32], b1[32], w2[32], b2
constexpr int kHistBins = 65;
constexpr int kHistCenter = 32;

// Workspace of the forward + backward pass over S samples (block partial sums).
size_t mlp_grad_ws_bytes(int64_t S);
int64_t mlp_grad_blocks(int64_t S);

hipError_t launch_mlp_grad(int dtype, const float* P, const void* keys, const float* target,
                           int64_t S, float* grad, float* loss, void* ws, hipStream_t st);
hipError_t launch_mlp_adam(float* P, float* M, float* V, const float* G, int64_t step, float lr,
                           float b1, float b2, float eps, hipStream_t st);
hipError_t launch_mlp_init(int dtype, const void* sorted_keys, const float* target, int64_t S,
                           float* P, hipStream_t st);
hipError_t launch_mlp_predict(int dtype, const float* P, const void* keys, int64_t q, int64_t len,
                              int64_t* rhat, hipStream_t st);
hipError_t launch_rank_search(int dtype, const void* X, int64_t len, const void* queries, int64_t q,
                              int is_high, const int64_t* guess, int64_t step0, int64_t window,
                              int64_t* ranks, int32_t* probes, int32_t* fallback, hipStream_t st);
hipError_t launch_learned_partition(int dtype, const void* keys, int64_t n, int64_t m, int64_t p_a,
                                    int64_t p_b, const float* model_b, const float* model_a,
                                    int64_t step0_a, int64_t step0_b, int64_t window, int64_t* xbar,
                                    int64_t* ybar, uint64_t* hist, uint64_t* counters,
                                    hipStream_t st);

// Workspace of training: the sampled keys and targets, the gradient
// partial sums, the gradient and the two Adam moments.
struct RankModelLayout {
    size_t off_keys, off_target, off_partial, off_grad, off_m, off_v, bytes;
};
RankModelLayout rank_model_layout(int64_t S, int dtype);

hipError_t launch_rank_model_train(int dtype, const void* X, int64_t len, const void* Q,
                                   int64_t q_len, int is_high, int64_t S, int64_t steps, float lr,
                                   uint64_t seed, float* P, float* loss, char* ws,
                                   const RankModelLayout& L, hipStream_t st);

}  // namespace sm
