// sm_learned.hip -- learned cross ranks (an addition to the paper's Steps 1-2).
//
// The paper finds every cross rank by binary search (Section 2, Steps 1-2).
// Here a 1 -> 32 (ReLU) -> 1 network models the cumulative distribution of
// the array searched, mapping a key to its normalised rank; its prediction
// is the starting point of a bounded exponential search that ends at the
// exact rank_low / rank_high, with the plain binary search as the fallback
// when the search would have to move farther than a window.  The network
// only decides where the search starts, never the result.
//
// Kernels: training-set sampling (exact ranks by the method's own binary
// search), knot initialisation, forward + backward over a sample with a
// fixed-order reduction (bitwise reproducible), Adam, prediction, the
// bounded search from given guesses, and the learned partition (Steps 1-2
// with predicted starting points, an error histogram and fallback / probe
// counters).
#include "sm_device.h"
#include "sm_launch.h"
#include "sm_learned.h"
#include "sm_learned_dev.h"

namespace sm {

namespace {

constexpr int H = kMlpHidden;
constexpr int NP = kMlpParams;
constexpr int NACC = NP + 1;  // the gradient and the squared-error sum
constexpr int kGradThreads = 256;

// Histogram bin of a rank error e = predicted - exact: 32 for 0, 32 + 1 +
// floor(log2 e) for e > 0 and 32 - 1 - floor(log2 -e) for e < 0, clipped
// to [0, 64].
__device__ __forceinline__ int error_bin(int64_t e) {
    if (e == 0) return kHistCenter;
    const uint64_t a = (uint64_t)(e < 0 ? -e : e);
    const int lg = 63 - __clzll((long long)a);
    int b = e > 0 ? kHistCenter + 1 + lg : kHistCenter - 1 - lg;
    return b < 0 ? 0 : (b > kHistBins - 1 ? kHistBins - 1 : b);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Training set: S queries drawn from the sorted Q by stratified sampling
// (sample k uniform in the k-th of S equal slices, so the sample is sorted),
// exact ranks in X by the plain binary search, targets r / len.
template <typename K>
__global__ __launch_bounds__(256) void rank_sample_kernel(const K* __restrict__ X, int64_t len,
                                                          const K* __restrict__ Q, int64_t q_len,
                                                          int is_high, int64_t S, uint64_t seed,
                                                          K* __restrict__ skeys,
                                                          float* __restrict__ target) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < S;
         k += (int64_t)gridDim.x * blockDim.x) {
        const double u = (double)(splitmix64(seed ^ (0x5851f42d4c957f2dull * (uint64_t)(k + 1))) >> 11) *
                         (1.0 / 9007199254740992.0);
        int64_t idx = (int64_t)(((double)k + u) * (double)q_len / (double)S);
        idx = idx < 0 ? 0 : (idx >= q_len ? q_len - 1 : idx);
        const K x = Q[idx];
        const int64_t r = is_high ? rank_high<K, int64_t>(X, len, x) : rank_low<K, int64_t>(X, len, x);
        skeys[k] = x;
        target[k] = (float)((double)r / (double)len);
    }
}

// Interpolating knot initialisation: hinge k at c_k = phi of sample
// i_k = floor((k + 1/2) S / 32) of the sorted sample (W1 = 1, b1 = -c_k), and
// an output layer that makes the network the piecewise-linear interpolant of
// the points (c_k, t_k): b2 = t_0, w2[k] = s_k - s_{k-1}, s_k the slope from
// knot k to knot k + 1 (0 for knots closer than 1e-6, and s_31 = 0).
template <typename K>
__global__ void mlp_init_kernel(const K* __restrict__ sorted_keys, const float* __restrict__ target,
                                int64_t S, float* __restrict__ P) {
    if (threadIdx.x != 0) return;
    if (S <= 0) {
        for (int j = 0; j < NP; ++j) P[j] = 0.0f;
        return;
    }
    float c_prev = 0.0f, t_prev = 0.0f, s_prev = 0.0f;
    for (int k = 0; k < H; ++k) {
        int64_t idx = (int64_t)(((double)k + 0.5) * (double)S / (double)H);
        idx = idx >= S ? S - 1 : idx;
        const float c = feature(sorted_keys[idx]);
        const float t = target[idx];
        P[k] = 1.0f;
        P[H + k] = -c;
        if (k == 0) {
            P[3 * H] = t;
        } else {
            const float gap = c - c_prev;
            const float s = gap > 1e-6f ? (t - t_prev) / gap : 0.0f;
            P[2 * H + k - 1] = s - s_prev;
            s_prev = s;
        }
        c_prev = c;
        t_prev = t;
    }
    P[2 * H + H - 1] = -s_prev;  // s_31 = 0: flat past the last knot
}

// Deterministic wave sum: butterfly over the 64 lanes in a fixed order.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Partial sums of d(loss * S)/dparams and of the squared errors over the
// samples of one block: dy = 2 (y - t); dw2_k += dy h_k; db2 += dy;
// dW1_k += dy w2_k [pre_k > 0] phi; db1_k += dy w2_k [pre_k > 0].
// Sample k goes to block k / per_block, thread (k % per_block) % 256: a
// fixed assignment and a fixed reduction tree, so the sums are bitwise
// reproducible.
template <typename K>
__global__ __launch_bounds__(kGradThreads) void mlp_grad_kernel(const float* __restrict__ P,
                                                                const K* __restrict__ keys,
                                                                const float* __restrict__ target,
                                                                int64_t S, int64_t per_block,
                                                                float* __restrict__ partial) {
    __shared__ float red[kGradThreads / 64][NACC];
    float acc[NACC];
#pragma unroll
    for (int j = 0; j < NACC; ++j) acc[j] = 0.0f;
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = b0 + per_block < S ? b0 + per_block : S;
    for (int64_t k = b0 + threadIdx.x; k < b1; k += kGradThreads) {
        const float phi = feature(keys[k]);
        float pre[H];
        float y = P[3 * H];
#pragma unroll
        for (int j = 0; j < H; ++j) {
            pre[j] = fmaf(P[j], phi, P[H + j]);
            y = fmaf(P[2 * H + j], fmaxf(pre[j], 0.0f), y);
        }
        const float d = y - target[k];
        const float dy = 2.0f * d;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const float h = fmaxf(pre[j], 0.0f);
            acc[2 * H + j] = fmaf(dy, h, acc[2 * H + j]);
            const float dh = pre[j] > 0.0f ? dy * P[2 * H + j] : 0.0f;
            acc[j] = fmaf(dh, phi, acc[j]);
            acc[H + j] += dh;
        }
        acc[3 * H] += dy;
        acc[NP] = fmaf(d, d, acc[NP]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < NACC; ++j) {
        const float s = wave_sum(acc[j]);
        if (lane == 0) red[wave][j] = s;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < NACC; j += kGradThreads) {
        float s = red[0][j];
#pragma unroll
        for (int w = 1; w < kGradThreads / 64; ++w) s += red[w][j];
        partial[(int64_t)blockIdx.x * NACC + j] = s;
    }
}

// grad[j] = (sum over blocks) / S; loss = squared-error sum / S.  One
// workgroup per entry j: thread t adds the partial sums of blocks t, t + 256,
// ... in order, then a fixed butterfly and a fixed LDS sum combine the
// threads: the same inputs give the same bits.
__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(const float* __restrict__ partial,
                                                              int64_t blocks, int64_t S,
                                                              float* __restrict__ grad,
                                                              float* __restrict__ loss) {
    __shared__ float red[4];
    const int j = blockIdx.x;
    float s = 0.0f;
    for (int64_t b = threadIdx.x; b < blocks; b += 256) s += partial[b * NACC + j];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float tot = (red[0] + red[1]) + (red[2] + red[3]);
        const float v = S > 0 ? tot / (float)S : 0.0f;
        if (j < NP) grad[j] = v;
        else if (loss) *loss = v;
    }
}

// Adam (Kingma and Ba, 2015) with bias correction factors c1 = 1 / (1 - b1^t),
// c2 = 1 / (1 - b2^t) computed by the host.
__global__ void mlp_adam_kernel(float* __restrict__ P, float* __restrict__ M, float* __restrict__ V,
                                const float* __restrict__ G, float lr, float b1, float b2,
                                float eps, float c1, float c2) {
    const int j = threadIdx.x;
    if (j >= NP) return;
    const float g = G[j];
    const float m = b1 * M[j] + (1.0f - b1) * g;
    const float v = b2 * V[j] + (1.0f - b2) * g * g;
    M[j] = m;
    V[j] = v;
    P[j] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

__global__ void fill_f32_kernel(float* __restrict__ p, int n, float v) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

template <typename K>
__global__ __launch_bounds__(256) void mlp_predict_kernel(const float* __restrict__ P,
                                                          const K* __restrict__ keys, int64_t q,
                                                          int64_t len, int64_t* __restrict__ rhat) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q;
         i += (int64_t)gridDim.x * blockDim.x)
        rhat[i] = predict(P, feature(keys[i]), len);
}

template <typename K>
__global__ __launch_bounds__(256) void rank_search_kernel(
    const K* __restrict__ X, int64_t len, const K* __restrict__ Qk, int64_t q, int is_high,
    const int64_t* __restrict__ guess, int64_t step0, int64_t window, int64_t* __restrict__ ranks,
    int32_t* __restrict__ probes, int32_t* __restrict__ fallback) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q;
         i += (int64_t)gridDim.x * blockDim.x) {
        int np;
        bool fb;
        const int64_t r = is_high
                              ? bounded_search<K, true>(X, len, Qk[i], guess[i], step0, window, np, fb)
                              : bounded_search<K, false>(X, len, Qk[i], guess[i], step0, window, np, fb);
        ranks[i] = r;
        if (probes) probes[i] = np;
        if (fallback) fallback[i] = fb ? 1 : 0;
    }
}

// Steps 1-2 with predicted starting points: the same xbar / ybar as the
// plain partition.  Thread t <= p_a handles A's block start x_t (rank_low in
// B, network model_b), the others B's block starts (rank_high in A,
// network model_a).  Per workgroup an LDS histogram of predicted - exact
// and counts of searches, fallbacks and probes, added to the global ones.
template <typename K>
__global__ __launch_bounds__(256) void learned_partition_kernel(
    const K* __restrict__ keys, int64_t n, int64_t m, int64_t p_a, int64_t p_b,
    const float* __restrict__ model_b, const float* __restrict__ model_a, int64_t step0_a,
    int64_t step0_b, int64_t window, int64_t* __restrict__ xbar, int64_t* __restrict__ ybar,
    unsigned long long* __restrict__ hist, unsigned long long* __restrict__ counters) {
    __shared__ unsigned int sh[kHistBins];
    __shared__ unsigned long long sc[3];
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) sh[i] = 0;
    if (threadIdx.x < 3) sc[threadIdx.x] = 0;
    __syncthreads();
    const K* A = keys;
    const K* B = keys + n;
    const Blocks<int64_t> BA(n, p_a), BB(m, p_b);
    // counts of this thread's searches, summed per wave and per workgroup
    // before they reach the device counters (every search of the grid
    // adding to the same three words would serialise on them)
    unsigned long long c_searched = 0, c_fb = 0, c_probes = 0;
    const int64_t total = p_a + 1 + p_b + 1;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        bool searched = false, fb = false;
        int np = 0;
        int64_t err = 0;
        if (t <= p_a) {
            const int64_t xi = BA.start(t);
            int64_t r = m;
            if (xi < n) {
                const K x = A[xi];
                const int64_t g = predict(model_b, feature(x), m);
                r = bounded_search<K, false>(B, m, x, g, step0_a, window, np, fb);
                err = g - r;
                searched = true;
            }
            xbar[t] = r;
        } else {
            const int64_t j = t - (p_a + 1);
            const int64_t yj = BB.start(j);
            int64_t r = n;
            if (yj < m) {
                const K y = B[yj];
                const int64_t g = predict(model_a, feature(y), n);
                r = bounded_search<K, true>(A, n, y, g, step0_b, window, np, fb);
                err = g - r;
                searched = true;
            }
            ybar[j] = r;
        }
        if (searched) {
            atomicAdd(&sh[error_bin(err)], 1u);
            c_searched += 1;
            c_fb += fb ? 1 : 0;
            c_probes += (unsigned long long)np;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        c_searched += __shfl_xor(c_searched, o);
        c_fb += __shfl_xor(c_fb, o);
        c_probes += __shfl_xor(c_probes, o);
    }
    if ((threadIdx.x & 63) == 0) {
        if (c_searched) atomicAdd(&sc[0], c_searched);
        if (c_fb) atomicAdd(&sc[1], c_fb);
        if (c_probes) atomicAdd(&sc[2], c_probes);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHistBins; i += blockDim.x)
        if (sh[i]) atomicAdd(&hist[i], (unsigned long long)sh[i]);
    if (threadIdx.x < 3 && sc[threadIdx.x]) atomicAdd(&counters[threadIdx.x], sc[threadIdx.x]);
}


unsigned grid_for(int64_t items, int64_t cap_blocks) {
    int64_t g = (items + 255) / 256;
    if (g > cap_blocks) g = cap_blocks;
    return (unsigned)(g < 1 ? 1 : g);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int64_t mlp_grad_blocks(int64_t S) {
    // about 8 samples per thread (the per-block reduction of 98 sums costs
    // about as much as a few samples), at most 4096 blocks
    int64_t blocks = (S + kGradThreads * 8 - 1) / (kGradThreads * 8);
    if (blocks > 4096) blocks = 4096;
    return blocks < 1 ? 1 : blocks;
}

size_t mlp_grad_ws_bytes(int64_t S) { return align256((size_t)mlp_grad_blocks(S) * NACC * 4); }

hipError_t launch_mlp_grad(int dtype, const float* P, const void* keys, const float* target,
                           int64_t S, float* grad, float* loss, void* ws, hipStream_t st) {
    const int64_t blocks = mlp_grad_blocks(S);
    const int64_t per_block = (S + blocks - 1) / blocks;
    float* partial = static_cast<float*>(ws);
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        mlp_grad_kernel<K><<<(unsigned)blocks, kGradThreads, 0, st>>>(
            P, static_cast<const K*>(keys), target, S, per_block > 0 ? per_block : 1, partial);
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    mlp_grad_reduce_kernel<<<NACC, 256, 0, st>>>(partial, blocks, S, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* P, float* M, float* V, const float* G, int64_t step, float lr,
                           float b1, float b2, float eps, hipStream_t st) {
    const double c1 = 1.0 / (1.0 - pow((double)b1, (double)step));
    const double c2 = 1.0 / (1.0 - pow((double)b2, (double)step));
    mlp_adam_kernel<<<1, 128, 0, st>>>(P, M, V, G, lr, b1, b2, eps, (float)c1, (float)c2);
    return hipGetLastError();
}

hipError_t launch_mlp_init(int dtype, const void* sorted_keys, const float* target, int64_t S,
                           float* P, hipStream_t st) {
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        mlp_init_kernel<K><<<1, 64, 0, st>>>(static_cast<const K*>(sorted_keys), target, S, P);
    });
    return hipGetLastError();
}

hipError_t launch_mlp_predict(int dtype, const float* P, const void* keys, int64_t q, int64_t len,
                              int64_t* rhat, hipStream_t st) {
    if (q <= 0) return hipSuccess;
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        mlp_predict_kernel<K><<<grid_for(q, 8192), 256, 0, st>>>(P, static_cast<const K*>(keys), q,
                                                                  len, rhat);
    });
    return hipGetLastError();
}

hipError_t launch_rank_search(int dtype, const void* X, int64_t len, const void* queries, int64_t q,
                              int is_high, const int64_t* guess, int64_t step0, int64_t window,
                              int64_t* ranks, int32_t* probes, int32_t* fallback, hipStream_t st) {
    if (q <= 0) return hipSuccess;
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        rank_search_kernel<K><<<grid_for(q, 8192), 256, 0, st>>>(
            static_cast<const K*>(X), len, static_cast<const K*>(queries), q, is_high, guess, step0,
            window, ranks, probes, fallback);
    });
    return hipGetLastError();
}

hipError_t launch_learned_partition(int dtype, const void* keys, int64_t n, int64_t m, int64_t p_a,
                                    int64_t p_b, const float* model_b, const float* model_a,
                                    int64_t step0_a, int64_t step0_b, int64_t window, int64_t* xbar,
                                    int64_t* ybar, uint64_t* hist, uint64_t* counters,
                                    hipStream_t st) {
    // a grid-stride loop over the p_a + 1 + p_b + 1 cross ranks with 64
    // workgroups per CU: at 2^25 ranks, 16 or fewer per CU leave the device
    // short of searches in flight, and one rank per thread (512 per CU)
    // spends the time on the per-workgroup counter atomics (measured 1.26,
    // 1.19 and 1.75 ms)
    const unsigned grid = grid_for(p_a + p_b + 2, (int64_t)device_cu_count() * 64);
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        learned_partition_kernel<K><<<grid, 256, 0, st>>>(
            static_cast<const K*>(keys), n, m, p_a, p_b, model_b, model_a, step0_a, step0_b, window,
            xbar, ybar, reinterpret_cast<unsigned long long*>(hist),
            reinterpret_cast<unsigned long long*>(counters));
    });
    return hipGetLastError();
}

RankModelLayout rank_model_layout(int64_t S, int dtype) {
    RankModelLayout L;
    const size_t kb = (int)dtype_bytes(dtype);
    size_t off = 0;
    L.off_keys = off; off += align256((size_t)S * kb);
    L.off_target = off; off += align256((size_t)S * 4);
    L.off_partial = off; off += mlp_grad_ws_bytes(S);
    L.off_grad = off; off += 512;
    L.off_m = off; off += 512;
    L.off_v = off; off += 512;
    L.bytes = off;
    return L;
}

hipError_t launch_rank_model_train(int dtype, const void* X, int64_t len, const void* Q,
                                   int64_t q_len, int is_high, int64_t S, int64_t steps, float lr,
                                   uint64_t seed, float* P, float* loss, char* ws,
                                   const RankModelLayout& L, hipStream_t st) {
    void* skeys = ws + L.off_keys;
    float* target = reinterpret_cast<float*>(ws + L.off_target);
    float* partial = reinterpret_cast<float*>(ws + L.off_partial);
    float* grad = reinterpret_cast<float*>(ws + L.off_grad);
    float* M = reinterpret_cast<float*>(ws + L.off_m);
    float* V = reinterpret_cast<float*>(ws + L.off_v);
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        rank_sample_kernel<K><<<grid_for(S, 4096), 256, 0, st>>>(
            static_cast<const K*>(X), len, static_cast<const K*>(Q), q_len, is_high, S, seed,
            static_cast<K*>(skeys), target);
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_mlp_init(dtype, skeys, target, S, P, st)) != hipSuccess) return e;
    fill_f32_kernel<<<1, 128, 0, st>>>(M, NP, 0.0f);
    fill_f32_kernel<<<1, 128, 0, st>>>(V, NP, 0.0f);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // cosine decay from lr to lr / 100 over the steps
    const double lr_min = lr / 100.0;
    for (int64_t t = 1; t <= steps; ++t) {
        const double c = 0.5 * (1.0 + cos(3.14159265358979323846 * (double)(t - 1) / (double)steps));
        const float lr_t = (float)(lr_min + (lr - lr_min) * c);
        if ((e = launch_mlp_grad(dtype, P, skeys, target, S, grad, nullptr, partial, st)) !=
            hipSuccess)
            return e;
        if ((e = launch_mlp_adam(P, M, V, grad, t, lr_t, 0.9f, 0.999f, 1e-8f, st)) != hipSuccess)
            return e;
    }
    // loss of the final parameters
    return launch_mlp_grad(dtype, P, skeys, target, S, grad, loss, partial, st);
}

}  // namespace sm
