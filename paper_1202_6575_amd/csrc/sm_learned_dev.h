// sm_learned_dev.h -- device side of the learned cross ranks (internal):
// the key feature, the network's forward pass, the predicted rank and the
// bounded search from it.  Shared by the learned partition kernels and the
// batch engine's learned partition (merge-sort passes).
#pragma once

#include "sm_device.h"
#include "sm_learned.h"

namespace sm {

// phi(key) = log2(u + 1) / bits, u the order-preserving unsigned form of the key.
__device__ __forceinline__ float feature(int32_t x) {
    const uint32_t u = (uint32_t)x ^ 0x80000000u;
    return log2f((float)u + 1.0f) * (1.0f / 32.0f);
}
__device__ __forceinline__ float feature(uint32_t x) {
    return log2f((float)x + 1.0f) * (1.0f / 32.0f);
}
__device__ __forceinline__ float feature(uint64_t x) {
    return log2f((float)x + 1.0f) * (1.0f / 64.0f);
}
__device__ __forceinline__ float feature(int64_t x) {
    return feature((uint64_t)((uint64_t)x ^ 0x8000000000000000ull));
}
// floats: the position in totalOrder, as an unsigned integer of the same width
__device__ __forceinline__ float feature(KeyF32 x) { return feature(order_bits(x)); }
__device__ __forceinline__ float feature(KeyF64 x) { return feature(order_bits(x)); }

// y = b2 + sum_k w2[k] * ReLU(W1[k] * phi + b1[k]); parameters W1[0:32],
// b1[32:64], w2[64:96], b2[96].
__device__ __forceinline__ float mlp_forward(const float* __restrict__ P, float phi) {
    float y = P[3 * kMlpHidden];
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) {
        const float h = fmaxf(fmaf(P[k], phi, P[kMlpHidden + k]), 0.0f);
        y = fmaf(P[2 * kMlpHidden + k], h, y);
    }
    return y;
}

// Predicted rank clamp(rint(y * len), 0, len); 0 when y is not a number.
__device__ __forceinline__ int64_t predict(const float* __restrict__ P, float phi, int64_t len) {
    const double r = rint((double)mlp_forward(P, phi) * (double)len);
    return !(r > 0.0) ? 0 : (r >= (double)len ? len : (int64_t)r);
}

// Bounded exponential search for the rank of x in X[0, len): probe the
// guess g, then step away from it by step0, 2 step0, 4 step0, ... until the
// rank is bracketed (or the array ends), then bisect the bracket at aligned
// points.  A step beyond `window` abandons the walk for the same bisection
// of all of [0, len].
// Low: pred(t) = X[t] < x (rank_low); high: pred(t) = X[t] <= x (rank_high);
// the rank is the number of t with pred(t).  `probes` counts reads of X.
template <typename K, bool HIGH>
__device__ __forceinline__ int64_t bounded_search(const K* __restrict__ X, int64_t len, K x,
                                                  int64_t g, int64_t step0, int64_t window,
                                                  int& probes, bool& fell_back) {
    int np = 0;
    auto pred = [&](int64_t t) {
        ++np;
        const K v = X[t];
        return HIGH ? !(x < v) : (v < x);
    };
    g = g < 0 ? 0 : (g > len ? len : g);
    int64_t lo = 0, hi = len;
    bool fb = false;
    int64_t d = step0 < 1 ? 1 : step0;
    if (g < len && pred(g)) {
        lo = g + 1;  // the rank is above g
        for (;;) {
            if (d > window) { fb = true; break; }
            const int64_t t = g + d;
            if (t >= len) { hi = len; break; }
            if (!pred(t)) { hi = t; break; }
            lo = t + 1;
            d <<= 1;
        }
    } else {
        hi = g;  // the rank is at most g
        for (;;) {
            if (d > window) { fb = true; break; }
            const int64_t t = g - d;
            if (t < 0) { lo = 0; break; }
            if (pred(t)) { lo = t + 1; break; }
            hi = t;
            d <<= 1;
        }
    }
    if (fb) {
        lo = 0;
        hi = len;
    }
    // the rank is in [lo, hi]: split at the number in (lo, hi] with the most
    // trailing zero bits (the top bit in which lo and hi differ set, the bits
    // below it clear); the rank is >= m exactly when X[m - 1] satisfies the
    // predicate.  The split points are aligned, so the lanes of a wave, whose
    // brackets overlap, read the same elements until their brackets part.
    if (len < (int64_t)1 << 31) {
        // the same splits in 32-bit arithmetic (lo, hi <= len)
        uint32_t l32 = (uint32_t)lo, h32 = (uint32_t)hi;
        while (l32 < h32) {
            const int h = 31 - __clz((int)(l32 ^ h32));
            const uint32_t m = (h32 >> h) << h;
            if (pred((int64_t)(m - 1))) l32 = m;
            else h32 = m - 1;
        }
        lo = l32;
    } else {
        while (lo < hi) {
            const int h = 63 - __clzll((long long)((uint64_t)lo ^ (uint64_t)hi));
            const int64_t m = (int64_t)(((uint64_t)hi >> h) << h);
            if (pred(m - 1)) lo = m;
            else hi = m - 1;
        }
    }
    probes = np;
    fell_back = fb;
    return lo;
}

}  // namespace sm
