// sm_keys.h -- the key types of the library and their order.
//
// dtype codes (include/stablemerge.h): 0 int32, 1 uint32, 2 uint64, 3 int64
// (numeric order), 4 float32, 5 float64.  Floating-point keys are ordered by
// IEEE 754 totalOrder: -NaN < -inf < negative numbers < -0 < +0 < positive
// numbers < +inf < +NaN, NaNs by payload.  Every key type moves as raw bits
// (the kernels copy 16-byte chunks); only its comparison differs.
//
// Descending order is a key type of its own, Desc<K>: the bits of K with the
// comparison reversed.  The kernels are templates over the key type, so a
// descending merge or sort runs the ascending code with this comparison and
// a sentinel that is largest in it (K's smallest value); equal keys stay
// equal, so the tie rules are unchanged.  Launchers take it as the kernel
// dtype code dtype | kDescending.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sm {

// A float key is its bit pattern.  Flipping every bit of a negative value and
// only the sign bit of a positive one turns totalOrder into unsigned order.
struct KeyF32 {
    uint32_t bits;
};
struct KeyF64 {
    uint64_t bits;
};

__host__ __device__ __forceinline__ uint32_t order_bits(KeyF32 k) {
    return k.bits ^ ((uint32_t)((int32_t)k.bits >> 31) | 0x80000000u);
}
__host__ __device__ __forceinline__ uint64_t order_bits(KeyF64 k) {
    return k.bits ^ ((uint64_t)((int64_t)k.bits >> 63) | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ bool operator<(KeyF32 a, KeyF32 b) {
    return order_bits(a) < order_bits(b);
}
__host__ __device__ __forceinline__ bool operator<(KeyF64 a, KeyF64 b) {
    return order_bits(a) < order_bits(b);
}
// equal in totalOrder means equal bits (order_bits is a bijection)
__host__ __device__ __forceinline__ bool operator!=(KeyF32 a, KeyF32 b) { return a.bits != b.bits; }
__host__ __device__ __forceinline__ bool operator!=(KeyF64 a, KeyF64 b) { return a.bits != b.bits; }

// The largest key of each type (the +inf sentinel of the merge windows).
template <typename K>
struct KeyMax;
template <> struct KeyMax<int32_t> { static constexpr int32_t v = 0x7fffffff; };
template <> struct KeyMax<uint32_t> { static constexpr uint32_t v = 0xffffffffu; };
template <> struct KeyMax<uint64_t> { static constexpr uint64_t v = ~0ull; };
template <> struct KeyMax<int64_t> { static constexpr int64_t v = 0x7fffffffffffffffll; };
// +NaN with the largest payload
template <> struct KeyMax<KeyF32> { static constexpr KeyF32 v = {0x7fffffffu}; };
template <> struct KeyMax<KeyF64> { static constexpr KeyF64 v = {0x7fffffffffffffffull}; };

// The smallest key of each type.
template <typename K>
struct KeyMin;
template <> struct KeyMin<int32_t> { static constexpr int32_t v = -0x7fffffff - 1; };
template <> struct KeyMin<uint32_t> { static constexpr uint32_t v = 0u; };
template <> struct KeyMin<uint64_t> { static constexpr uint64_t v = 0ull; };
template <> struct KeyMin<int64_t> { static constexpr int64_t v = -0x7fffffffffffffffll - 1; };
// -NaN with the largest payload
template <> struct KeyMin<KeyF32> { static constexpr KeyF32 v = {0xffffffffu}; };
template <> struct KeyMin<KeyF64> { static constexpr KeyF64 v = {~0ull}; };

// K in descending order.
template <typename K>
struct Desc {
    K v;
};
template <typename K>
__host__ __device__ __forceinline__ bool operator<(Desc<K> a, Desc<K> b) {
    return b.v < a.v;
}
template <typename K>
__host__ __device__ __forceinline__ bool operator!=(Desc<K> a, Desc<K> b) {
    return a.v != b.v;
}
template <typename K>
struct KeyMax<Desc<K>> {
    static constexpr Desc<K> v = {KeyMin<K>::v};
};
template <typename K>
struct IsDesc {
    static constexpr bool value = false;
};
template <typename K>
struct IsDesc<Desc<K>> {
    static constexpr bool value = true;
};

// Public dtype codes, and the kernel codes that add the order.
constexpr int kDescending = 8;
inline bool dtype_known(int dtype) { return dtype >= 0 && dtype <= 5; }
inline int kernel_dtype(int dtype, bool descending) {
    return descending ? dtype | kDescending : dtype;
}
inline size_t dtype_bytes(int dtype) {
    const int t = dtype & ~kDescending;
    return t == 2 || t == 3 || t == 5 ? 8 : 4;
}

// Calls f with a value of the (ascending) key type of dtype; the order bit
// is ignored (host-side dispatch for kernels that have no descending form).
template <typename F>
inline void with_key_type_asc(int dtype, F&& f) {
    switch (dtype & ~kDescending) {
        case 0: f((int32_t)0); break;
        case 1: f((uint32_t)0); break;
        case 2: f((uint64_t)0); break;
        case 3: f((int64_t)0); break;
        case 4: f(KeyF32{0}); break;
        default: f(KeyF64{0}); break;
    }
}

// Calls f with a value of the key type of a kernel dtype code, Desc<K> when
// the order bit is set.
template <typename F>
inline void with_key_type(int dtype, F&& f) {
    if (dtype & kDescending)
        with_key_type_asc(dtype, [&](auto z) { f(Desc<decltype(z)>{z}); });
    else
        with_key_type_asc(dtype, f);
}

}  // namespace sm
