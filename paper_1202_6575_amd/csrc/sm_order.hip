// sm_order.hip -- descending order by an order-reversing key transform.
//
// For every key type there is an involution that reverses the key order:
// bitwise NOT for integers (two's complement: ~x = -x - 1; unsigned:
// ~x = max - x), and a sign-bit flip for floats (IEEE 754 totalOrder read
// backwards is the order of the negated values, -0 and +0 and NaNs
// included).  A stable sort or merge in descending order is the ascending
// one of the transformed keys, transformed back: equal keys stay equal, so
// the tie rules carry over unchanged.
#include "sm_keys.h"
#include "sm_launch.h"

namespace sm {

namespace {

// dst = flip(src) over `words` 32-bit words, 16 bytes per lane and step
// (src == dst is allowed, hence no __restrict__): `mask` is XORed into every
// word, or with `only_hi` into the odd words only (the high words of 8-byte
// float keys).
__global__ __launch_bounds__(256) void flip_kernel(const uint32_t* src,
                                                   uint32_t* dst, int64_t words,
                                                   uint32_t mask, int only_hi) {
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    constexpr int U = 4;    // chunks in flight per lane
    const u4 m4 = only_hi ? u4{0u, mask, 0u, mask} : u4{mask, mask, mask, mask};
    const u4* s4 = reinterpret_cast<const u4*>(src);
    u4* d4 = reinterpret_cast<u4*>(dst);
    const int64_t chunks = words / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // all U loads of a step are issued before its stores; chunk indices of
    // one step are distinct, so src == dst is safe
    for (; c + (U - 1) * stride < chunks; c += U * stride) {
        u4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = s4[c + k * stride];
#pragma unroll
        for (int k = 0; k < U; ++k) d4[c + k * stride] = v[k] ^ m4;
    }
    for (; c < chunks; c += stride) d4[c] = s4[c] ^ m4;
    // the words past the last whole chunk (fewer than 4; words of 8-byte keys
    // come in pairs, so a high word is an odd word)
    if (blockIdx.x == 0 && threadIdx.x < words - chunks * 4) {
        const int64_t w = chunks * 4 + threadIdx.x;
        dst[w] = src[w] ^ (only_hi && (w & 1) == 0 ? 0u : mask);
    }
}

}  // namespace

hipError_t launch_flip_order(int dtype, const void* src, void* dst, int64_t N, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    const int64_t words = N * (int64_t)(dtype_bytes(dtype) / 4);
    const bool is_float = dtype == 4 || dtype == 5;
    const uint32_t mask = is_float ? 0x80000000u : 0xffffffffu;
    const int only_hi = dtype == 5 ? 1 : 0;
    // four 16-byte chunks per lane and step; at most 16 workgroups per CU
    int64_t g = (words / 16 + 255) / 256;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    flip_kernel<<<(unsigned)g, 256, 0, st>>>(static_cast<const uint32_t*>(src),
                                             static_cast<uint32_t*>(dst), words, mask, only_hi);
    return hipGetLastError();
}

}  // namespace sm
