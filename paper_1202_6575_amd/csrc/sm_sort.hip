// sm_sort.hip -- stable merge sort built from stable merges (Section 3).
//
// Run formation: every workgroup sorts one run of RUN consecutive elements
// in LDS.  Each round merges neighbouring sorted pieces of width w by cross
// ranks with blocks of one element: an element of the left piece moves by
// its rank_low in the right piece, an element of the right piece by its
// rank_high in the left piece (Section 2 with every block a single element,
// so every subproblem is one element and its output position is the sum of
// its two ranks).  log2(RUN) rounds give a stably sorted run.
//
// Merge passes: pass w merges runs [2kw, 2kw + w) and [2kw + w, 2kw + 2w)
// for every k as one batch of jobs (the batch engine splits every job by
// the method); a lone last run is a job with an empty B, i.e. a copy.
// Buffers alternate between the output and a workspace copy, and run
// formation writes to whichever makes the last pass end in the output.
#include "sm_device.h"
#include "sm_launch.h"
#include "sm_batch.h"
#include "sm_sort.h"

namespace sm {

namespace {

// threads sorting one run: two elements each, at most 1024 (the rank
// searches are chains of dependent LDS reads, so the more waves share a CU
// the better their latency is hidden)
template <int RUN>
constexpr int run_threads() { return RUN / 2 < 1024 ? RUN / 2 : 1024; }

template <typename K, bool PAY, int RUN>
struct RunSmem {
    K key[2][RUN];
    uint32_t pay[PAY ? 2 : 1][PAY ? RUN : 1];
};

// Stable sort of keys[r0, r0 + len) (len <= RUN) into out[r0, r0 + len).
// Positions past len hold the largest key; they start behind every real
// element and every round keeps them there (a right element ties behind the
// whole left piece), so the real elements' order is the stable one.
template <typename K, bool PAY, int RUN>
// keys / out (and pay / out_pay) may be the same array: a workgroup reads
// its whole run before it writes any of it.
__global__ __launch_bounds__(run_threads<RUN>()) void sort_runs_kernel(const K* keys, const uint32_t* pay,
                                                                int64_t N, K* out,
                                                                uint32_t* out_pay) {
    constexpr int T = run_threads<RUN>();
    constexpr int E = RUN / T;
    static_assert(RUN % T == 0 && (RUN & (RUN - 1)) == 0, "RUN: power of two, multiple of T");
    __shared__ RunSmem<K, PAY, RUN> s;
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * RUN;
    const int64_t rem = N - r0;
    const int len = rem < RUN ? (int)rem : RUN;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + T * e;
        s.key[0][i] = i < len ? keys[r0 + i] : KeyMax<K>::v;
        if (PAY) s.pay[0][i] = i < len ? pay[r0 + i] : 0u;
    }
    __syncthreads();
    int cur = 0;
    for (int w = 1; w < RUN; w <<= 1) {
        K kv[E];
        uint32_t pv[E];
        int dst[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = t + T * e;
            const K x = s.key[cur][i];
            const int lo = i & ~(2 * w - 1);   // start of the pair of pieces
            const bool right = (i & w) != 0;
            const K* other = &s.key[cur][right ? lo : lo + w];
            const int r = right ? upper_bound_lds<K>(other, w, x) : lower_bound_lds<K>(other, w, x);
            dst[e] = lo + (i - lo - (right ? w : 0)) + r;
            kv[e] = x;
            if (PAY) pv[e] = s.pay[cur][i];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            s.key[cur ^ 1][dst[e]] = kv[e];
            if (PAY) s.pay[cur ^ 1][dst[e]] = pv[e];
        }
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = t + T * e;
        if (i < len) {
            out[r0 + i] = s.key[cur][i];
            if (PAY) out_pay[r0 + i] = s.pay[cur][i];
        }
    }
}

// Jobs of merge pass w: job k merges [2kw, min(2kw + w, N)) with
// [min(2kw + w, N), min(2kw + 2w, N)).  Runs are separate arrays here, so
// no segment has a successor.
__global__ __launch_bounds__(256) void sort_pass_jobs_kernel(int64_t N, int64_t w, int64_t count,
                                                             PieceDesc* __restrict__ jobs) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = 2 * k * w;
        const int64_t mid = lo + w < N ? lo + w : N;
        const int64_t hi = lo + 2 * w < N ? lo + 2 * w : N;
        PieceDesc j;
        j.ka0 = lo;
        j.kb0 = mid;
        j.out0 = lo;
        j.a_f = (uint32_t)(mid - lo);
        j.b_f = (uint32_t)(hi - mid);
        jobs[k] = j;
    }
}


template <typename K, bool PAY>
hipError_t launch_runs_t(const K* keys, const uint32_t* pay, int64_t N, K* out, uint32_t* out_pay,
                         int run, hipStream_t st) {
    const int64_t g = (N + run - 1) / run;
    switch (run) {
        case 256: sort_runs_kernel<K, PAY, 256><<<(unsigned)g, run_threads<256>(), 0, st>>>(keys, pay, N, out, out_pay); break;
        case 512: sort_runs_kernel<K, PAY, 512><<<(unsigned)g, run_threads<512>(), 0, st>>>(keys, pay, N, out, out_pay); break;
        case 1024: sort_runs_kernel<K, PAY, 1024><<<(unsigned)g, run_threads<1024>(), 0, st>>>(keys, pay, N, out, out_pay); break;
        case 2048: sort_runs_kernel<K, PAY, 2048><<<(unsigned)g, run_threads<2048>(), 0, st>>>(keys, pay, N, out, out_pay); break;
        case 4096:
            // 32-bit keys only: two buffers of 4096 keys and payloads fill 64 KiB
            if constexpr (sizeof(K) == 4) {
                sort_runs_kernel<K, PAY, 4096><<<(unsigned)g, run_threads<4096>(), 0, st>>>(keys, pay, N, out, out_pay);
                break;
            } else {
                return hipErrorInvalidValue;
            }
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

bool sort_run_ok(int run, int dtype) {
    return run == 256 || run == 512 || run == 1024 || run == 2048 || (run == 4096 && dtype_bytes(dtype) == 4);
}

int sort_passes(int64_t N, int run) {
    int p = 0;
    for (int64_t w = run; w < N; w *= 2) ++p;
    return p;
}

SortLayout sort_layout(int64_t N, int dtype, bool pay, int run, int64_t tile) {
    SortLayout L;
    const size_t kb = (int)dtype_bytes(dtype);
    L.passes = sort_passes(N, run);
    L.count_max = N > run ? (N + 2 * (int64_t)run - 1) / (2 * (int64_t)run) : 1;
    size_t off = 0;
    L.off_tmp_keys = off; off += align256((size_t)N * kb);
    L.off_tmp_pay = off; off += pay ? align256((size_t)N * 4) : 0;
    L.off_jobs = off; off += align256((size_t)L.count_max * kPieceDescBytes);
    L.off_batch = off;
    // the first pass has the most jobs; later passes reuse the same bytes
    L.batch = batch_layout(L.count_max, N, tile);
    off += L.batch.bytes;
    L.bytes = off;
    return L;
}

hipError_t launch_sort(int dtype, const void* keys, const uint32_t* pay, int64_t N, void* out_keys,
                       uint32_t* out_pay, int run, int64_t tile, char* ws, const SortLayout& L,
                       hipStream_t st) {
    if (N <= 0) return hipSuccess;
    char* tmp_k = ws + L.off_tmp_keys;
    uint32_t* tmp_p = pay ? reinterpret_cast<uint32_t*>(ws + L.off_tmp_pay) : nullptr;
    PieceDesc* jobs = reinterpret_cast<PieceDesc*>(ws + L.off_jobs);
    // run formation writes where an even number of passes remains before the output
    const bool runs_to_out = (L.passes % 2) == 0;
    char* src_k = runs_to_out ? static_cast<char*>(out_keys) : tmp_k;
    uint32_t* src_p = runs_to_out ? out_pay : tmp_p;
    char* dst_k = runs_to_out ? tmp_k : static_cast<char*>(out_keys);
    uint32_t* dst_p = runs_to_out ? tmp_p : out_pay;
    hipError_t e = hipSuccess;
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        e = pay ? launch_runs_t<K, true>(static_cast<const K*>(keys), pay, N,
                                         reinterpret_cast<K*>(src_k), src_p, run, st)
                : launch_runs_t<K, false>(static_cast<const K*>(keys), nullptr, N,
                                          reinterpret_cast<K*>(src_k), nullptr, run, st);
    });
    if (e != hipSuccess) return e;
    for (int64_t w = run; w < N; w *= 2) {
        const int64_t count = (N + 2 * w - 1) / (2 * w);
        int64_t g = (count + 255) / 256;
        if (g > 4096) g = 4096;
        sort_pass_jobs_kernel<<<(unsigned)g, 256, 0, st>>>(N, w, count, jobs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const BatchLayout BL = batch_layout(count, N, tile);
        e = launch_batch(dtype, src_k, src_p, N, dst_k, dst_p, N, jobs, count, tile,
                         ws + L.off_batch, BL, st);
        if (e != hipSuccess) return e;
        char* tk = src_k; src_k = dst_k; dst_k = tk;
        uint32_t* tp = src_p; src_p = dst_p; dst_p = tp;
    }
    return hipSuccess;
}

}  // namespace sm
