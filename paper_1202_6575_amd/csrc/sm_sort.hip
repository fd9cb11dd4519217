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

// Threads sorting one run: eight consecutive elements each.
template <int RUN>
constexpr int run_threads() { return RUN / 8; }

// LDS of one run: two buffers of keys (and payloads).
template <typename K, bool PAY, int RUN>
struct RunSmem {
    K key[2][RUN];
    uint32_t pay[PAY ? 2 : 1][PAY ? RUN : 1];
};

// Segments (the segmented sort): segment s is [offsets[s], offsets[s + 1]).
// Work item k of segment s at width W (its k-th run, or its k-th pair of
// runs) gets the slot s + floor(offsets[s] / W) + k.  This is one-to-one
// over k < ceil(len_s / W): the first slot of segment s + 1 is at least
// 1 + floor(offsets[s + 1] / W), beyond the last slot of segment s.  So
// count + N / W + 1 slots cover every item, and a slot finds its segment
// by binary search, with no prefix sums.  Returns false for a slot that
// holds no item.
__device__ __forceinline__ bool seg_slot(const int64_t* __restrict__ offsets, int64_t count,
                                         int64_t W, int64_t t, int64_t& seg, int64_t& k) {
    if (count <= 0 || offsets[0] / W > t) return false;
    int64_t lo = 0, hi = count - 1;   // last s with s + offsets[s] / W <= t
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (mid + offsets[mid] / W <= t) lo = mid;
        else hi = mid - 1;
    }
    seg = lo;
    k = t - (lo + offsets[lo] / W);
    const int64_t len = offsets[lo + 1] - offsets[lo];
    return k < (len + W - 1) / W;
}

// Eight consecutive elements of the run into registers; positions at or
// past len hold the largest key (and payload 0).  vec: the eight start on a
// 16-byte boundary in memory.
template <typename K, bool PAY>
__device__ __forceinline__ void load8(const K* keys, const uint32_t* pay, int64_t at, int valid,
                                      bool vec, K (&k)[8], uint32_t (&p)[8]) {
    if (vec && valid >= 8) {
        constexpr int V = 16 / sizeof(K);
#pragma unroll
        for (int c = 0; c < 8 / V; ++c) {
            const u32x4 v = *reinterpret_cast<const u32x4*>(keys + at + c * V);
            __builtin_memcpy(&k[c * V], &v, 16);
        }
        if (PAY) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const u32x4 v = *reinterpret_cast<const u32x4*>(pay + at + c * 4);
                p[4 * c] = v.x; p[4 * c + 1] = v.y; p[4 * c + 2] = v.z; p[4 * c + 3] = v.w;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            k[e] = e < valid ? keys[at + e] : KeyMax<K>::v;
            if (PAY) p[e] = e < valid ? pay[at + e] : 0u;
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
        if (!PAY) p[e] = 0u;
}

template <typename K, bool PAY>
__device__ __forceinline__ void store8(K* out, uint32_t* out_pay, int64_t at, int valid, bool vec,
                                       const K (&k)[8], const uint32_t (&p)[8]) {
    if (vec && valid >= 8) {
        constexpr int V = 16 / sizeof(K);
#pragma unroll
        for (int c = 0; c < 8 / V; ++c) {
            u32x4 v;
            __builtin_memcpy(&v, &k[c * V], 16);
            *reinterpret_cast<u32x4*>(out + at + c * V) = v;
        }
        if (PAY) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                u32x4 v;
                v.x = p[4 * c]; v.y = p[4 * c + 1]; v.z = p[4 * c + 2]; v.w = p[4 * c + 3];
                *reinterpret_cast<u32x4*>(out_pay + at + c * 4) = v;
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            if (e < valid) {
                out[at + e] = k[e];
                if (PAY) out_pay[at + e] = p[e];
            }
        }
    }
}

// Stable sort of keys[r0, r0 + len) (len <= RUN) into out[r0, r0 + len):
// r0 = blockIdx.x * RUN without segments; with segments, the block's slot
// names a run of a segment, which starts at the segment's start.
//   1. Every thread places its eight elements by their stable ranks: the
//      rank of element e is the number of the eight with a smaller key plus
//      the number before e with an equal key (28 comparisons), and e goes to
//      slot 8t + rank in LDS.
//   2. Rounds w = 8, 16, ..., RUN / 2 merge neighbouring sorted pieces of w
//      elements.  Thread t produces outputs [8t, 8t + 8) of its pair: the
//      number i of the pair's first 8t outputs (counted from the pair's
//      start) that come from the left piece is found by binary search (the
//      left piece's element a is among them iff a <= the right piece's
//      element on the same diagonal), then eight steps of the stable
//      two-pointer merge (right only if strictly smaller) from (i, d - i).
//      A step reads only the next element of the side it took; payloads
//      are read after the eight steps from the positions recorded.
//      Outputs gather in registers and go to the other LDS buffer, the last
//      round's straight to memory.
// Positions past len hold the largest key; they start behind every real
// element and every step keeps them there (equal keys keep their order), so
// the real elements' order is the stable one.
// keys / out (and pay / out_pay) may be the same array: a workgroup reads
// its whole run before it writes any of it.
template <typename K, bool PAY, int RUN>
__global__ __launch_bounds__(run_threads<RUN>()) void sort_runs_kernel(
    const K* keys, const uint32_t* pay, int64_t N, K* out, uint32_t* out_pay,
    const int64_t* __restrict__ seg_offsets, int64_t seg_count) {
    static_assert(RUN % 16 == 0 && (RUN & (RUN - 1)) == 0, "RUN: a power of two");
    __shared__ __align__(16) RunSmem<K, PAY, RUN> s;
    const int t = threadIdx.x;
    int64_t r0 = (int64_t)blockIdx.x * RUN, end = N;
    if (seg_offsets) {
        int64_t sg, r;
        if (!seg_slot(seg_offsets, seg_count, RUN, blockIdx.x, sg, r)) return;
        r0 = seg_offsets[sg] + r * RUN;
        end = seg_offsets[sg + 1];
    }
    const int64_t rem = end - r0;
    const int len = rem < RUN ? (int)rem : RUN;
    const int o0 = 8 * t;
    const int valid = len - o0;   // may be <= 0
    // 16-byte access needs the run start (and payload start) aligned
    const bool vec = ((reinterpret_cast<uintptr_t>(keys + r0) | reinterpret_cast<uintptr_t>(out + r0)) & 15) == 0 &&
                     (!PAY || ((reinterpret_cast<uintptr_t>(pay + r0) |
                                reinterpret_cast<uintptr_t>(out_pay + r0)) & 15) == 0);
    K k[8];
    uint32_t p[8];
    load8<K, PAY>(keys, pay, r0 + o0, valid, vec, k, p);

    // 1. stable ranks among the eight (a later element with an equal key
    //    ranks behind), then each element to its slot
    int rk[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) rk[e] = e;
#pragma unroll
    for (int e = 1; e < 8; ++e) {
#pragma unroll
        for (int f = 0; f < e; ++f) {
            const int c = k[e] < k[f] ? 1 : 0;   // e passes f
            rk[e] -= c;
            rk[f] += c;
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        s.key[0][o0 + rk[e]] = k[e];
        if (PAY) s.pay[0][o0 + rk[e]] = p[e];
    }

    // 2. merge rounds
    int cur = 0;
#pragma unroll 1
    for (int w = 8; w < RUN; w <<= 1) {
        __syncthreads();
        const int base = o0 & ~(2 * w - 1);
        const int d = o0 - base;
        const K* A = &s.key[cur][base];
        const K* B = A + w;
        const K* Bend = B + w;
        int lo = d > w ? d - w : 0, hi = d < w ? d : w;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (!(B[d - 1 - mid] < A[mid])) lo = mid + 1;
            else hi = mid;
        }
        // pa, pb: the heads of the two pieces (at B and at Bend: exhausted)
        const K* pa = A + lo;
        const K* pb = B + (d - lo);
        K ka = *(pa < B ? pa : B - 1), kb = *(pb < Bend ? pb : Bend - 1);
        const K* from[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const bool takeB = (pb < Bend) & ((pa >= B) | (kb < ka));
            k[e] = takeB ? kb : ka;
            from[e] = takeB ? pb : pa;
            pa += takeB ? 0 : 1;
            pb += takeB ? 1 : 0;
            // the next element of the side taken (past its end: a stale
            // value that the bounds above never let win)
            const K* nx = takeB ? pb : pa;
            const K v = *(nx < Bend ? nx : Bend - 1);
            ka = takeB ? ka : v;
            kb = takeB ? v : kb;
        }
        if (PAY) {
#pragma unroll
            for (int e = 0; e < 8; ++e) p[e] = s.pay[cur][from[e] - s.key[cur]];
        }
        if (2 * w < RUN) {
            // the other buffer was last read in the round before this one,
            // which every thread finished before this round's barrier
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                s.key[cur ^ 1][o0 + e] = k[e];
                if (PAY) s.pay[cur ^ 1][o0 + e] = p[e];
            }
        }
        cur ^= 1;
    }
    store8<K, PAY>(out, out_pay, r0 + o0, valid, vec, k, p);
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


// Jobs of merge pass w and their plan for the batch engine, when the pairs
// exceed one merge workgroup: every job but the last is two full runs, so
// it has uni_p subproblems and uni_s cross ranks, and the engine's
// exclusive starts are k * uni_p and k * uni_s (the totals, from the host,
// close the lists).  Replaces the per-job counts and scans of the general
// engine.
__global__ __launch_bounds__(256) void sort_pass_plan_kernel(
    int64_t N, int64_t w, int64_t count, PieceDesc* __restrict__ jobs,
    int64_t* __restrict__ pstart, int64_t* __restrict__ sstart, int64_t* __restrict__ totals,
    int64_t uni_p, int64_t uni_s, int64_t P, int64_t S) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= count;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (k == count) {
            pstart[count] = P;
            sstart[count] = S;
            totals[0] = P;
            totals[1] = S;
            continue;
        }
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
        pstart[k] = k * uni_p;
        sstart[k] = k * uni_s;
    }
}

// Jobs of merge pass w of the segmented sort: slot t (at width 2w) holds
// pair k of segment s: [lo, lo + w) with [lo + w, lo + 2w), clipped to the
// segment, lo = offsets[s] + 2kw; a slot with no pair is an empty job.
__global__ __launch_bounds__(256) void seg_pass_jobs_kernel(const int64_t* __restrict__ offsets,
                                                            int64_t count, int64_t w,
                                                            int64_t nslots,
                                                            PieceDesc* __restrict__ jobs) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nslots;
         t += (int64_t)gridDim.x * blockDim.x) {
        PieceDesc j;
        j.ka0 = j.kb0 = j.out0 = 0;
        j.a_f = j.b_f = 0;
        int64_t sg, k;
        if (seg_slot(offsets, count, 2 * w, t, sg, k)) {
            const int64_t end = offsets[sg + 1];
            const int64_t lo = offsets[sg] + 2 * k * w;
            const int64_t mid = lo + w < end ? lo + w : end;
            const int64_t hi = lo + 2 * w < end ? lo + 2 * w : end;
            j.ka0 = lo;
            j.kb0 = mid;
            j.out0 = lo;
            j.a_f = (uint32_t)(mid - lo);
            j.b_f = (uint32_t)(hi - mid);
        }
        jobs[t] = j;
    }
}

// Sets *bad unless offsets run from 0 to N without decreasing and no segment
// is longer than max_len.
__global__ __launch_bounds__(256) void seg_check_kernel(const int64_t* __restrict__ offsets,
                                                        int64_t count, int64_t N, int64_t max_len,
                                                        int* __restrict__ bad) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = offsets[s], b = offsets[s + 1];
        if (b < a || b - a > max_len || (s == 0 && a != 0) || (s == count - 1 && b != N))
            *bad = 1;
    }
}

template <typename K, bool PAY>
hipError_t launch_runs_t(const K* keys, const uint32_t* pay, int64_t N, K* out, uint32_t* out_pay,
                         int run, const int64_t* seg_offsets, int64_t seg_count,
                         hipStream_t st) {
    // without segments one workgroup per run; with them one per slot
    const int64_t g = seg_offsets ? seg_count + N / run + 1 : (N + run - 1) / run;
    if (g <= 0) return hipSuccess;
    auto go = [&](auto kern, int threads) {
        kern<<<(unsigned)g, threads, 0, st>>>(keys, pay, N, out, out_pay, seg_offsets, seg_count);
    };
    switch (run) {
        case 256: go(sort_runs_kernel<K, PAY, 256>, run_threads<256>()); break;
        case 512: go(sort_runs_kernel<K, PAY, 512>, run_threads<512>()); break;
        case 1024: go(sort_runs_kernel<K, PAY, 1024>, run_threads<1024>()); break;
        case 2048: go(sort_runs_kernel<K, PAY, 2048>, run_threads<2048>()); break;
        case 4096:
            // 32-bit keys only: two buffers of 4096 keys and payloads fill 64 KiB
            if constexpr (sizeof(K) == 4) {
                go(sort_runs_kernel<K, PAY, 4096>, run_threads<4096>());
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

SortLayout sort_layout(int64_t N, int dtype, bool pay, int run, int64_t tile, int64_t seg_count,
                       int64_t max_len) {
    SortLayout L;
    const size_t kb = (int)dtype_bytes(dtype);
    if (seg_count > 0) {
        // passes until the longest segment is one run; the first pass has
        // the most job slots
        L.passes = sort_passes(max_len, run);
        L.count_max = seg_count + N / (2 * (int64_t)run) + 1;
    } else {
        L.passes = sort_passes(N, run);
        L.count_max = N > run ? (N + 2 * (int64_t)run - 1) / (2 * (int64_t)run) : 1;
    }
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
                       hipStream_t st, const int64_t* seg_offsets, int64_t seg_count,
                       const LearnedSearch* ls) {
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
                                         reinterpret_cast<K*>(src_k), src_p, run, seg_offsets,
                                         seg_count, st)
                : launch_runs_t<K, false>(static_cast<const K*>(keys), nullptr, N,
                                          reinterpret_cast<K*>(src_k), nullptr, run, seg_offsets,
                                          seg_count, st);
    });
    if (e != hipSuccess) return e;
    int64_t w = run;
    const uint32_t cap = merge_cap_for_tile((int32_t)tile);
    for (int pass = 0; pass < L.passes; ++pass, w *= 2) {
        // job slots of this pass: one per pair of runs, or (segments) the
        // slot bound at width 2w
        const int64_t count = seg_offsets ? seg_count + N / (2 * w) + 1 : (N + 2 * w - 1) / (2 * w);
        int64_t g = (count + 1 + 255) / 256;
        if (g > 4096) g = 4096;
        const bool whole = !seg_offsets && 2 * w <= (int64_t)cap;
        const BatchLayout BL = batch_layout(count, N, tile);
        // subproblems and cross ranks of a job of a + b elements, as the
        // batch engine counts them
        auto counts = [&](int64_t a, int64_t b, int64_t& np, int64_t& ns) {
            if (a + b <= (int64_t)cap) {
                np = a + b > 0 ? 1 : 0;
                ns = 0;
                return;
            }
            const int64_t pa = a > 0 ? (a + tile - 1) / tile : 1, pb = b > 0 ? (b + tile - 1) / tile : 1;
            np = pa + pb;
            ns = pa + pb + 2;
        };
        int64_t uni_p = 0, uni_s = 0;
        if (seg_offsets) {
            seg_pass_jobs_kernel<<<(unsigned)g, 256, 0, st>>>(seg_offsets, seg_count, w, count, jobs);
        } else if (whole) {
            sort_pass_jobs_kernel<<<(unsigned)g, 256, 0, st>>>(N, w, count, jobs);
        } else {
            const int64_t lo = 2 * (count - 1) * w;
            const int64_t mid = lo + w < N ? lo + w : N, hi = lo + 2 * w < N ? lo + 2 * w : N;
            int64_t np_l, ns_l;
            counts(w, w, uni_p, uni_s);
            counts(mid - lo, hi - mid, np_l, ns_l);
            char* bw = ws + L.off_batch;
            sort_pass_plan_kernel<<<(unsigned)g, 256, 0, st>>>(
                N, w, count, jobs, reinterpret_cast<int64_t*>(bw + BL.off_pstart),
                reinterpret_cast<int64_t*>(bw + BL.off_sstart),
                reinterpret_cast<int64_t*>(bw + BL.off_totals), uni_p, uni_s,
                (count - 1) * uni_p + np_l, (count - 1) * uni_s + ns_l);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (whole) {
            // a pair of runs fits one merge workgroup: each job is merged
            // whole, with no cross ranks to find
            e = launch_merge_desc(dtype, src_k, src_p, N, dst_k, dst_p, N, jobs, count, nullptr,
                                  cap, st);
        } else if (seg_offsets) {
            e = launch_batch(dtype, src_k, src_p, N, dst_k, dst_p, N, jobs, count, tile,
                             ws + L.off_batch, BL, st, ls);
        } else {
            e = launch_batch_planned(dtype, src_k, src_p, N, dst_k, dst_p, N, jobs, count, tile,
                                     ws + L.off_batch, BL, st, ls, uni_p, uni_s);
        }
        if (e != hipSuccess) return e;
        char* tk = src_k; src_k = dst_k; dst_k = tk;
        uint32_t* tp = src_p; src_p = dst_p; dst_p = tp;
    }
    return hipSuccess;
}

hipError_t launch_sort_runs(int dtype, const void* keys, const uint32_t* pay, int64_t N,
                            void* out_keys, uint32_t* out_pay, int run, hipStream_t st) {
    hipError_t e = hipSuccess;
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        e = pay ? launch_runs_t<K, true>(static_cast<const K*>(keys), pay, N,
                                         static_cast<K*>(out_keys), out_pay, run, nullptr, 0, st)
                : launch_runs_t<K, false>(static_cast<const K*>(keys), nullptr, N,
                                          static_cast<K*>(out_keys), nullptr, run, nullptr, 0, st);
    });
    return e;
}

hipError_t launch_seg_check(const int64_t* offsets, int64_t count, int64_t N, int64_t max_len,
                            int* bad, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 4096) g = 4096;
    seg_check_kernel<<<(unsigned)g, 256, 0, st>>>(offsets, count, N, max_len, bad);
    return hipGetLastError();
}

}  // namespace sm
