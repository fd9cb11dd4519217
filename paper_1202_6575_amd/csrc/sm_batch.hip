// sm_batch.hip -- many independent merges ("jobs") in one fixed launch sequence.
//
// A job is a merge of keys[ka0, ka0 + a) (its A) with keys[kb0, kb0 + b)
// (its B) into out[out0, out0 + a + b), described by a PieceDesc.  The
// sequence, for any number of jobs of any sizes:
//   plan + scan   per job: a job that fits one workgroup is one subproblem;
//                 a larger one is split by the paper's method with blocks of
//                 `tile` elements (p_a = ceil(a / tile), p_b = ceil(b / tile)),
//                 giving p_a + p_b subproblems and p_a + p_b + 2 cross ranks.
//                 Exclusive scans of both counts place every job's ranks and
//                 subproblems in flat arrays (Section 3: the merge working
//                 in parallel on all pairs at once).
//   partition     Steps 1-2 for every job, one lane per block start.
//   cases         Steps 3-4 for every subproblem (a whole small job passes
//                 through unchanged).
//   merge         the persistent merge kernel over all subproblems.
// Every grid size is fixed by the host from upper bounds, and the device
// reads the actual counts, so the whole sequence is capturable in a graph.
#include "sm_device.h"
#include "sm_launch.h"
#include "sm_batch.h"
#include "sm_learned_dev.h"

namespace sm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanBlock = kScanThreads * kScanItems;  // jobs per scan block

__device__ __forceinline__ void job_counts(const PieceDesc& j, int64_t tile, uint32_t cap,
                                           int64_t& pieces, int64_t& splitters, int64_t& p_a,
                                           int64_t& p_b) {
    const int64_t a = desc_a(j), b = desc_b(j);
    if (a + b <= (int64_t)cap) {
        pieces = a + b > 0 ? 1 : 0;   // an empty job costs no merge step
        splitters = 0;
        p_a = p_b = 0;
        return;
    }
    const double rt = 1.0 / (double)tile;
    p_a = a > 0 ? RcpBlocks::div(a + tile - 1, tile, rt) : 1;
    p_b = b > 0 ? RcpBlocks::div(b + tile - 1, tile, rt) : 1;
    pieces = p_a + p_b;
    splitters = p_a + p_b + 2;
}

// Exclusive scan of 256 pairs in LDS (Hillis-Steele, both sums at once).
__device__ __forceinline__ void block_exclusive_scan2(int64_t& x, int64_t& y, int64_t* sx,
                                                      int64_t* sy, int64_t& tx, int64_t& ty) {
    const int t = threadIdx.x;
    sx[t] = x;
    sy[t] = y;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int64_t ax = t >= d ? sx[t - d] : 0;
        const int64_t ay = t >= d ? sy[t - d] : 0;
        __syncthreads();
        sx[t] += ax;
        sy[t] += ay;
        __syncthreads();
    }
    tx = sx[kScanThreads - 1];
    ty = sy[kScanThreads - 1];
    const int64_t ix = sx[t] - x, iy = sy[t] - y;
    __syncthreads();
    x = ix;
    y = iy;
}

// Per job: subproblem and cross-rank counts; per scan block: local exclusive
// prefixes into pstart / sstart and the block totals into bsum.
__global__ __launch_bounds__(kScanThreads) void plan_scan_kernel(
    const PieceDesc* __restrict__ jobs, int64_t count, int64_t tile, uint32_t cap,
    int64_t* __restrict__ pstart, int64_t* __restrict__ sstart, int64_t* __restrict__ bsum_p,
    int64_t* __restrict__ bsum_s) {
    __shared__ int64_t sx[kScanThreads], sy[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
    int64_t cp[kScanItems], cs[kScanItems];
    int64_t sp = 0, ss = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        cp[i] = cs[i] = 0;
        if (base + i < count) {
            int64_t pa, pb;
            job_counts(jobs[base + i], tile, cap, cp[i], cs[i], pa, pb);
        }
        sp += cp[i];
        ss += cs[i];
    }
    int64_t tp, ts;
    block_exclusive_scan2(sp, ss, sx, sy, tp, ts);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < count) {
            pstart[base + i] = sp;
            sstart[base + i] = ss;
        }
        sp += cp[i];
        ss += cs[i];
    }
    if (threadIdx.x == 0) {
        bsum_p[blockIdx.x] = tp;
        bsum_s[blockIdx.x] = ts;
    }
}

// One workgroup: exclusive scan of the block totals in place; totals[0] = P,
// totals[1] = S (all subproblems, all cross ranks).
__global__ __launch_bounds__(kScanThreads) void scan_top_kernel(int64_t* __restrict__ bsum_p,
                                                                int64_t* __restrict__ bsum_s,
                                                                int64_t nblocks,
                                                                int64_t* __restrict__ totals) {
    __shared__ int64_t sx[kScanThreads], sy[kScanThreads];
    int64_t carry_p = 0, carry_s = 0;
    for (int64_t off = 0; off < nblocks; off += kScanThreads) {
        const int64_t k = off + threadIdx.x;
        int64_t x = k < nblocks ? bsum_p[k] : 0;
        int64_t y = k < nblocks ? bsum_s[k] : 0;
        int64_t tx, ty;
        block_exclusive_scan2(x, y, sx, sy, tx, ty);
        if (k < nblocks) {
            bsum_p[k] = x + carry_p;
            bsum_s[k] = y + carry_s;
        }
        carry_p += tx;
        carry_s += ty;
    }
    if (threadIdx.x == 0) {
        totals[0] = carry_p;
        totals[1] = carry_s;
    }
}

__global__ __launch_bounds__(256) void scan_add_kernel(int64_t* __restrict__ pstart,
                                                       int64_t* __restrict__ sstart,
                                                       const int64_t* __restrict__ bsum_p,
                                                       const int64_t* __restrict__ bsum_s,
                                                       int64_t count,
                                                       const int64_t* __restrict__ totals) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= count;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (k == count) {
            pstart[count] = totals[0];
            sstart[count] = totals[1];
        } else {
            pstart[k] += bsum_p[k / kScanBlock];
            sstart[k] += bsum_s[k / kScanBlock];
        }
    }
}

// Job owning flat index w: the last k with start[k] <= w (start has count + 1
// non-decreasing entries, start[count] = total).
__device__ __forceinline__ int64_t owner(const int64_t* start, int64_t count, int64_t w) {
    int64_t lo = 0, n = count;
    while (n > 0) {
        const int64_t half = n >> 1;
        if (start[lo + half + 1] <= w) { lo += half + 1; n -= half + 1; }
        else n = half;
    }
    return lo;
}

// Owner of flat index w when every job but the last has `uni` entries (and
// the last one starts at (count - 1) * uni): a division; otherwise (uni =
// 0) the search over the starts.
__device__ __forceinline__ int64_t owner_of(const int64_t* start, int64_t count, int64_t w,
                                            int64_t uni, double rcp_uni) {
    if (uni > 0) {
        const int64_t k = RcpBlocks::div(w, uni, rcp_uni);
        return k < count - 1 ? k : count - 1;
    }
    return owner(start, count, w);
}

// Rank of x in X[0, len) (rank_high if HIGH) by bounded search from the
// model's guess; adds the probes to `probes`.
template <bool HIGH, typename K>
__device__ __forceinline__ int64_t learned_rank(const K* X, int64_t len, K x, const float* model,
                                                float step_frac, unsigned long long& probes) {
    if constexpr (IsDesc<K>::value) {
        return HIGH ? rank_high<K, int64_t>(X, len, x) : rank_low<K, int64_t>(X, len, x);
    } else {
        const int64_t g = predict(model, feature(x), len);
        const float s = step_frac * (float)len;
        const int64_t step0 = s >= 2.0f ? (int64_t)1 << (int)floorf(log2f(s)) : 1;
        int np;
        bool fb;
        // a window of 2 len never ends the walk early: a step of len or more
        // from any guess already leaves the array
        const int64_t r = bounded_search<K, HIGH>(X, len, x, g, step0, 2 * len + 2, np, fb);
        probes += (unsigned long long)np;
        return r;
    }
}

// Steps 1-2 for every split job: flat cross-rank index s -> (job, block).
// With `model` the searches start at learned guesses (same ranks).
template <typename K>
__global__ __launch_bounds__(256) void batch_partition_kernel(
    const K* __restrict__ keys, const PieceDesc* __restrict__ jobs, int64_t count, int64_t tile,
    uint32_t cap, const int64_t* __restrict__ sstart, const int64_t* __restrict__ totals,
    int64_t s_max, int64_t* __restrict__ ranks, const float* __restrict__ model, float step_frac,
    unsigned long long* __restrict__ counters, int64_t uni_s) {
    // the counts bound S by s_max; the clamp only keeps a corrupted job list
    // inside the workspace
    const int64_t S = min(totals[1], s_max);
    const double rcp_s = uni_s > 0 ? 1.0 / (double)uni_s : 0.0;
    unsigned long long n_search = 0, n_probe = 0;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = owner_of(sstart, count, s, uni_s, rcp_s);
        const PieceDesc j = jobs[k];
        int64_t np, ns, p_a, p_b;
        job_counts(j, tile, cap, np, ns, p_a, p_b);
        const int64_t a = desc_a(j), b = desc_b(j);
        const K* A = keys + j.ka0;
        const K* B = keys + j.kb0;
        const int64_t u = s - sstart[k];
        int64_t r;
        if (u <= p_a) {
            const int64_t xu = RcpBlocks(a, p_a).start(u);
            if (xu >= a) r = b;
            else if (model) {
                r = learned_rank<false, K>(B, b, A[xu], model, step_frac, n_probe);
                ++n_search;
            } else r = rank_low<K, int64_t>(B, b, A[xu]);
        } else {
            const int64_t v = u - (p_a + 1);
            const int64_t yv = RcpBlocks(b, p_b).start(v);
            if (yv >= b) r = a;
            else if (model) {
                r = learned_rank<true, K>(A, a, B[yv], model, step_frac, n_probe);
                ++n_search;
            } else r = rank_high<K, int64_t>(A, a, B[yv]);
        }
        ranks[s] = r;
    }
    if (counters) {
        // summed per wave, one atomic per wave and counter
        for (int o = 32; o > 0; o >>= 1) {
            n_search += __shfl_xor(n_search, o);
            n_probe += __shfl_xor(n_probe, o);
        }
        if ((threadIdx.x & 63) == 0 && n_search) {
            atomicAdd(&counters[0], n_search);
            atomicAdd(&counters[1], n_probe);
        }
    }
}

// Steps 3-4 for every subproblem of every job.  A subproblem's successor
// exists when its range ends inside the job's segment, or at its end when
// the job's own successor exists.
__global__ __launch_bounds__(256) void batch_cases_kernel(
    const PieceDesc* __restrict__ jobs, int64_t count, int64_t tile, uint32_t cap,
    const int64_t* __restrict__ pstart, const int64_t* __restrict__ sstart,
    const int64_t* __restrict__ totals, const int64_t* __restrict__ ranks, int64_t p_max,
    PieceDesc* __restrict__ desc, int64_t uni_p) {
    const int64_t P = min(totals[0], p_max);
    const double rcp_p = uni_p > 0 ? 1.0 / (double)uni_p : 0.0;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < P;
         w += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = owner_of(pstart, count, w, uni_p, rcp_p);
        const PieceDesc j = jobs[k];
        int64_t np, ns, p_a, p_b;
        job_counts(j, tile, cap, np, ns, p_a, p_b);
        if (np == 1) {
            PieceDesc d = j;
            d.b_f |= kFirstBit;
            desc[w] = d;
            continue;
        }
        const int64_t a = desc_a(j), b = desc_b(j);
        const int64_t* xbar = ranks + sstart[k];
        const int64_t* ybar = xbar + (p_a + 1);
        const RcpBlocks BA(a, p_a), BB(b, p_b);
        const int64_t v = w - pstart[k];
        const Piece<int64_t> pc = v < p_a ? step3_piece<int64_t>(BA, BB, xbar, ybar, v)
                                          : step4_piece<int64_t>(BA, BB, xbar, ybar, v - p_a);
        // the job's subproblems in output order (as cases_kernel orders a
        // single merge's), the first one marked
        const int64_t ne_a = a > 0 ? BA.of(a - 1) + 1 : 0, ne_b = b > 0 ? BB.of(b - 1) + 1 : 0;
        auto starts_below = [](const RcpBlocks& Bk, int64_t x) {
            return x <= 0 ? (int64_t)0 : Bk.of(x - 1) + 1;
        };
        int64_t place;
        if (v < p_a) {
            place = v < ne_a ? v + starts_below(BB, xbar[v] < b ? xbar[v] : b) : ne_b + v;
        } else {
            const int64_t u = v - p_a;
            place = u < ne_b ? u + starts_below(BA, ybar[u] < a ? ybar[u] : a) : p_a + u;
        }
        if (place < 0 || place >= np) place = v;   // inputs that are not sorted
        PieceDesc d;
        d.ka0 = j.ka0 + pc.a_lo;
        d.kb0 = j.kb0 + pc.b_lo;
        d.out0 = j.out0 + pc.a_lo + pc.b_lo;
        if (!(0 <= pc.a_lo && pc.a_lo <= pc.a_hi && pc.a_hi <= a && 0 <= pc.b_lo &&
              pc.b_lo <= pc.b_hi && pc.b_hi <= b)) {
            d.a_f = d.b_f = 0;  // a bug would empty the subproblem, never write outside C
        } else {
            const bool sa = pc.a_hi < a || (j.a_f & kSuccBit);
            const bool sb = pc.b_hi < b || (j.b_f & kSuccBit);
            d.a_f = (uint32_t)(pc.a_hi - pc.a_lo) | (sa ? kSuccBit : 0u);
            d.b_f = (uint32_t)(pc.b_hi - pc.b_lo) | (sb ? kSuccBit : 0u);
        }
        if (place == 0) d.b_f |= kFirstBit;
        desc[pstart[k] + place] = d;
    }
}

// Jobs of the batched entry point: pair k is keys[offsets[k], offsets[k+1])
// with its first n_a[k] elements as A.  Pairs are independent arrays, so no
// segment has a successor.  A pair whose sizes are inconsistent becomes an
// empty job and sets *bad.
__global__ __launch_bounds__(256) void jobs_from_pairs_kernel(const int64_t* __restrict__ offsets,
                                                              const int64_t* __restrict__ n_a,
                                                              int64_t count, int64_t total,
                                                              PieceDesc* __restrict__ jobs,
                                                              int* __restrict__ bad) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t lo = offsets[k], hi = offsets[k + 1], na = n_a[k];
        PieceDesc j;
        j.ka0 = lo;
        j.kb0 = lo + na;
        j.out0 = lo;
        if (lo < 0 || hi < lo || hi > total || na < 0 || na > hi - lo || hi - lo >= (1ll << 30)) {
            j.a_f = j.b_f = 0;
            j.ka0 = j.kb0 = j.out0 = 0;
            *bad = 1;
        } else {
            j.a_f = (uint32_t)na;
            j.b_f = (uint32_t)(hi - lo - na);
        }
        jobs[k] = j;
    }
}

// Sortedness of every A and B of a batch: element i is compared with i + 1
// unless i + 1 starts a B or the next pair.
template <typename K>
__global__ __launch_bounds__(256) void batch_validate_kernel(const K* __restrict__ keys,
                                                             const int64_t* __restrict__ offsets,
                                                             const int64_t* __restrict__ n_a,
                                                             int64_t count,
                                                             int* __restrict__ bad) {
    const int64_t lo = offsets[0], hi = offsets[count];
    bool ok = true;
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i + 1 < hi;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = owner(offsets, count, i);
        const int64_t next = offsets[k + 1];
        const int64_t b0 = offsets[k] + n_a[k];
        if (i + 1 != next && i + 1 != b0 && keys[i + 1] < keys[i]) ok = false;
    }
    if (!ok) *bad = 1;
}

__global__ void clear_kernel(int* __restrict__ p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}


inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

BatchLayout batch_layout(int64_t count, int64_t total, int64_t tile) {
    BatchLayout L;
    const int64_t nblocks = (count + kScanBlock - 1) / kScanBlock;
    L.count = count;
    L.nblocks = nblocks;
    L.p_max = (total + tile - 1) / tile + 2 * count + 1;
    L.s_max = L.p_max + 2 * count;
    size_t off = 0;
    L.off_pstart = off; off += align256((size_t)(count + 1) * 8);
    L.off_sstart = off; off += align256((size_t)(count + 1) * 8);
    L.off_bsum_p = off; off += align256((size_t)(nblocks + 1) * 8);
    L.off_bsum_s = off; off += align256((size_t)(nblocks + 1) * 8);
    L.off_totals = off; off += 256;
    L.off_flag = off; off += 256;
    L.off_ranks = off; off += align256((size_t)L.s_max * 8);
    L.off_desc = off; off += align256((size_t)L.p_max * kPieceDescBytes);
    L.bytes = off;
    return L;
}

hipError_t launch_jobs_from_pairs(const int64_t* offsets, const int64_t* n_a, int64_t count,
                                  int64_t total, PieceDesc* jobs, int* bad, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    int64_t g = (count + 255) / 256;
    if (g > 4096) g = 4096;
    jobs_from_pairs_kernel<<<(unsigned)g, 256, 0, st>>>(offsets, n_a, count, total, jobs, bad);
    return hipGetLastError();
}

hipError_t launch_batch_validate(int dtype, const void* keys, const int64_t* offsets,
                                 const int64_t* n_a, int64_t count, int64_t total, int* bad,
                                 hipStream_t st) {
    if (count <= 0 || total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    const int64_t gmax = (int64_t)device_cu_count() * 8;
    if (g > gmax) g = gmax;
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        batch_validate_kernel<K><<<(unsigned)g, 256, 0, st>>>(static_cast<const K*>(keys), offsets,
                                                              n_a, count, bad);
    });
    return hipGetLastError();
}

hipError_t launch_clear(int* p, int n, hipStream_t st) {
    clear_kernel<<<1, 256, 0, st>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_batch(int dtype, const void* keys, const uint32_t* pay, int64_t nkeys,
                        void* out_keys, uint32_t* out_pay, int64_t nout, const PieceDesc* jobs,
                        int64_t count, int64_t tile, char* ws, const BatchLayout& L,
                        hipStream_t st, const LearnedSearch* ls) {
    if (count <= 0) return hipSuccess;
    if (ls && (dtype & kDescending)) return hipErrorInvalidValue;  // ascending models only
    const uint32_t cap = merge_cap_for_tile((int32_t)tile);
    int64_t* pstart = reinterpret_cast<int64_t*>(ws + L.off_pstart);
    int64_t* sstart = reinterpret_cast<int64_t*>(ws + L.off_sstart);
    int64_t* bsum_p = reinterpret_cast<int64_t*>(ws + L.off_bsum_p);
    int64_t* bsum_s = reinterpret_cast<int64_t*>(ws + L.off_bsum_s);
    int64_t* totals = reinterpret_cast<int64_t*>(ws + L.off_totals);

    plan_scan_kernel<<<(unsigned)L.nblocks, kScanThreads, 0, st>>>(jobs, count, tile, cap, pstart,
                                                                    sstart, bsum_p, bsum_s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    scan_top_kernel<<<1, kScanThreads, 0, st>>>(bsum_p, bsum_s, L.nblocks, totals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t g = (count + 1 + 255) / 256;
    if (g > 4096) g = 4096;
    scan_add_kernel<<<(unsigned)g, 256, 0, st>>>(pstart, sstart, bsum_p, bsum_s, count, totals);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    return launch_batch_planned(dtype, keys, pay, nkeys, out_keys, out_pay, nout, jobs, count, tile,
                                ws, L, st, ls, 0, 0);
}

hipError_t launch_batch_planned(int dtype, const void* keys, const uint32_t* pay, int64_t nkeys,
                                void* out_keys, uint32_t* out_pay, int64_t nout,
                                const PieceDesc* jobs, int64_t count, int64_t tile, char* ws,
                                const BatchLayout& L, hipStream_t st, const LearnedSearch* ls,
                                int64_t uni_p, int64_t uni_s) {
    if (count <= 0) return hipSuccess;
    if (ls && (dtype & kDescending)) return hipErrorInvalidValue;  // ascending models only
    const uint32_t cap = merge_cap_for_tile((int32_t)tile);
    const int64_t* pstart = reinterpret_cast<const int64_t*>(ws + L.off_pstart);
    const int64_t* sstart = reinterpret_cast<const int64_t*>(ws + L.off_sstart);
    const int64_t* totals = reinterpret_cast<const int64_t*>(ws + L.off_totals);
    int64_t* ranks = reinterpret_cast<int64_t*>(ws + L.off_ranks);
    PieceDesc* desc = reinterpret_cast<PieceDesc*>(ws + L.off_desc);
    hipError_t e;
    const int64_t grid = (int64_t)device_cu_count() * 8;
    int64_t gs = (L.s_max + 255) / 256;
    if (gs > grid) gs = grid;
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        batch_partition_kernel<K><<<(unsigned)gs, 256, 0, st>>>(
            static_cast<const K*>(keys), jobs, count, tile, cap, sstart, totals, L.s_max, ranks,
            ls ? ls->model : nullptr, ls ? ls->step_frac : 0.0f, ls ? ls->counters : nullptr, uni_s);
    });
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t gp = (L.p_max + 255) / 256;
    if (gp > grid) gp = grid;
    batch_cases_kernel<<<(unsigned)gp, 256, 0, st>>>(jobs, count, tile, cap, pstart, sstart, totals,
                                                     ranks, L.p_max, desc, uni_p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_merge_desc(dtype, keys, pay, nkeys, out_keys, out_pay, nout, desc, L.p_max,
                             totals, merge_pack_cap(dtype, pay != nullptr, cap), st, /*packed=*/true);
}

}  // namespace sm
