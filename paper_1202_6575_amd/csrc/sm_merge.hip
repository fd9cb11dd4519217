// sm_merge.hip -- the plain stable merge on gfx950.
//
// K1 partition_kernel: Steps 1-2 of Section 2, one lane per block start, a
//    binary search in global memory per lane.  The kernel boundary is the
//    method's single synchronisation.
// K2 cases_kernel: Steps 3-4 case selection, one thread per subproblem,
//    writes a descriptor (the five cases in two-select form).
// K3 merge_persistent_kernel / merge_direct_kernel: the merges, one
//    workgroup per subproblem at a time (the workgroup merge of sm_device.h).
#include <atomic>
#include "sm_device.h"
#include "sm_launch.h"

namespace sm {

template <typename K>
__global__ __launch_bounds__(256) void partition_kernel(const K* __restrict__ keys, int64_t n,
                                                        int64_t m, int64_t p_a, int64_t p_b,
                                                        int64_t* __restrict__ xbar,
                                                        int64_t* __restrict__ ybar) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const K* A = keys;
    const K* B = keys + n;
    if (t <= p_a) {
        const Blocks<int64_t> BA(n, p_a);
        const int64_t xi = BA.start(t);
        xbar[t] = xi < n ? rank_low<K, int64_t>(B, m, A[xi]) : m;
    } else if (t <= p_a + 1 + p_b) {
        const int64_t j = t - (p_a + 1);
        const Blocks<int64_t> BB(m, p_b);
        const int64_t yj = BB.start(j);
        ybar[j] = yj < m ? rank_high<K, int64_t>(A, n, B[yj]) : n;
    }
}

// Steps 1-2 for a few block starts, where the dependent loads of the
// searches, not their traffic, set the time: G lanes share one search and
// probe G evenly spaced elements per round, which leaves an interval 1/G as
// long, so a rank over len elements takes about log_G(len) rounds of loads
// instead of log2(len).  The ranks are those of partition_kernel (the same
// definitions, rank_low for A block starts and rank_high for B's).
template <typename K, int G>
__global__ __launch_bounds__(256) void partition_group_kernel(const K* __restrict__ keys,
                                                              int64_t n, int64_t m, int64_t p_a,
                                                              int64_t p_b,
                                                              int64_t* __restrict__ xbar,
                                                              int64_t* __restrict__ ybar) {
    static_assert(G >= 2 && G <= 64 && 64 % G == 0, "a search group lies inside one wave");
    const int64_t qy = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    const int g = (int)(threadIdx.x % G);
    const int first = (int)(threadIdx.x & 63) - g;   // the group's first lane in the wave
    // every branch below is taken by whole groups
    if (qy > p_a + 1 + p_b) return;
    const bool low = qy <= p_a;   // an A block start searched in B
    const int64_t j = qy - (p_a + 1);
    const int64_t start = low ? RcpBlocks(n, p_a).start(qy) : RcpBlocks(m, p_b).start(j);
    const int64_t own = low ? n : m, len = low ? m : n;
    int64_t lo = len;
    if (start < own) {
        const K x = keys[low ? start : n + start];
        const K* S = low ? keys + n : keys;
        int64_t hi = len;
        lo = 0;
        // [lo, hi) holds the elements not yet compared; the rank is in [lo, hi]
        while (lo < hi) {
            const int64_t step = (hi - lo + G - 1) / G;
            const int64_t e = lo + (int64_t)(g + 1) * step - 1;
            bool below = false;   // S[e] counts towards the rank
            if (e < hi) {
                const K v = S[e];
                below = low ? v < x : !(x < v);
            }
            // the probes that count form a prefix of the group's lanes
            const uint64_t bits = (__ballot(below) >> first) & (G == 64 ? ~0ull : (1ull << G) - 1);
            const int c = __popcll(bits);
            lo += (int64_t)c * step;
            // probe c (if there is one) did not count: the rank is at most its index
            const int64_t ec = lo + step - 1;
            if (c < G && ec < hi) hi = ec;
        }
    }
    if (g == 0) {
        if (low) xbar[qy] = lo;
        else ybar[j] = lo;
    }
}

// Steps 3-4 of subproblem w (A block w for w < p_a, else B block w - p_a)
// as a descriptor: the five cases in two-select form.
__device__ __forceinline__ PieceDesc case_desc(const RcpBlocks& BA, const RcpBlocks& BB,
                                               const int64_t* __restrict__ xbar,
                                               const int64_t* __restrict__ ybar, int64_t w) {
    const int64_t n = BA.len, m = BB.len, p_a = BA.p;
    const Piece<int64_t> pc = w < p_a ? step3_piece<int64_t>(BA, BB, xbar, ybar, w)
                                      : step4_piece<int64_t>(BA, BB, xbar, ybar, w - p_a);
    PieceDesc d;
    d.ka0 = pc.a_lo;
    d.kb0 = n + pc.b_lo;
    d.out0 = pc.a_lo + pc.b_lo;
    // a subproblem outside the arrays would be a bug: it is emptied, so the
    // merge kernel never writes outside C (the output is then wrong, not unsafe)
    if (!(0 <= pc.a_lo && pc.a_lo <= pc.a_hi && pc.a_hi <= n && 0 <= pc.b_lo &&
          pc.b_lo <= pc.b_hi && pc.b_hi <= m && pc.a_hi - pc.a_lo < (1 << 30) &&
          pc.b_hi - pc.b_lo < (1 << 30))) {
        d.a_f = 0;
        d.b_f = 0;
    } else {
        d.a_f = (uint32_t)(pc.a_hi - pc.a_lo) | (pc.a_hi < n ? kSuccBit : 0u);
        d.b_f = (uint32_t)(pc.b_hi - pc.b_lo) | (pc.b_hi < m ? kSuccBit : 0u);
    }
    return d;
}

// Steps 3-4 case selection: one thread per subproblem writes its descriptor
// (the five cases in two-select form).  Subproblems 0..p_a-1 belong to the
// processing elements of A blocks (Step 3), p_a..p_a+p_b-1 to B blocks
// (Step 4).  The output position of every subproblem is a_lo + b_lo (the
// stable-merge position identity of Section 2).
//
// The descriptors are stored in output order.  The subproblem of A block i
// starts with A[x_i], placed after the B block starts y_j < xbar_i (B[y_j]
// precedes A[x_i] exactly when y_j < rank_low(A[x_i])) and after the A
// pieces before it: its place is i + #{j : y_j < xbar_i}.  Likewise the
// subproblem of B block j has place j + #{i : x_i < ybar_j}.  Blocks that
// start at the end of their array (more blocks than elements) hold empty
// subproblems; they take the places after all others, A's first.
__global__ __launch_bounds__(256) void cases_kernel(RcpBlocks BA, RcpBlocks BB,
                                                    const int64_t* __restrict__ xbar,
                                                    const int64_t* __restrict__ ybar,
                                                    PieceDesc* __restrict__ desc) {
    const int64_t n = BA.len, m = BB.len, p_a = BA.p, p_b = BB.p;
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= p_a + p_b) return;
    // blocks that hold an element; block starts below x (x <= len)
    const int64_t ne_a = n > 0 ? BA.of(n - 1) + 1 : 0, ne_b = m > 0 ? BB.of(m - 1) + 1 : 0;
    auto starts_below = [](const RcpBlocks& Bk, int64_t x) {
        return x <= 0 ? (int64_t)0 : Bk.of(x - 1) + 1;
    };
    int64_t place;
    if (w < p_a) {
        place = w < ne_a ? w + starts_below(BB, xbar[w] < m ? xbar[w] : m) : ne_b + w;
    } else {
        const int64_t j = w - p_a;
        place = j < ne_b ? j + starts_below(BA, ybar[j] < n ? ybar[j] : n) : p_a + j;
    }
    // out of range only for inputs that are not sorted (the subproblems then
    // overlap); the merge kernel checks every descriptor it reads
    if (place < 0 || place >= p_a + p_b) place = w;
    desc[place] = case_desc(BA, BB, xbar, ybar, w);
}

// Persistent merge: workgroup g of G merges subproblems g, g + G, g + 2G, ...
// (interleaved: at any moment the grid works on neighbouring subproblems,
// so it sweeps the arrays front to back, and a workgroup's share is a
// sample of the whole list rather than one stretch of it, which evens out
// lists of uneven subproblems).  While it merges subproblem w, the 16-byte
// loads of its next subproblem are in flight in registers (R chunks per
// thread) and the stores of its previous one are draining.
template <typename K, bool PAY, int L, int R>
__global__ __launch_bounds__(L) void merge_persistent_kernel(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, int64_t nkeys,
    K* __restrict__ out, uint32_t* __restrict__ out_pay, int64_t nout,
    const PieceDesc* __restrict__ desc, int64_t P, const int64_t* __restrict__ P_dev, uint32_t cap) {
    extern __shared__ __align__(16) char smem[];
    const SmemPtrs<K, PAY, L> sp(smem, cap);
    // the subproblem count comes from device memory when it was computed there
    // (batched merges); P is then its upper bound
    if (P_dev) {
        const int64_t pd = *P_dev;
        P = pd < P ? (pd > 0 ? pd : 0) : P;
    }
    const int64_t G = gridDim.x;
    const int64_t w0 = blockIdx.x;
    if (w0 >= P) return;
    u32x4 rk[R], rp[R];
    PieceDesc d = desc[w0];
    if (!desc_ok(d, nkeys, nout, cap)) d.a_f = d.b_f = 0;
    SegPlan cur = make_plan<K, PAY>(d);
    SegPlan prev = cur;
    prefetch<K, PAY, L, R>(cur, keys, (uint64_t)nkeys, pay, rk, rp);
    for (int64_t w = w0; w < P; w += G) {
        const bool more = w + G < P;
        PieceDesc dn;
        dn.ka0 = dn.kb0 = dn.out0 = 0;
        dn.a_f = dn.b_f = 0;
        if (more) {
            dn = desc[w + G];
            if (!desc_ok(dn, nkeys, nout, cap)) dn.a_f = dn.b_f = 0;
        }
        const SegPlan nxt = make_plan<K, PAY>(dn);
        // Order: wait for this piece's loads (commit), issue the next piece's
        // loads, then the previous piece's stores, then merge.  Stores and loads
        // share one completion counter, so nothing waits on a store until the
        // next commit, a whole merge later.  The write-back reads sOut / sIdx,
        // which this piece's merge rewrites only after its first barrier.
        // one wait for everything in flight (this piece's loads, and stores
        // issued a whole merge ago): afterwards no register has a load pending,
        // so the compiler adds no waits further down the iteration
        __builtin_amdgcn_s_setprio(2);   // staging and memory first, as in merge_pipelined
        wait_vm<0>();
        commit<K, PAY, L, R>(cur, rk, rp, sp.sKey, sp.sPay);
        __syncthreads();
        if (more) prefetch<K, PAY, L, R>(nxt, keys, (uint64_t)nkeys, pay, rk, rp);
        if (w > w0) write_back<K, PAY, L, R>(prev, sp.sOut, sp.sIdx, out, out_pay);
        __builtin_amdgcn_s_setprio(0);
        if (cur.s > 0) merge_lanes<K, PAY, L>(cur, sp.sKey, sp.sPay, sp.sOut, sp.sIdx, sp.sXb, sp.sYb);
        prev = cur;
        cur = nxt;
    }
    write_back<K, PAY, L, R>(prev, sp.sOut, sp.sIdx, out, out_pay);
}

// Packed steps.  With the descriptors in output order, consecutive
// subproblems chain: each starts in A, in B and in C where the one before
// ends.  The union of a run of them is then itself a merge subproblem (a
// contiguous A range, B range and output range), and the element after each
// of its ranges is the one after the last member's range, so the sentinel
// rule holds for it as for its members.  A step of the packed form merges
// the union of up to kPackMax consecutive subproblems that fits the
// workgroup's capacity: the subproblems average half the capacity (each has
// at most one block of A and one of B), so a step moves about twice the
// data.  The lane-level split is applied to the union.  Descriptors that do
// not chain (another caller's list) are merged one per step.
constexpr int kPackMax = 4;

struct PackGroup {
    PieceDesc d;
    int64_t next;   // list index after the group
};

// d[0 .. avail) are the list entries from index k on (avail <= kPackMax).
__device__ __forceinline__ PackGroup pack_group(const PieceDesc (&d)[kPackMax], int avail,
                                                int64_t k, int64_t nkeys, int64_t nout,
                                                uint32_t cap) {
    PackGroup g;
    g.d.ka0 = g.d.kb0 = g.d.out0 = 0;
    g.d.a_f = g.d.b_f = 0;
    g.next = k;
    if (avail <= 0) return g;
    g.next = k + 1;
    if (!desc_ok(d[0], nkeys, nout, cap)) return g;
    // the union's ends so far (fixed indices only: a runtime index into d
    // would move the array to memory)
    int64_t ea = d[0].ka0 + piece_a(d[0]), eb = d[0].kb0 + piece_b(d[0]);
    int64_t ec = d[0].out0 + piece_a(d[0]) + piece_b(d[0]);
    uint32_t sa = d[0].a_f & kSuccBit, sb = d[0].b_f & kSuccBit;
    int cnt = 1;
    bool open = true;
#pragma unroll
    for (int t = 1; t < kPackMax; ++t) {
        const PieceDesc& e = d[t];
        const int64_t ee = e.out0 + piece_a(e) + piece_b(e);
        const bool ok = open && t < avail && !(e.b_f & kFirstBit) && desc_ok(e, nkeys, nout, cap) &&
                        e.ka0 == ea && e.kb0 == eb && e.out0 == ec &&
                        ee - d[0].out0 <= (int64_t)cap;
        if (ok) {
            ea = e.ka0 + piece_a(e);
            eb = e.kb0 + piece_b(e);
            ec = ee;
            sa = e.a_f & kSuccBit;
            sb = e.b_f & kSuccBit;
            cnt = t + 1;
        }
        open = ok;
    }
    g.d.ka0 = d[0].ka0;
    g.d.kb0 = d[0].kb0;
    g.d.out0 = d[0].out0;
    g.d.a_f = (uint32_t)(ea - d[0].ka0) | sa;
    g.d.b_f = (uint32_t)(eb - d[0].kb0) | sb;
    g.next = k + cnt;
    return g;
}

// The two-register-set pipeline of merge_pipelined (below) over packed
// steps of the workgroup's own stretch of the list.  The descriptors of the
// step after next are read a step ahead: lanes 0..7 load the kPackMax
// entries from the step's first index (16 bytes each), and the fields are
// read out of those lanes.
template <typename K, bool PAY, int L, int R, bool WHOLE>
__device__ __forceinline__ void merge_pipelined_packed(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, int64_t nkeys,
    K* __restrict__ out, uint32_t* __restrict__ out_pay, int64_t nout,
    const PieceDesc* __restrict__ desc, int64_t P, const int64_t* __restrict__ P_dev, uint32_t cap) {
    extern __shared__ __align__(16) char smem[];
    const SmemPtrs<K, PAY, L> sp(smem, cap);
    if (P_dev) {
        const int64_t pd = *P_dev;
        P = pd < P ? (pd > 0 ? pd : 0) : P;
    }
    const int64_t G = gridDim.x;
    const int64_t lo = P * (int64_t)blockIdx.x / G;
    const int64_t hi = P * ((int64_t)blockIdx.x + 1) / G;
    if (lo >= hi) return;
    static_assert(kPackMax * (int)sizeof(PieceDesc) == 8 * 16, "eight lanes load the entries");
    const __amdgpu_buffer_rsrc_t rdesc = make_rsrc(desc, (uint64_t)hi * sizeof(PieceDesc));
    const int lane = threadIdx.x & 63;
    // entries [k, min(k + kPackMax, hi)): lane l < 8 holds bytes [16 l, 16 l + 16)
    auto desc_load = [&](int64_t k, u32x4& v) {
        const bool in = lane < 8 && k < hi;
        v = buf_load16(rdesc, in ? (uint32_t)(k * (int64_t)sizeof(PieceDesc)) + 16u * (uint32_t)lane
                                 : kOffNone);
    };
    auto group_from = [&](const u32x4& v, int64_t k) {
        PieceDesc d[kPackMax];
#pragma unroll
        for (int t = 0; t < kPackMax; ++t) {
            const uint32_t a0 = __builtin_amdgcn_readlane(v.x, 2 * t), a1 = __builtin_amdgcn_readlane(v.y, 2 * t);
            const uint32_t b0 = __builtin_amdgcn_readlane(v.z, 2 * t), b1 = __builtin_amdgcn_readlane(v.w, 2 * t);
            const uint32_t c0 = __builtin_amdgcn_readlane(v.x, 2 * t + 1), c1 = __builtin_amdgcn_readlane(v.y, 2 * t + 1);
            d[t].ka0 = (int64_t)(((uint64_t)a1 << 32) | a0);
            d[t].kb0 = (int64_t)(((uint64_t)b1 << 32) | b0);
            d[t].out0 = (int64_t)(((uint64_t)c1 << 32) | c0);
            d[t].a_f = __builtin_amdgcn_readlane(v.z, 2 * t + 1);
            d[t].b_f = __builtin_amdgcn_readlane(v.w, 2 * t + 1);
        }
        const int64_t left = hi - k;
        return pack_group(d, (int)(left < kPackMax ? (left > 0 ? left : 0) : kPackMax), k, nkeys,
                          nout, cap);
    };
    auto group_at = [&](int64_t k) {
        PieceDesc d[kPackMax];
#pragma unroll
        for (int t = 0; t < kPackMax; ++t) {
            if (k + t < hi) {
                d[t] = desc[k + t];
            } else {
                d[t].ka0 = d[t].kb0 = d[t].out0 = 0;
                d[t].a_f = d[t].b_f = 0;
            }
        }
        const int64_t left = hi - k;
        return pack_group(d, (int)(left < kPackMax ? (left > 0 ? left : 0) : kPackMax), k, nkeys,
                          nout, cap);
    };
    static_assert(WHOLE || !PAY, "arrays of 4 GiB or more: keys-only form");
    constexpr int RS = WHOLE ? R : R + 1;   // key register slots per set
    u32x4 rkA[RS], rpA[R], rkB[RS], rpB[R];
    const PackGroup g0 = group_at(lo);
    const PackGroup g1 = group_at(g0.next);
    SegPlan cur = make_plan<K, PAY>(g0.d);
    SegPlan nxt = make_plan<K, PAY>(g1.d);
    int64_t kcur = lo, knxt = g0.next, knn = g1.next;
    u32x4 dv;
    desc_load(knn, dv);
    // the descriptor load must stay older than both sets' loads (the waits
    // below count on it): no instruction moves across this point
    __builtin_amdgcn_sched_barrier(0);
    SegPlan prev = cur;
    const __amdgpu_buffer_rsrc_t rkeys = make_rsrc(keys, (uint64_t)nkeys * sizeof(K));
    const __amdgpu_buffer_rsrc_t rpay = make_rsrc(PAY ? pay : nullptr, PAY ? (uint64_t)nkeys * 4 : 0);
    auto load = [&](const SegPlan& p, u32x4 (&rk)[RS], u32x4 (&rp)[R]) {
        if constexpr (WHOLE) prefetch_whole<K, PAY, L, R>(p, rkeys, rpay, rk, rp);
        else prefetch_split<K, L, RS>(p, keys, (uint64_t)nkeys, rk);
    };
    load(cur, rkA, rpA);
    load(nxt, rkB, rpB);
    auto step = [&](u32x4 (&rk)[RS], u32x4 (&rp)[R]) {
        __builtin_amdgcn_s_setprio(2);
        wait_vm<PAY ? 2 * R : RS>();
        if constexpr (WHOLE) commit<K, PAY, L, R>(cur, rk, rp, sp.sKey, sp.sPay);
        else commit_split<K, L, RS>(cur, rk, sp.sKey);
        __syncthreads();
        if (kcur > lo) write_back<K, PAY, L, R>(prev, sp.sOut, sp.sIdx, out, out_pay);
        // the descriptors loaded a step ago have landed (the wait above)
        const PackGroup gn = group_from(dv, knn);
        desc_load(gn.next, dv);
        __builtin_amdgcn_sched_barrier(0);
        const SegPlan nn = make_plan<K, PAY>(gn.d);
        load(nn, rk, rp);
        __builtin_amdgcn_s_setprio(0);
        if (cur.s > 0)
            merge_lanes<K, PAY, L, (!PAY || R <= 3)>(cur, sp.sKey, sp.sPay, sp.sOut, sp.sIdx,
                                                    sp.sXb, sp.sYb);
        prev = cur;
        cur = nxt;
        nxt = nn;
        kcur = knxt;
        knxt = knn;
        knn = gn.next;
    };
    // steps in pairs, so that the sets alternate A, B, A, ... with no exit
    // between them; a step past the stretch is empty (its loads read nothing,
    // it merges nothing, and its write-back is the last real step's)
    do {
        step(rkA, rpA);
        step(rkB, rpB);
    } while (kcur < hi);
    write_back<K, PAY, L, R>(prev, sp.sOut, sp.sIdx, out, out_pay);
}

// The same with two subproblems in flight: while the workgroup merges
// subproblem w, the loads of w + G and w + 2G (its next two) are in flight
// in two register sets, so every load has two merges' time to land.  Per
// step: wait for the oldest set, commit it to LDS, write back w - G, issue
// the loads of w + 2G into the freed set, merge w.  The write-back (and a
// descriptor load) precede the loads, so at the next wait the operations
// younger than the awaited loads are one write-back, one descriptor load
// and then the other set's loads: waiting until no more than that set's
// load count is in flight leaves at most that set in flight.
// WHOLE: the arrays are below 4 GiB and one buffer resource spans each;
// otherwise (keys only) every window gets a resource of its own and the
// register sets one more slot (prefetch_split).
//
// PACK: the workgroup takes the contiguous stretch [P g / G, P (g + 1) / G)
// of an output-ordered list and merges it in packed steps (see pack_group).
template <typename K, bool PAY, int L, int R, bool WHOLE, bool PACK>
__device__ __forceinline__ void merge_pipelined(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, int64_t nkeys,
    K* __restrict__ out, uint32_t* __restrict__ out_pay, int64_t nout,
    const PieceDesc* __restrict__ desc, int64_t P, const int64_t* __restrict__ P_dev, uint32_t cap) {
    if constexpr (PACK) {
        merge_pipelined_packed<K, PAY, L, R, WHOLE>(keys, pay, nkeys, out, out_pay, nout, desc, P,
                                                    P_dev, cap);
        return;
    }
    extern __shared__ __align__(16) char smem[];
    const SmemPtrs<K, PAY, L> sp(smem, cap);
    if (P_dev) {
        const int64_t pd = *P_dev;
        P = pd < P ? (pd > 0 ? pd : 0) : P;
    }
    const int64_t G = gridDim.x;
    const int64_t w0 = blockIdx.x;
    const int64_t w1 = P;
    if (w0 >= w1) return;
    // Descriptors are read one step before their plan is needed, with vector
    // loads (a scalar load would be waited for at the next LDS wait, which
    // covers scalar loads too): the loads of step w's next-but-two
    // descriptor go out with its prefetch and are complete at the next
    // step's wait.  Past the range a load returns zeros: an empty plan.
    const __amdgpu_buffer_rsrc_t rdesc = make_rsrc(desc, (uint64_t)w1 * sizeof(PieceDesc));
    auto desc_load = [&](int64_t w, u32x4& lo, u32x4& hi) {
        const uint32_t o = w < w1 ? (uint32_t)(w * (int64_t)sizeof(PieceDesc)) : kOffNone;
        lo = buf_load16(rdesc, o);
        hi = buf_load16(rdesc, o + 16u);
    };
    auto desc_from = [&](const u32x4& lo, const u32x4& hi) {
        PieceDesc d;
        const uint32_t w0_ = __builtin_amdgcn_readfirstlane(lo.x), w1_ = __builtin_amdgcn_readfirstlane(lo.y);
        const uint32_t w2_ = __builtin_amdgcn_readfirstlane(lo.z), w3_ = __builtin_amdgcn_readfirstlane(lo.w);
        const uint32_t w4_ = __builtin_amdgcn_readfirstlane(hi.x), w5_ = __builtin_amdgcn_readfirstlane(hi.y);
        d.ka0 = (int64_t)(((uint64_t)w1_ << 32) | w0_);
        d.kb0 = (int64_t)(((uint64_t)w3_ << 32) | w2_);
        d.out0 = (int64_t)(((uint64_t)w5_ << 32) | w4_);
        d.a_f = __builtin_amdgcn_readfirstlane(hi.z);
        d.b_f = __builtin_amdgcn_readfirstlane(hi.w);
        if (!desc_ok(d, nkeys, nout, cap)) d.a_f = d.b_f = 0;
        return make_plan<K, PAY>(d);
    };
    auto plan_of = [&](int64_t w) {
        PieceDesc d;
        d.ka0 = d.kb0 = d.out0 = 0;
        d.a_f = d.b_f = 0;
        if (w < w1) {
            d = desc[w];
            if (!desc_ok(d, nkeys, nout, cap)) d.a_f = d.b_f = 0;
        }
        return make_plan<K, PAY>(d);
    };
    static_assert(WHOLE || !PAY, "arrays of 4 GiB or more: keys-only form");
    constexpr int RS = WHOLE ? R : R + 1;   // key register slots per set
    u32x4 rkA[RS], rpA[R], rkB[RS], rpB[R];
    SegPlan cur = plan_of(w0);
    SegPlan nxt = plan_of(w0 + G);
    u32x4 dlo, dhi;
    desc_load(w0 + 2 * G, dlo, dhi);
    // the descriptor loads must stay older than both sets' loads (the waits
    // below count on it): no instruction moves across this point
    __builtin_amdgcn_sched_barrier(0);
    SegPlan prev = cur;
    // Every step issues its loads, also for a subproblem past the range (an
    // empty one, whose few loads are never used): the awaited set is then
    // always older than the other set's loads on every path, which is what
    // lets the wait below (and the compiler's own) leave that set in flight.
    const __amdgpu_buffer_rsrc_t rkeys = make_rsrc(keys, (uint64_t)nkeys * sizeof(K));
    const __amdgpu_buffer_rsrc_t rpay = make_rsrc(PAY ? pay : nullptr, PAY ? (uint64_t)nkeys * 4 : 0);
    auto load = [&](const SegPlan& p, u32x4 (&rk)[RS], u32x4 (&rp)[R]) {
        if constexpr (WHOLE) prefetch_whole<K, PAY, L, R>(p, rkeys, rpay, rk, rp);
        else prefetch_split<K, L, RS>(p, keys, (uint64_t)nkeys, rk);
    };
    load(cur, rkA, rpA);
    load(nxt, rkB, rpB);
    auto step = [&](u32x4 (&rk)[RS], u32x4 (&rp)[R], int64_t w) {
        // the staging and memory phase runs at raised priority, so that the
        // waves of a SIMD commit, pass the barrier and issue their stores
        // and loads before the others' merges
        __builtin_amdgcn_s_setprio(2);
        wait_vm<PAY ? 2 * R : RS>();
        if constexpr (WHOLE) commit<K, PAY, L, R>(cur, rk, rp, sp.sKey, sp.sPay);
        else commit_split<K, L, RS>(cur, rk, sp.sKey);
        __syncthreads();
        if (w > w0) write_back<K, PAY, L, R>(prev, sp.sOut, sp.sIdx, out, out_pay);
        // the descriptor loaded a step ago has landed (the wait above)
        const SegPlan nn = desc_from(dlo, dhi);
        desc_load(w + 3 * G, dlo, dhi);
        __builtin_amdgcn_sched_barrier(0);
        load(nn, rk, rp);
        __builtin_amdgcn_s_setprio(0);
        if (cur.s > 0)
            merge_lanes<K, PAY, L, (!PAY || R <= 3)>(cur, sp.sKey, sp.sPay, sp.sOut, sp.sIdx,
                                                    sp.sXb, sp.sYb);
        prev = cur;
        cur = nxt;
        nxt = nn;
    };
    // pairs of steps, then a lone last step: no path through the loop runs a
    // set's step twice in a row (its loads would then be the youngest)
    int64_t w = w0;
    for (; w + G < w1; w += 2 * G) {
        step(rkA, rpA, w);
        step(rkB, rpB, w + G);
    }
    if (w < w1) step(rkA, rpA, w);
    write_back<K, PAY, L, R>(prev, sp.sOut, sp.sIdx, out, out_pay);
}

// Four waves per SIMD need at most 128 registers per lane: four workgroups
// per compute unit then fit both registers and LDS.  64-bit keys with
// payloads need more (the wide form, three workgroups).
template <typename K, bool PAY, int L, int R, bool WHOLE, bool PACK>
__global__ __launch_bounds__(L) __attribute__((amdgpu_waves_per_eu(4))) void merge_pipelined_kernel(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, int64_t nkeys,
    K* __restrict__ out, uint32_t* __restrict__ out_pay, int64_t nout,
    const PieceDesc* __restrict__ desc, int64_t P, const int64_t* __restrict__ P_dev, uint32_t cap) {
    merge_pipelined<K, PAY, L, R, WHOLE, PACK>(keys, pay, nkeys, out, out_pay, nout, desc, P, P_dev,
                                               cap);
}

template <typename K, bool PAY, int L, int R, bool WHOLE, bool PACK>
__global__ __launch_bounds__(L) void merge_pipelined_wide_kernel(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, int64_t nkeys,
    K* __restrict__ out, uint32_t* __restrict__ out_pay, int64_t nout,
    const PieceDesc* __restrict__ desc, int64_t P, const int64_t* __restrict__ P_dev, uint32_t cap) {
    merge_pipelined<K, PAY, L, R, WHOLE, PACK>(keys, pay, nkeys, out, out_pay, nout, desc, P, P_dev,
                                               cap);
}

// One workgroup per subproblem, staged straight into LDS; for subproblems
// larger than the register-pipelined kernel holds.
template <typename K, bool PAY, int L>
__global__ __launch_bounds__(L) void merge_direct_kernel(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, int64_t nkeys,
    K* __restrict__ out, uint32_t* __restrict__ out_pay, int64_t nout,
    const PieceDesc* __restrict__ desc, int64_t P, const int64_t* __restrict__ P_dev, uint32_t cap) {
    extern __shared__ __align__(16) char smem[];
    const SmemPtrs<K, PAY, L> sp(smem, cap);
    if (P_dev && (int64_t)blockIdx.x >= *P_dev) return;
    const PieceDesc d = desc[blockIdx.x];
    if (!desc_ok(d, nkeys, nout, cap) || piece_a(d) + piece_b(d) == 0) return;
    const SegPlan p = make_plan<K, PAY>(d);
    stage_direct<K, PAY, L>(p, keys, (uint64_t)nkeys, pay, sp.sKey, sp.sPay);
    __syncthreads();
    merge_lanes<K, PAY, L>(p, sp.sKey, sp.sPay, sp.sOut, sp.sIdx, sp.sXb, sp.sYb);
    write_back<K, PAY, L, 0>(p, sp.sOut, sp.sIdx, out, out_pay);
}

// LDS of merge_cases_direct_kernel: the key and payload windows and the
// lane-level ranks; the merged outputs go straight to memory.
template <typename K, bool PAY, int L>
struct DirectSmem {
    static __host__ __device__ uint32_t key_bytes(uint32_t cap) {
        return MergeSmem<K, PAY, L>::key_slots(cap) * (uint32_t)sizeof(K);
    }
    static __host__ __device__ uint32_t pay_bytes(uint32_t cap) {
        return PAY ? MergeSmem<K, PAY, L>::pay_slots(cap) * 4u : 0u;
    }
    static __host__ __device__ uint32_t bytes(uint32_t cap) {
        return (key_bytes(cap) + pay_bytes(cap) + 2u * (L + 1) * 4u + 15u) & ~15u;
    }
};

// Steps 3-4 and the merge of one subproblem per workgroup, for a few large
// subproblems: the workgroup takes its descriptor from the cross ranks itself
// (no descriptor pass), stages the subproblem with all of its 16-byte loads
// in flight at once (R chunks per thread), and runs L lanes, so that each
// lane's share stays short and the compute unit holds enough waves to cover
// the latency of its LDS reads.  The lanes write their merged pieces to
// memory themselves, which leaves LDS to the inputs: two such workgroups
// share a compute unit where one with output buffers would fit.
template <typename K, bool PAY, int L, int R>
__global__ __launch_bounds__(L) void merge_cases_direct_kernel(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, RcpBlocks BA, RcpBlocks BB,
    const int64_t* __restrict__ xbar, const int64_t* __restrict__ ybar, K* __restrict__ out,
    uint32_t* __restrict__ out_pay, uint32_t cap) {
    using S = DirectSmem<K, PAY, L>;
    extern __shared__ __align__(16) char smem[];
    K* sKey = reinterpret_cast<K*>(smem);
    uint32_t* sPay = reinterpret_cast<uint32_t*>(smem + S::key_bytes(cap));
    int* sXb = reinterpret_cast<int*>(smem + S::key_bytes(cap) + S::pay_bytes(cap));
    int* sYb = sXb + (L + 1);
    const int64_t nk = BA.len + BB.len;
    const PieceDesc d = case_desc(BA, BB, xbar, ybar, blockIdx.x);
    if (!desc_ok(d, nk, nk, cap) || piece_a(d) + piece_b(d) == 0) return;
    const SegPlan p = make_plan<K, PAY>(d);
    u32x4 rk[R], rp[R];
    prefetch<K, PAY, L, R>(p, keys, (uint64_t)nk, pay, rk, rp);
    wait_vm<0>();
    commit<K, PAY, L, R>(p, rk, rp, sKey, sPay);
    __syncthreads();
    merge_lanes_to_memory<K, PAY, L>(p, sKey, sPay, sXb, sYb, out, out_pay);
}

// ---------------------------------------------------------------------------
// Steps 3-4 for partitions into small blocks (subproblems of at most a few
// dozen elements), without descriptors.
//
// Workgroup g owns the A blocks [i0, i1) (kFineG of them) and every B block
// whose start y_j lies in [xbar_i0, xbar_i1).  The outputs of these pieces
// are exactly C[x_i0 + xbar_i0, x_i1 + xbar_i1) (workgroup 0 starts at 0):
// the elements placed there are A[x_i0, x_i1) and B[xbar_i0, xbar_i1), since
// A[x_i] lands at x_i + xbar_i.  So the workgroup stages both input ranges
// with 16-byte loads, merges each piece from LDS into an LDS copy of its
// output range, and writes that range with 16-byte stores.  A range too
// large for the staging buffers (many B elements between two A block
// starts) falls back to merging each piece straight from global memory.
// ---------------------------------------------------------------------------
constexpr int kFineG = 64;     // A blocks per workgroup
constexpr int kFineL = 128;    // threads per workgroup

// One piece merged straight from global memory with the stable two-pointer
// rule (B first only when strictly smaller).
template <typename K, bool PAY>
__device__ __forceinline__ void fine_piece_global(const K* __restrict__ keys,
                                                  const uint32_t* __restrict__ pay, int64_t n,
                                                  const Piece<int64_t>& pc, K* __restrict__ out,
                                                  uint32_t* __restrict__ out_pay) {
    const K* A = keys;
    const K* B = keys + n;
    int64_t ia = pc.a_lo, ib = pc.b_lo, o = pc.a_lo + pc.b_lo;
    while (ia < pc.a_hi && ib < pc.b_hi) {
        const K ka = A[ia], kb = B[ib];
        const bool tb = kb < ka;
        out[o] = tb ? kb : ka;
        if (PAY) out_pay[o] = tb ? pay[n + ib] : pay[ia];
        ib += tb;
        ia += !tb;
        ++o;
    }
    // the rest of one part is a copy: eight loads in flight before the
    // stores (under heavy duplicates most pieces here are copies of a B
    // block)
    auto copy = [&](const K* src, const uint32_t* psrc, int64_t i, int64_t end) {
        for (; i + 8 <= end; i += 8, o += 8) {
            K v[8];
            uint32_t q[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                v[e] = src[i + e];
                if (PAY) q[e] = psrc[i + e];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                out[o + e] = v[e];
                if (PAY) out_pay[o + e] = q[e];
            }
        }
        for (; i < end; ++i, ++o) {
            out[o] = src[i];
            if (PAY) out_pay[o] = psrc[i];
        }
    };
    copy(A, pay, ia, pc.a_hi);
    copy(B, PAY ? pay + n : nullptr, ib, pc.b_hi);
}

// LDS of the staged small-block merge: A window, B window, output window
// (keys; payloads alike), each with a 16-byte alignment margin.
struct FineSmem {
    int ka, kb, kc;   // slots per window
    __host__ __device__ FineSmem(int capA, int capB) {
        ka = (capA + 16 + 7) & ~7;
        kb = (capB + 16 + 7) & ~7;
        kc = (capA + capB + 16 + 7) & ~7;
    }
    // esz = bytes per element: key size, plus 4 with payloads
    __host__ __device__ uint32_t bytes_for(int esz) const {
        return (uint32_t)(ka + kb + kc) * (uint32_t)esz;
    }
};

// The A and B input ranges of a small-block workgroup (keys[a_lo, a_lo +
// na) and keys[b0, b0 + nb), payloads alike) into LDS in 16-byte chunks
// (src 16-byte aligned at index 0): element lo + k of a range lands at
// dst[lo % V + k].  fine_load issues up to R chunks per thread of an array,
// so that every array of the workgroup is in flight before the first LDS
// store and staging costs one round trip to memory; fine_store writes them
// and moves chunks past R per thread one by one.
template <typename E, int L, int R>
__device__ __forceinline__ void fine_load(const E* src, uint64_t src_len, int64_t a_lo, int na,
                                          int64_t b0, int nb, u32x4 (&r)[R], int& nA, int& nB) {
    constexpr int V = 16 / sizeof(E);
    const int offA = (int)(a_lo % V), offB = (int)(b0 % V);
    nA = (offA + na + V - 1) / V;
    nB = (offB + nb + V - 1) / V;
    load_windows<L, R>(reinterpret_cast<const char*>(src), src_len * sizeof(E),
                       (a_lo - offA) * (int64_t)sizeof(E), nA, (b0 - offB) * (int64_t)sizeof(E), nB,
                       r);
}

template <typename E, int L, int R>
__device__ __forceinline__ void fine_store(const E* src, uint64_t src_len, int64_t a_lo, int64_t b0,
                                           const u32x4 (&r)[R], int nA, int nB, E* dA, E* dB) {
    constexpr int V = 16 / sizeof(E);
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int q = i * L + t;
        if (q < nA) *reinterpret_cast<u32x4*>(dA + q * V) = r[i];
        else if (q < nA + nB) *reinterpret_cast<u32x4*>(dB + (q - nA) * V) = r[i];
    }
    if (nA + nB > R * L) {
        const int64_t alA = a_lo - (int)(a_lo % V), alB = b0 - (int)(b0 % V);
        const __amdgpu_buffer_rsrc_t rA = make_rsrc(src + alA, (src_len - (uint64_t)alA) * sizeof(E));
        const __amdgpu_buffer_rsrc_t rB = make_rsrc(src + alB, (src_len - (uint64_t)alB) * sizeof(E));
        for (int q = R * L + t; q < nA + nB; q += L) {
            if (q < nA) *reinterpret_cast<u32x4*>(dA + q * V) = buf_load16(rA, (uint32_t)q * 16u);
            else *reinterpret_cast<u32x4*>(dB + (q - nA) * V) = buf_load16(rB, (uint32_t)(q - nA) * 16u);
        }
    }
}

// 16-byte chunks per thread of each array that fine_merge_staged_kernel keeps
// in flight while staging.
constexpr int kFineChunks = 8;

template <typename K, bool PAY>
__global__ __launch_bounds__(kFineL) void fine_merge_staged_kernel(
    const K* __restrict__ keys, const uint32_t* __restrict__ pay, RcpBlocks BA, RcpBlocks BB,
    const int64_t* __restrict__ xbar, const int64_t* __restrict__ ybar, K* __restrict__ out,
    uint32_t* __restrict__ out_pay, int capA, int capB) {
    constexpr int L = kFineL;
    extern __shared__ __align__(16) char smem[];
    const FineSmem fs(capA, capB);
    K* sA = reinterpret_cast<K*>(smem);
    K* sB = sA + fs.ka;
    K* sC = sB + fs.kb;
    uint32_t* qA = reinterpret_cast<uint32_t*>(sC + fs.kc);
    uint32_t* qB = qA + fs.ka;
    uint32_t* qC = qB + fs.kb;

    const int64_t n = BA.len, m = BB.len, p_a = BA.p, p_b = BB.p;
    const int64_t i0 = (int64_t)blockIdx.x * kFineG;
    if (i0 >= p_a) return;
    const int64_t i1 = i0 + kFineG < p_a ? i0 + kFineG : p_a;
    const int64_t a_lo = BA.start(i0), a_hi = BA.start(i1);
    const int64_t b_lo = blockIdx.x == 0 ? 0 : xbar[i0];
    const int64_t b_hi = xbar[i1];
    const int64_t c_lo = a_lo + b_lo;
    // B blocks whose start lies in [b_lo, b_hi)
    auto first_start_at_or_after = [&](int64_t pos) {
        int64_t j = BB.of(pos);
        if (j < p_b && BB.start(j) < pos) ++j;
        return j;
    };
    const int64_t j0 = first_start_at_or_after(b_lo), j1 = first_start_at_or_after(b_hi);
    const int64_t na = a_hi - a_lo, nb = b_hi - b_lo;
    const int64_t npa = i1 - i0, npieces = npa + (j1 - j0);
    if (!(0 <= b_lo && b_lo <= b_hi && b_hi <= m && j0 <= j1)) return;  // cannot happen

    auto piece = [&](int64_t idx) {
        return idx < npa ? step3_piece<int64_t>(BA, BB, xbar, ybar, i0 + idx)
                         : step4_piece<int64_t>(BA, BB, xbar, ybar, j0 + (idx - npa));
    };
    auto inside = [&](const Piece<int64_t>& pc) {
        return a_lo <= pc.a_lo && pc.a_lo <= pc.a_hi && pc.a_hi <= a_hi && b_lo <= pc.b_lo &&
               pc.b_lo <= pc.b_hi && pc.b_hi <= b_hi;
    };

    if (na > capA || nb > capB) {
        // too many elements to stage: each piece from global memory
        for (int64_t idx = threadIdx.x; idx < npieces; idx += L) {
            const Piece<int64_t> pc = piece(idx);
            if (inside(pc)) fine_piece_global<K, PAY>(keys, pay, n, pc, out, out_pay);
        }
        return;
    }

    // this thread's first piece: its cross-rank reads go out before the
    // staging loads
    const bool has0 = threadIdx.x < npieces;
    Piece<int64_t> pc0;
    pc0.a_lo = pc0.a_hi = a_lo;
    pc0.b_lo = pc0.b_hi = b_lo;
    pc0.c_off = c_lo;
    if (has0) pc0 = piece(threadIdx.x);

    const uint64_t total = (uint64_t)(n + m);
    constexpr int RC = kFineChunks;
    u32x4 rk[RC], rp[RC];
    int nkA, nkB, npA = 0, npB = 0;
    fine_load<K, L, RC>(keys, total, a_lo, (int)na, n + b_lo, (int)nb, rk, nkA, nkB);
    if (PAY) fine_load<uint32_t, L, RC>(pay, total, a_lo, (int)na, n + b_lo, (int)nb, rp, npA, npB);
    fine_store<K, L, RC>(keys, total, a_lo, n + b_lo, rk, nkA, nkB, sA, sB);
    if (PAY) fine_store<uint32_t, L, RC>(pay, total, a_lo, n + b_lo, rp, npA, npB, qA, qB);
    constexpr int V = 16 / sizeof(K);
    const int offA = (int)(a_lo % V), offB = (int)((n + b_lo) % V);
    const int offC = (int)(c_lo % V);
    const int offCP = (int)(c_lo % 4);
    const int offPA = (int)(a_lo % 4), offPB = (int)((n + b_lo) % 4);
    __syncthreads();

    for (int64_t idx = threadIdx.x; idx < npieces; idx += L) {
        const Piece<int64_t> pc = idx == threadIdx.x ? pc0 : piece(idx);
        if (!inside(pc)) continue;  // cannot happen for cross ranks of sorted inputs
        const int la = (int)(pc.a_hi - pc.a_lo), lb = (int)(pc.b_hi - pc.b_lo);
        const int ia = offA + (int)(pc.a_lo - a_lo), ib = offB + (int)(pc.b_lo - b_lo);
        const int oc = (int)(pc.c_off - c_lo);
        if (!PAY && la <= 16 && lb <= 16) {
            // both parts into registers (past a part: the key type's maximum),
            // Batcher's odd-even merge, the first la + lb back to LDS; without
            // payloads the order among equal keys is not observable
            K v[32];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                v[i] = i < la ? sA[ia + i] : KeyMax<K>::v;
                v[16 + i] = i < lb ? sB[ib + i] : KeyMax<K>::v;
            }
            OddEvenMerge<0, 31, 1>::template run<K>(v);
#pragma unroll
            for (int k = 0; k < 32; ++k)
                if (k < la + lb) sC[offC + oc + k] = v[k];
        } else {
            // stable two-pointer merge in LDS
            const int pa0 = offPA + (int)(pc.a_lo - a_lo), pb0 = offPB + (int)(pc.b_lo - b_lo);
            int x = 0, y = 0, k = offC + oc, kp = offCP + oc;
            while (x < la && y < lb) {
                const K ka = sA[ia + x], kb = sB[ib + y];
                const bool tb = kb < ka;
                sC[k++] = tb ? kb : ka;
                if (PAY) qC[kp++] = tb ? qB[pb0 + y] : qA[pa0 + x];
                y += tb;
                x += !tb;
            }
            for (; x < la; ++x) {
                sC[k++] = sA[ia + x];
                if (PAY) qC[kp++] = qA[pa0 + x];
            }
            for (; y < lb; ++y) {
                sC[k++] = sB[ib + y];
                if (PAY) qC[kp++] = qB[pb0 + y];
            }
        }
    }
    __syncthreads();
    const int s = (int)(na + nb);
    write_out<K, L, 0>(sC, offC, s, out + (c_lo - offC));
    if (PAY) write_out<uint32_t, L, 0>(qC, offCP, s, out_pay + (c_lo - offCP));
}

template <typename K>
__global__ __launch_bounds__(256) void validate_kernel(const K* __restrict__ keys, int64_t n,
                                                       int64_t m, int* flag) {
    const int64_t total = n + m;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k + 1 < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (k + 1 == n) continue;  // boundary between A and B
        if (keys[k + 1] < keys[k]) *flag = 1;
    }
}

// ---------------------------------------------------------------------------


uint32_t merge_lds_bytes(int dtype, bool pay, uint32_t cap) {
    uint32_t r = 0;
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        r = pay ? MergeSmem<K, true, kMergeThreads>::bytes(cap)
                : MergeSmem<K, false, kMergeThreads>::bytes(cap);
    });
    return r;
}

hipError_t launch_partition(int dtype, const void* keys, int64_t n, int64_t m, int64_t p_a,
                            int64_t p_b, int64_t* xbar, int64_t* ybar, hipStream_t st) {
    const int64_t searches = p_a + p_b + 2;
    // few searches: their rounds of dependent loads set the time, and a
    // group of lanes per search takes fewer rounds (for more loads)
    const bool group = searches <= kGroupSearchMax;
    const int64_t threads = group ? searches * kSearchGroup : searches;
    const unsigned grid = (unsigned)((threads + 255) / 256);
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        if (group)
            partition_group_kernel<K, kSearchGroup><<<grid, 256, 0, st>>>(
                static_cast<const K*>(keys), n, m, p_a, p_b, xbar, ybar);
        else
            partition_kernel<K><<<grid, 256, 0, st>>>(static_cast<const K*>(keys), n, m, p_a, p_b,
                                                      xbar, ybar);
    });
    return hipGetLastError();
}

int device_cu_count() {
    static std::atomic<int> cached{0};
    int cus = cached.load(std::memory_order_relaxed);
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached.store(cus, std::memory_order_relaxed);
    }
    return cus;
}

template <typename Kern>
static hipError_t allow_big_lds(Kern kern) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds);
}

// allow_big_lds once per kernel: `done` is that kernel's own flag (setting
// the attribute twice, from two threads racing on the first call, is
// harmless)
template <typename Kern>
static hipError_t allow_big_lds_once(Kern kern, std::atomic<bool>& done) {
    if (done.load(std::memory_order_acquire)) return hipSuccess;
    const hipError_t e = allow_big_lds(kern);
    if (e == hipSuccess) done.store(true, std::memory_order_release);
    return e;
}

// Workgroups of a persistent merge kernel that fit one compute unit at once.
// LDS is handed out in granules of kLdsGranule bytes (measured: workgroups
// with X bytes co-reside k to a CU exactly while k * ceil(X / 1280) <= 128),
// which the runtime's occupancy calculator does not apply; it still bounds
// the count by registers and waves.  A grid sized past the true count runs
// the surplus workgroups as a second, serial wave: each takes a fixed share
// of the subproblems, so that doubles the time.  Each kernel caches the
// answer for the last LDS size.
template <typename Kern>
static int resident_per_cu(Kern kern, uint32_t lds, std::atomic<uint64_t>& last) {
    const uint64_t c = last.load(std::memory_order_relaxed);
    if (c != 0 && (uint32_t)(c >> 32) == lds) return (int)(uint32_t)c;
    const uint32_t granted = (lds + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
    int n = (int)(kMaxLds / (granted > 0 ? granted : kLdsGranule));
    int by_regs = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&by_regs, kern, kMergeThreads, lds) ==
            hipSuccess &&
        by_regs >= 1) {
        if (by_regs < n) n = by_regs;
    } else {
        (void)hipGetLastError();
    }
    if (n > 8) n = 8;
    if (n < 1) n = 1;
    last.store(((uint64_t)lds << 32) | (uint32_t)n, std::memory_order_relaxed);
    return n;
}

// Largest subproblem the register-pipelined kernel with R chunks per thread
// can stage: key chunks <= cap / V + 4 and payload chunks <= cap / 4 + 4 must
// not exceed R * L.
template <typename K, bool PAY, int L = kMergeThreads>
static bool fits_regs(uint32_t cap, int R) {
    constexpr int V = Vec<K>::N;
    const int64_t slots = (int64_t)R * L;
    if ((int64_t)cap / V + 5 > slots) return false;
    if (PAY && (int64_t)cap / 4 + 4 > slots) return false;
    return true;
}

template <typename K, bool PAY, int R>
static hipError_t launch_persistent(const K* keys, const uint32_t* pay, int64_t nkeys, K* out,
                                    uint32_t* out_pay, int64_t nout, const PieceDesc* desc,
                                    int64_t P, const int64_t* P_dev, uint32_t cap, bool packed,
                                    hipStream_t st) {
    constexpr int L = kMergeThreads;
    // two register sets in flight where they fit the register budget; one
    // buffer resource spans each array below 4 GiB, larger arrays take one
    // per window
    const bool whole = (uint64_t)nkeys * sizeof(K) < (1ull << 32) - 4096 &&
                       (uint64_t)nout * sizeof(K) < (1ull << 32) - 4096;
    if constexpr (R <= 5) {
        auto go = [&](auto kern, std::atomic<bool>& attr2,
                      std::atomic<uint64_t>& occ) -> hipError_t {
            const hipError_t e = allow_big_lds_once(kern, attr2);
            if (e != hipSuccess) return e;
            const uint32_t lds = MergeSmem<K, PAY, L>::bytes(cap);
            int64_t grid = (int64_t)device_cu_count() * resident_per_cu(kern, lds, occ);
            if (grid > P) grid = P;
            kern<<<(unsigned)grid, L, lds, st>>>(keys, pay, nkeys, out, out_pay, nout, desc, P,
                                                 P_dev, cap);
            return hipGetLastError();
        };
        static std::atomic<bool> attr2{false}, attr3{false}, attr4{false}, attr5{false};
        static std::atomic<uint64_t> occ2{0}, occ3{0}, occ4{0}, occ5{0};
        if constexpr (sizeof(K) == 8 && PAY) {
            if (whole) return go(merge_pipelined_wide_kernel<K, PAY, L, R, true, false>, attr2, occ2);
        } else if constexpr (PAY && R > 3) {
            if (whole) return go(merge_pipelined_kernel<K, PAY, L, R, true, false>, attr2, occ2);
        } else if constexpr (PAY) {
            if (whole)
                return packed ? go(merge_pipelined_kernel<K, PAY, L, R, true, true>, attr4, occ4)
                              : go(merge_pipelined_kernel<K, PAY, L, R, true, false>, attr2, occ2);
        } else {
            if (packed)
                return whole ? go(merge_pipelined_kernel<K, PAY, L, R, true, true>, attr4, occ4)
                             : go(merge_pipelined_kernel<K, PAY, L, R, false, true>, attr5, occ5);
            return whole ? go(merge_pipelined_kernel<K, PAY, L, R, true, false>, attr2, occ2)
                         : go(merge_pipelined_kernel<K, PAY, L, R, false, false>, attr3, occ3);
        }
    }
    auto kern = merge_persistent_kernel<K, PAY, L, R>;
    static std::atomic<bool> attr{false};
    {
        const hipError_t e = allow_big_lds_once(kern, attr);
        if (e != hipSuccess) return e;
    }
    const uint32_t lds = MergeSmem<K, PAY, L>::bytes(cap);
    static std::atomic<uint64_t> occ{0};
    int64_t grid = (int64_t)device_cu_count() * resident_per_cu(kern, lds, occ);
    if (grid > P) grid = P;
    kern<<<(unsigned)grid, L, lds, st>>>(keys, pay, nkeys, out, out_pay, nout, desc, P, P_dev, cap);
    return hipGetLastError();
}

template <typename K, bool PAY>
static hipError_t launch_merge_t(const void* keys_v, const uint32_t* pay, int64_t nkeys,
                                 void* out_v, uint32_t* out_pay, int64_t nout,
                                 const PieceDesc* desc, int64_t P, const int64_t* P_dev, uint32_t cap,
                                 bool packed, hipStream_t st) {
    const K* keys = static_cast<const K*>(keys_v);
    K* out = static_cast<K*>(out_v);
    if (P <= 0) return hipSuccess;
    // 32-bit keys with payloads at the default block lengths need only three
    // chunks per thread: the freed registers pay for the lean lane level
    if constexpr (PAY && sizeof(K) == 4) {
        if (fits_regs<K, PAY>(cap, 3))
            return launch_persistent<K, PAY, 3>(keys, pay, nkeys, out, out_pay, nout, desc, P, P_dev,
                                                cap, packed, st);
    }
    if (fits_regs<K, PAY>(cap, 5))
        return launch_persistent<K, PAY, 5>(keys, pay, nkeys, out, out_pay, nout, desc, P, P_dev, cap,
                                            packed, st);
    if (fits_regs<K, PAY>(cap, 9))
        return launch_persistent<K, PAY, 9>(keys, pay, nkeys, out, out_pay, nout, desc, P, P_dev, cap,
                                            false, st);
    constexpr int L = kMergeThreads;
    auto kern = merge_direct_kernel<K, PAY, L>;
    static std::atomic<bool> attr{false};
    {
        const hipError_t e = allow_big_lds_once(kern, attr);
        if (e != hipSuccess) return e;
    }
    const uint32_t lds = MergeSmem<K, PAY, L>::bytes(cap);
    kern<<<(unsigned)P, L, lds, st>>>(keys, pay, nkeys, out, out_pay, nout, desc, P, P_dev, cap);
    return hipGetLastError();
}

uint32_t merge_cap_for_tile(int32_t tile) { return 2u * (uint32_t)tile; }

// Register slots the pipelined merge uses for a capacity (as launch_merge_t
// picks them); 0 for the unpipelined forms.
template <typename K, bool PAY>
static int merge_regs(uint32_t cap) {
    if (PAY && sizeof(K) == 4 && fits_regs<K, PAY>(cap, 3)) return 3;
    if (fits_regs<K, PAY>(cap, 5)) return 5;
    return fits_regs<K, PAY>(cap, 9) ? 9 : 0;
}

uint32_t merge_pack_cap(int dtype, bool pay, uint32_t cap) {
    uint32_t best = cap;
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        auto regs = [&](uint32_t c) { return pay ? merge_regs<K, true>(c) : merge_regs<K, false>(c); };
        auto lds = [&](uint32_t c) {
            return pay ? MergeSmem<K, true, kMergeThreads>::bytes(c)
                       : MergeSmem<K, false, kMergeThreads>::bytes(c);
        };
        auto granules = [&](uint32_t c) { return (lds(c) + kLdsGranule - 1) / kLdsGranule; };
        const int r0 = regs(cap);
        const uint32_t g0 = granules(cap);
        if (r0 == 0 || r0 == 9) return;
        for (uint32_t c = cap + 8; c <= 2 * cap && regs(c) == r0 && granules(c) == g0; c += 8)
            best = c;
    });
    return best;
}

// Register chunks per thread for merge_cases_direct_kernel (0: none fits).
template <typename K, bool PAY>
static int direct_regs(uint32_t cap) {
    if (fits_regs<K, PAY, kWideMergeThreads>(cap, 2)) return 2;
    return fits_regs<K, PAY, kWideMergeThreads>(cap, 5) ? 5 : 0;
}

bool merge_cases_direct_applies(int dtype, bool pay, uint32_t cap, int64_t P) {
    if (P <= 0 || P > (int64_t)kWideMergeMaxWgPerCu * device_cu_count()) return false;
    bool ok = false;
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        // subproblems past the register-pipelined kernels' reach (one
        // 256-lane workgroup per compute unit there), or fewer subproblems
        // than compute units
        const int r = pay ? merge_regs<K, true>(cap) : merge_regs<K, false>(cap);
        const bool big = r >= 9 || r == 0;
        const bool regs = (pay ? direct_regs<K, true>(cap) : direct_regs<K, false>(cap)) > 0;
        const uint32_t lds = pay ? DirectSmem<K, true, kWideMergeThreads>::bytes(cap)
                                 : DirectSmem<K, false, kWideMergeThreads>::bytes(cap);
        ok = (big || P <= device_cu_count()) && regs && lds <= kMaxLds;
    });
    return ok;
}

hipError_t launch_merge_cases_direct(int dtype, const void* keys, const uint32_t* pay, int64_t n,
                                     int64_t m, int64_t p_a, int64_t p_b, const int64_t* xbar,
                                     const int64_t* ybar, void* out_keys, uint32_t* out_pay,
                                     uint32_t cap, hipStream_t st) {
    const int64_t P = p_a + p_b;
    if (P <= 0) return hipSuccess;
    constexpr int L = kWideMergeThreads;
    hipError_t e = hipErrorInvalidValue;   // no register layout holds cap
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        auto go = [&](auto kern, std::atomic<bool>& attr, uint32_t lds) {
            e = allow_big_lds_once(kern, attr);
            if (e != hipSuccess) return;
            kern<<<(unsigned)P, L, lds, st>>>(static_cast<const K*>(keys), pay, RcpBlocks(n, p_a),
                                              RcpBlocks(m, p_b), xbar, ybar,
                                              static_cast<K*>(out_keys), out_pay, cap);
            e = hipGetLastError();
        };
        if (pay) {
            const uint32_t lds = DirectSmem<K, true, L>::bytes(cap);
            const int r = direct_regs<K, true>(cap);
            static std::atomic<bool> attr2{false}, attr5{false};
            if (r == 2) go(merge_cases_direct_kernel<K, true, L, 2>, attr2, lds);
            else if (r == 5) go(merge_cases_direct_kernel<K, true, L, 5>, attr5, lds);
        } else {
            const uint32_t lds = DirectSmem<K, false, L>::bytes(cap);
            const int r = direct_regs<K, false>(cap);
            static std::atomic<bool> attr2{false}, attr5{false};
            if (r == 2) go(merge_cases_direct_kernel<K, false, L, 2>, attr2, lds);
            else if (r == 5) go(merge_cases_direct_kernel<K, false, L, 5>, attr5, lds);
        }
    });
    return e;
}

hipError_t launch_cases(int64_t n, int64_t m, int64_t p_a, int64_t p_b, const int64_t* xbar,
                        const int64_t* ybar, PieceDesc* desc, hipStream_t st) {
    const int64_t P = p_a + p_b;
    cases_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(RcpBlocks(n, p_a), RcpBlocks(m, p_b),
                                                              xbar, ybar, desc);
    return hipGetLastError();
}

hipError_t launch_merge_desc(int dtype, const void* keys, const uint32_t* pay, int64_t nkeys,
                             void* out_keys, uint32_t* out_pay, int64_t nout,
                             const PieceDesc* desc, int64_t P, const int64_t* P_dev, uint32_t cap,
                             hipStream_t st, bool packed) {
    hipError_t e = hipSuccess;
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        e = pay ? launch_merge_t<K, true>(keys, pay, nkeys, out_keys, out_pay, nout, desc, P, P_dev,
                                          cap, packed, st)
                : launch_merge_t<K, false>(keys, nullptr, nkeys, out_keys, nullptr, nout, desc, P,
                                           P_dev, cap, packed, st);
    });
    return e;
}

hipError_t launch_fine_merge(int dtype, const void* keys, const uint32_t* pay, int64_t n,
                            int64_t m, int64_t p_a, int64_t p_b, const int64_t* xbar,
                            const int64_t* ybar, void* out_keys, uint32_t* out_pay,
                            hipStream_t st) {
    if (p_a + p_b <= 0 || n + m <= 0) return hipSuccess;
    if (dtype & kDescending) return hipErrorInvalidValue;  // ascending order only
    const unsigned grid = (unsigned)((p_a + kFineG - 1) / kFineG);
    // staging capacity: the workgroup's A blocks in full, and twice that (at
    // least 2048) of B, within 64 KiB of LDS (B shrinks first; if A alone
    // does not fit, nothing is staged); a workgroup whose ranges exceed the
    // capacity merges from global memory
    const int64_t la_max = (n + p_a - 1) / p_a;
    const int ksz = (int)dtype_bytes(dtype);
    const int esz = ksz + (pay ? 4 : 0);
    int capA = (int)(kFineG * (la_max > 0 ? la_max : 1));
    int capB = 2 * capA > 2048 ? 2 * capA : 2048;
    constexpr uint32_t kFineLds = 64 * 1024;
    while (capB > capA && FineSmem(capA, capB).bytes_for(esz) > kFineLds) capB /= 2;
    if (FineSmem(capA, capB).bytes_for(esz) > kFineLds) capA = capB = 0;
    const FineSmem fs(capA, capB);
    hipError_t e = hipSuccess;
    with_key_type_asc(dtype, [&](auto z) {
        using K = decltype(z);
        const uint32_t lds = fs.bytes_for(esz);
        if (pay) {
            auto kern = fine_merge_staged_kernel<K, true>;
            static std::atomic<bool> attr{false};
            e = allow_big_lds_once(kern, attr);
            if (e == hipSuccess)
                kern<<<grid, kFineL, lds, st>>>(static_cast<const K*>(keys), pay, RcpBlocks(n, p_a),
                                                RcpBlocks(m, p_b), xbar, ybar,
                                                static_cast<K*>(out_keys), out_pay, capA, capB);
        } else {
            auto kern = fine_merge_staged_kernel<K, false>;
            static std::atomic<bool> attr{false};
            e = allow_big_lds_once(kern, attr);
            if (e == hipSuccess)
                kern<<<grid, kFineL, lds, st>>>(static_cast<const K*>(keys), nullptr,
                                                RcpBlocks(n, p_a), RcpBlocks(m, p_b), xbar, ybar,
                                                static_cast<K*>(out_keys), nullptr, capA, capB);
        }
    });
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_validate(int dtype, const void* keys, int64_t n, int64_t m, int* flag,
                           hipStream_t st) {
    const int64_t total = n + m;
    int64_t g = (total + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    with_key_type(dtype, [&](auto z) {
        using K = decltype(z);
        validate_kernel<K><<<(unsigned)g, 256, 0, st>>>(static_cast<const K*>(keys), n, m, flag);
    });
    return hipGetLastError();
}

}  // namespace sm
