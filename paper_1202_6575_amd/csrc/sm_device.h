// sm_device.h -- device-side building blocks of the stable merge (gfx950).
//
// Block decomposition and membership (Section 2), binary-search ranks
// rank_low / rank_high (Section 2 definitions), the two-select form of the
// five cases of Steps 3-4, and the per-workgroup merge of one subproblem:
// LDS staging with 128-bit loads, the same method again at lane level, a
// per-lane stable sequential merge, and a coalesced write-back through LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sm_keys.h"

namespace sm {

// ---------------------------------------------------------------------------
// Block decomposition (Section 2): the first r = len mod p blocks hold
// ceil(len/p) elements, the others floor(len/p).  start(i) = x_i with
// x_p = len; of(k) is the block holding index k, with of(k) = p for k >= len
// (the position of the +inf sentinel).
// ---------------------------------------------------------------------------
template <typename I>
struct Blocks {
    I len, p, q, r, c, rc;
    __device__ __host__ Blocks(I len_, I p_) : len(len_), p(p_) {
        q = len / p;
        r = len - q * p;
        c = q + (r != 0);
        rc = r * c;
    }
    __device__ __host__ I start(I i) const {
        if (i >= p) return len;
        return i < r ? i * c : i * q + r;
    }
    __device__ __host__ I of(I k) const {
        if (k >= len) return p;
        return k < rc ? k / c : (k - rc) / q + r;
    }
};

// The same decomposition with the divisions done as products with
// double-precision reciprocals (exact after one correction step for
// positions below 2^50): 64-bit integer division is a long instruction
// sequence on this hardware, and kernels that place hundreds of thousands
// of blocks would spend their time there.  Built on the host (and passed
// to a kernel) or in a kernel (one per job of a batch); both give the same
// values.
struct RcpBlocks {
    int64_t len, p, q, r, c, rc;
    double rcp_c, rcp_q;
    __host__ __device__ RcpBlocks(int64_t len_, int64_t p_) : len(len_), p(p_) {
        q = p > 0 ? div(len, p, 1.0 / (double)p) : 0;
        r = len - q * p;
        c = q + (r != 0);
        rc = r * c;
        rcp_c = c > 0 ? 1.0 / (double)c : 0.0;
        rcp_q = q > 0 ? 1.0 / (double)q : 0.0;
    }
    __device__ int64_t start(int64_t i) const {
        if (i >= p) return len;
        return i < r ? i * c : i * q + r;
    }
    // k / d for 0 <= k < 2^50, d >= 1, rd = 1 / d
    __host__ __device__ static int64_t div(int64_t k, int64_t d, double rd) {
        int64_t x = (int64_t)((double)k * rd);
        const int64_t rem = k - x * d;
        x += (rem >= d) - (rem < 0);
        return x;
    }
    __device__ int64_t of(int64_t k) const {
        if (k >= len) return p;
        return k < rc ? div(k, c, rcp_c) : div(k - rc, q, rcp_q) + r;
    }
};

// Quotient k / d for 0 <= k < 2^22 and a workgroup-uniform divisor d >= 1
// with rd ~ 1 / d (hardware reciprocal, within an ulp): the float product is
// within one of the quotient, and one exact correction step fixes it.
__device__ __forceinline__ int fast_div(int k, int d, float rd) {
    int q = (int)((float)k * rd);
    const int r = k - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

// The same decomposition for the lane level: p = L blocks (a power of two),
// lengths below 2^22, divisions by the uniform block sizes via fast_div.
// SEL picks select-based arithmetic (fewer instructions) over branches
// (fewer registers live: the payload kernels sit at their register limit).
template <int L, bool SEL = true>
struct LaneBlocks {
    int len, q, r, c, rc;
    float rcp_c, rcp_q;
    static constexpr int p = L;
    __device__ LaneBlocks(int len_) : len(len_) {
        q = len / L;
        r = len - q * L;
        c = q + (r != 0);
        rc = r * c;
        rcp_c = c > 0 ? __builtin_amdgcn_rcpf((float)c) : 0.0f;
        rcp_q = q > 0 ? __builtin_amdgcn_rcpf((float)q) : 0.0f;
    }
    // both written with selects, not branches: lanes of a wave disagree on
    // which side of r they are, and a divergent branch would run both sides
    // anyway.  start(i) = i*q + min(i, r) is at most len for i <= L.
    __device__ int start(int i) const {
        if constexpr (SEL) {
            const int s = i * q + (i < r ? i : r);
            return s < len ? s : len;
        } else {
            if (i >= L) return len;
            return i < r ? i * c : i * q + r;
        }
    }
    // one quotient, with divisor and offset picked per lane: k / c below
    // rc, (k - rc) / q + r from there on (q = 0 only when every k < len is
    // below rc; for k >= len the quotient is discarded)
    __device__ int of(int k) const {
        if constexpr (SEL) {
            const bool lng = k < rc;
            const int blk =
                fast_div(lng ? k : k - rc, lng ? c : q, lng ? rcp_c : rcp_q) + (lng ? 0 : r);
            return k >= len ? L : blk;
        } else {
            if (k >= len) return L;
            return k < rc ? fast_div(k, c, rcp_c) : fast_div(k - rc, q, rcp_q) + r;
        }
    }
};

// ---------------------------------------------------------------------------
// Ranks by binary search (Section 2): rank_low(x, X) = #{X[t] < x},
// rank_high(x, X) = #{X[t] <= x}, over X[0, len).
// ---------------------------------------------------------------------------
template <typename K, typename I>
__device__ __forceinline__ I rank_low(const K* X, I len, K x) {
    I lo = 0, n = len;
    while (n > 0) {
        I half = n >> 1;
        if (X[lo + half] < x) { lo += half + 1; n -= half + 1; }
        else n = half;
    }
    return lo;
}

template <typename K, typename I>
__device__ __forceinline__ I rank_high(const K* X, I len, K x) {
    I lo = 0, n = len;
    while (n > 0) {
        I half = n >> 1;
        if (!(x < X[lo + half])) { lo += half + 1; n -= half + 1; }
        else n = half;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Steps 3-4 in two-select form.  For the processing element of A block i:
// outside case (e) (xbar_i != xbar_{i+1} and xbar_i = y_j) the B range ends
// at min(xbar_{i+1}, y_{j+1}) and the A range at ybar_{j+1} if
// xbar_{i+1} > y_{j+1}, else at x_{i+1}; this covers cases (a)-(d).
// Case (e) takes A[x_i, ybar_j) alone.  B blocks mirror it with A and B,
// rank_low and rank_high exchanged; the tie rule stays A before B.
// The ybar / xbar arrays have p + 1 entries; indices are clamped so that a
// block whose cross rank is the sentinel (j = p) never reads past them.
// ---------------------------------------------------------------------------
template <typename I>
struct Piece {
    I a_lo, a_hi, b_lo, b_hi, c_off;
};

template <typename I, typename BK, typename R>
__device__ __forceinline__ Piece<I> step3_piece(const BK& BA, const BK& BB, const R* xbar,
                                                const R* ybar, I i) {
    Piece<I> s;
    const I pb = (I)BB.p;
    const I xi = BA.start(i), xi1 = BA.start(i + 1);
    const I xb = (I)xbar[i], xb1 = (I)xbar[i + 1];
    const I j = BB.of(xb);
    const I yj = BB.start(j), yj1 = BB.start(j + 1);
    const I j1 = j + 1 < pb ? j + 1 : pb;
    s.a_lo = xi;
    s.b_lo = xb;
    s.c_off = xi + xb;
    if (xb != xb1 && xb == yj) {
        s.a_hi = (I)ybar[j < pb ? j : pb];
        s.b_hi = xb;
    } else {
        s.b_hi = xb1 < yj1 ? xb1 : yj1;
        s.a_hi = xb1 > yj1 ? (I)ybar[j1] : xi1;
    }
    return s;
}

template <typename I, typename BK, typename R>
__device__ __forceinline__ Piece<I> step4_piece(const BK& BA, const BK& BB, const R* xbar,
                                                const R* ybar, I j) {
    Piece<I> s;
    const I pa = (I)BA.p;
    const I yj = BB.start(j), yj1 = BB.start(j + 1);
    const I yb = (I)ybar[j], yb1 = (I)ybar[j + 1];
    const I i = BA.of(yb);
    const I xi = BA.start(i), xi1 = BA.start(i + 1);
    const I i1 = i + 1 < pa ? i + 1 : pa;
    s.b_lo = yj;
    s.a_lo = yb;
    s.c_off = yj + yb;
    if (yb != yb1 && yb == xi) {
        s.b_hi = (I)xbar[i < pa ? i : pa];
        s.a_hi = yb;
    } else {
        s.a_hi = yb1 < xi1 ? yb1 : xi1;
        s.b_hi = yb1 > xi1 ? (I)xbar[i1] : yj1;
    }
    return s;
}

// ---------------------------------------------------------------------------
// Raw buffer access.  A buffer resource bounds every load to the valid bytes,
// so the aligned 16-byte chunks that cover a segment never read past the
// caller's array: out-of-range lanes read zero and are never used.
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The base and size are workgroup-uniform; readfirstlane states that, so the
// resource lives in scalar registers (no per-lane waterfall around loads).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint64_t bytes) {
    const uint32_t nrec = bytes > 0xFFFFFFF0ull ? 0xFFFFFFF0u : (uint32_t)bytes;
    const uint64_t b = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    void* ub = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(ub, (short)0, (int)__builtin_amdgcn_readfirstlane(nrec),
                                             0x00020000);
}

// Non-temporal (cache policy bit 1, "nt" on gfx950): every caller streams
// data it reads once (staging windows, descriptors), and keeping those lines
// out of the caches' reuse order leaves room for what is read again, such
// as the upper levels of the cross-rank searches.
__device__ __forceinline__ u32x4 buf_load16(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 2);
}

// ---------------------------------------------------------------------------
// A subproblem in absolute element positions of the caller's arrays: merge
// keys[ka0, ka0 + a) (from A) with keys[kb0, kb0 + b) (from B) into
// out[out0, out0 + a + b).  Payloads use the same positions as their keys.
// Bit 31 of a_f (b_f) is set when keys[ka0 + a] (keys[kb0 + b]) is the next
// element of the same source array, i.e. the segment's successor exists.
// Written by the case-selection kernel (Steps 3-4), read by the merge kernel.
// Jobs of the batch engine (whole merges) use the same record; a job's
// lengths may reach 2^30.  In a subproblem, whose lengths stay below the
// merge capacity, bit 30 of b_f marks the first subproblem of a merge in a
// list that holds several independent merges: packed steps never join
// across it.
// ---------------------------------------------------------------------------
struct PieceDesc {
    int64_t ka0, kb0, out0;
    uint32_t a_f, b_f;
};
static_assert(sizeof(PieceDesc) == 32, "descriptors are read as two 16-byte chunks");
constexpr uint32_t kSuccBit = 0x80000000u;
constexpr uint32_t kFirstBit = 0x40000000u;
// lengths of a job
__host__ __device__ inline int desc_a(const PieceDesc& d) { return (int)(d.a_f & ~kSuccBit); }
__host__ __device__ inline int desc_b(const PieceDesc& d) { return (int)(d.b_f & ~kSuccBit); }
// lengths of a subproblem
__host__ __device__ inline int piece_a(const PieceDesc& d) {
    return (int)(d.a_f & ~(kSuccBit | kFirstBit));
}
__host__ __device__ inline int piece_b(const PieceDesc& d) {
    return (int)(d.b_f & ~(kSuccBit | kFirstBit));
}

template <typename K>
struct Vec { static constexpr int N = 16 / sizeof(K); };


// rank_low / rank_high of x over X[0, n) in LDS, branch-free (the halving
// length is workgroup-uniform, so only the base moves per lane): the answer
// stays in [base, base + len] while len halves.
template <typename K>
__device__ __forceinline__ int lower_bound_lds(const K* X, int n, K x) {
    if (n <= 0) return 0;
    int base = 0;
    for (int len = n; len > 1;) {
        const int half = len >> 1;
        base = X[base + half] < x ? base + half : base;
        len -= half;
    }
    return base + (X[base] < x ? 1 : 0);
}

template <typename K>
__device__ __forceinline__ int upper_bound_lds(const K* X, int n, K x) {
    if (n <= 0) return 0;
    int base = 0;
    for (int len = n; len > 1;) {
        const int half = len >> 1;
        base = !(x < X[base + half]) ? base + half : base;
        len -= half;
    }
    return base + (!(x < X[base]) ? 1 : 0);
}

// Both lane-level searches at once: lower_bound of x in X[0, nx) and
// upper_bound of y in Y[0, ny).  The two probe chains are independent, so
// each step issues both reads before waiting: half the dependent LDS round
// trips of running them one after the other.
template <typename K, int STEPS, bool TOGETHER>
__device__ __forceinline__ void paired_bounds_lds(const K* X, int nx, K x, const K* Y, int ny, K y,
                                                  int& rx, int& ry) {
    if constexpr (!TOGETHER) {
        // one chain after the other: fewer registers live at once (the
        // payload kernels keep two sets of payload loads in flight as well)
        rx = nx > 0 ? lower_bound_lds<K>(X, nx, x) : 0;
        ry = ny > 0 ? upper_bound_lds<K>(Y, ny, y) : 0;
        return;
    }
    // the bases are LDS pointers: a step is one add (probe address), the
    // read, the compare and one select
    const K* bx = X;
    const K* by = Y;
    int lx = nx, ly = ny;
    // STEPS >= ceil(log2(max(nx, ny))); once a length reaches 1 its half is
    // 0 and the step re-reads the same slot without moving.  (A count taken
    // from the lengths saves steps on small segments but, as a loop the
    // compiler cannot unroll, measured slower on full ones.)
#pragma unroll
    for (int i = 0; i < STEPS; ++i) {
        const int hx = lx >> 1, hy = ly >> 1;
        const K* px = bx + hx;
        const K* py = by + hy;
        const K vx = *px;
        const K vy = *py;
        bx = vx < x ? px : bx;
        by = !(y < vy) ? py : by;
        lx -= hx;
        ly -= hy;
    }
    // an empty side leaves its base at the start and must not add the last
    // compare; the compare is masked rather than branched on, so the
    // compiler keeps both chains in one block and issues their reads together
    // slot index = byte distance / sizeof(K), in 32-bit arithmetic (the low
    // half of a generic LDS address is the LDS offset)
    const uint32_t dx = (uint32_t)(uintptr_t)bx - (uint32_t)(uintptr_t)X;
    const uint32_t dy = (uint32_t)(uintptr_t)by - (uint32_t)(uintptr_t)Y;
    rx = (int)(dx / sizeof(K)) + (int)((nx > 0) & (*bx < x));
    ry = (int)(dy / sizeof(K)) + (int)((ny > 0) & !(y < *by));
}

template <typename K, bool TOGETHER>
__device__ __forceinline__ void paired_bounds_any(const K* X, int nx, K x, const K* Y, int ny, K y,
                                                  int& rx, int& ry) {
    const int n = nx > ny ? nx : ny;
    if (n <= 4096) {
        paired_bounds_lds<K, 12, TOGETHER>(X, nx, x, Y, ny, y, rx, ry);
    } else {
        rx = lower_bound_lds<K>(X, nx, x);
        ry = upper_bound_lds<K>(Y, ny, y);
    }
}

// ---------------------------------------------------------------------------
// Workgroup merge of one subproblem, in phases:
//   plan     uniform window geometry of the A and B segments and of C
//   prefetch 16-byte chunk loads of both windows into registers (the loads
//            stay in flight while the workgroup merges the previous piece)
//   commit   registers -> LDS
//   merge    lane-level cross ranks, per-lane merges, write-back
//
// LDS layout (slot = one key):
//   sKey[0, wa)            A window: 16-byte chunks from A's aligned start,
//                          A[i] at slot offA + i, successor at offA + a
//   sKey[wa, wa + nb*V)    B window, B[j] at slot wa + offB + j, successor
//                          at wa + offB + b
//   sPay                   payload windows, A[i] at offPA + i, B[j] at
//                          waP + offPB + j (for 32-bit keys the same slots
//                          as the keys: offPA = offA, waP = wa, offPB = offB)
//   sOut                   merged keys, output k at offC + k
//   sIdx                   payloads of the outputs, output k at offCP + k
//                          (64-bit keys: first the key slot of output k,
//                          replaced by its payload in a gather pass)
//   sXb[L+1], sYb[L+1]     lane-level cross ranks
//
// Lane level: the workgroup is p = L processing elements.  The A and B
// segments are split into L blocks each (the paper's block decomposition);
// lane t computes xbar_t = rank_low(A[x_t], B) and ybar_t = rank_high(B[y_t], A)
// by binary search in LDS; after one barrier it merges its Step-3 subproblem
// and its Step-4 subproblem with a sequential stable merge (take B only if
// strictly smaller), writing each output to its slot in LDS.  After a second
// barrier the workgroup writes C with aligned 16-byte stores, and element
// stores at the two partial ends.
//
// Sentinels.  In every case of Steps 3-4 the element right after a
// subproblem's A range is strictly greater than all of its B elements, and
// the element right after its B range is greater than or equal to all of its
// A elements (both follow from the cross-rank definitions).  So when one side
// runs out, its next element steers the comparison "take B iff B < A" to the
// other side, and the merge loop needs no bounds checks.  The windows stage
// one element past each segment for this.  Where a segment ends its array,
// the slot holds the key type's maximum: correct for the B side always, and
// for the A side unless the segment's B part contains that maximum -- then
// the workgroup uses the bounds-checked loop instead.
// ---------------------------------------------------------------------------
template <typename K, bool PAY, int L>
struct MergeSmem {
    // a lane keeps merging past its own range until the slowest lane of its
    // wave is done (at most one lane subproblem, ceil(cap / L) + 1 elements),
    // so key and output slots carry that much slack past the subproblem
    static __host__ __device__ uint32_t slack(uint32_t cap) { return 2 * ((cap + L - 1) / L) + 16; }
    static __host__ __device__ uint32_t key_slots(uint32_t cap) {
        return (cap + 4 * Vec<K>::N + 8 + slack(cap) + 7) & ~7u;
    }
    static __host__ __device__ uint32_t pay_slots(uint32_t cap) { return (cap + 24 + 7) & ~7u; }
    static __host__ __device__ uint32_t out_slots(uint32_t cap) {
        return (cap + Vec<K>::N + 8 + slack(cap) + 7) & ~7u;
    }
    static __host__ __device__ uint32_t bytes(uint32_t cap) {
        uint32_t b = key_slots(cap) * sizeof(K) + out_slots(cap) * sizeof(K);
        if (PAY) b += pay_slots(cap) * 4 + out_slots(cap) * 4;
        b += 2 * (L + 1) * 4;
        return (b + 15) & ~15u;
    }
};

struct SegPlan {
    int a, b, s;
    int offA, offB, wa, nca, ncb;      // key windows (chunks of V keys)
    int offPA, offPB, waP, ncpa, ncpb; // payload windows (chunks of 4)
    int offC, offCP;                   // alignment of the outputs
    int qsA, esA, qsB, esB;            // chunk / element holding each successor slot
    bool succA, succB;                 // successor present in the source array
    int64_t ka_al, kb_al, c0;          // aligned absolute starts, output start
};

template <typename K, bool PAY>
__device__ __forceinline__ SegPlan make_plan(const PieceDesc& d) {
    constexpr int V = Vec<K>::N;
    SegPlan p;
    p.a = piece_a(d);
    p.b = piece_b(d);
    p.s = p.a + p.b;
    p.succA = (d.a_f & kSuccBit) != 0;
    p.succB = (d.b_f & kSuccBit) != 0;
    // arrays start 16-byte aligned, so alignment follows from the index
    p.offA = (int)(d.ka0 & (V - 1));
    p.offB = (int)(d.kb0 & (V - 1));
    p.ka_al = d.ka0 - p.offA;
    p.kb_al = d.kb0 - p.offB;
    // one extra slot per window for the successor
    p.nca = (p.offA + p.a + 1 + V - 1) / V;
    p.ncb = (p.offB + p.b + 1 + V - 1) / V;
    p.wa = p.nca * V;
    p.qsA = (p.offA + p.a) / V;
    p.esA = (p.offA + p.a) % V;
    p.qsB = p.nca + (p.offB + p.b) / V;
    p.esB = (p.offB + p.b) % V;
    p.offPA = (int)(d.ka0 & 3);
    p.offPB = (int)(d.kb0 & 3);
    if constexpr (PAY && sizeof(K) == 4) {
        // 32-bit keys: the payload windows take the key windows' geometry
        // slot for slot (successor chunk included), so the payload of the
        // key in slot i sits in payload slot i
        p.ncpa = p.nca;
        p.ncpb = p.ncb;
    } else {
        p.ncpa = PAY ? (p.offPA + p.a + 3) / 4 : 0;
        p.ncpb = PAY ? (p.offPB + p.b + 3) / 4 : 0;
    }
    p.waP = p.ncpa * 4;
    p.c0 = d.out0;
    p.offC = (int)(d.out0 & (V - 1));
    p.offCP = (int)(d.out0 & 3);
    return p;
}

// Issue the 16-byte loads of two windows into registers: chunk q goes to
// rk[q / L] of thread q % L (first window first).  Every slot is loaded
// unconditionally; slots past both windows use an offset beyond the buffer
// resource's range, which returns zeros without a memory access.  (A
// conditional load would have to merge with the register's previous value,
// making the load wait for everything in flight, stores included.)  When both
// windows lie within 4 GiB of the lower one, one resource based there serves
// both; otherwise each window gets its own and every slot issues two loads.
constexpr uint32_t kOffNone = 0xFFFFFFF0u;

template <int L, int R>
__device__ __forceinline__ void load_windows(const char* base, uint64_t bytes_to_end, int64_t wa0,
                                             int na, int64_t wb0, int nb, u32x4 (&rk)[R]) {
    const int t = threadIdx.x;
    const int64_t lo = wa0 < wb0 ? wa0 : wb0;
    const int64_t hi = (wa0 + 16ll * na) > (wb0 + 16ll * nb) ? (wa0 + 16ll * na) : (wb0 + 16ll * nb);
    if (hi - lo <= 0xFFFFFF00ll) {
        const __amdgpu_buffer_rsrc_t r = make_rsrc(base + lo, bytes_to_end - (uint64_t)lo);
        const uint32_t oa = (uint32_t)(wa0 - lo), ob = (uint32_t)(wb0 - lo);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int q = i * L + t;
            const uint32_t off = q < na ? oa + q * 16 : (q < na + nb ? ob + (q - na) * 16 : kOffNone);
            rk[i] = buf_load16(r, off);
        }
    } else {
        const __amdgpu_buffer_rsrc_t rA = make_rsrc(base + wa0, bytes_to_end - (uint64_t)wa0);
        const __amdgpu_buffer_rsrc_t rB = make_rsrc(base + wb0, bytes_to_end - (uint64_t)wb0);
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int q = i * L + t;
            const u32x4 va = buf_load16(rA, q < na ? q * 16 : kOffNone);
            const u32x4 vb = buf_load16(rB, q >= na && q < na + nb ? (q - na) * 16 : kOffNone);
            rk[i] = q < na ? va : vb;
        }
    }
}

template <typename K, bool PAY, int L, int R>
__device__ __forceinline__ void prefetch(const SegPlan& p, const K* keys, uint64_t nkeys,
                                         const uint32_t* pay, u32x4 (&rk)[R], u32x4 (&rp)[R]) {
    load_windows<L, R>(reinterpret_cast<const char*>(keys), nkeys * sizeof(K),
                       p.ka_al * (int64_t)sizeof(K), p.nca, p.kb_al * (int64_t)sizeof(K), p.ncb, rk);
    if (PAY)
        load_windows<L, R>(reinterpret_cast<const char*>(pay), nkeys * 4,
                           (p.ka_al + p.offA - p.offPA) * 4, p.ncpa,
                           (p.kb_al + p.offB - p.offPB) * 4, p.ncpb, rp);
}

// The same loads with one buffer resource spanning the whole array, for
// arrays below 4 GiB: every slot is one load at a 32-bit byte offset, and
// the registers are not touched again until the commit that consumes them.
template <int L, int R>
__device__ __forceinline__ void load_windows_whole(__amdgpu_buffer_rsrc_t r, int64_t wa0, int na,
                                                   int64_t wb0, int nb, u32x4 (&rk)[R]) {
    const int t = threadIdx.x;
    const uint32_t oa = (uint32_t)wa0, ob = (uint32_t)wb0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int q = i * L + t;
        const uint32_t off = q < na ? oa + q * 16 : (q < na + nb ? ob + (q - na) * 16 : kOffNone);
        rk[i] = buf_load16(r, off);
    }
}

template <typename K, bool PAY, int L, int R>
__device__ __forceinline__ void prefetch_whole(const SegPlan& p, __amdgpu_buffer_rsrc_t rkeys,
                                               __amdgpu_buffer_rsrc_t rpay, u32x4 (&rk)[R],
                                               u32x4 (&rp)[R]) {
    load_windows_whole<L, R>(rkeys, p.ka_al * (int64_t)sizeof(K), p.nca,
                             p.kb_al * (int64_t)sizeof(K), p.ncb, rk);
    if (PAY)
        load_windows_whole<L, R>(rpay, (p.ka_al + p.offA - p.offPA) * 4, p.ncpa,
                                 (p.kb_al + p.offB - p.offPB) * 4, p.ncpb, rp);
}

// Window loads for keys of arrays of 4 GiB or more (no payloads): each
// window gets a buffer resource of its own, A's chunks fill the register
// slots [0, sA) with sA = ceil(nca / L) and B's chunks the slots from sA
// on, so each slot's load uses one (workgroup-uniform) resource and no slot
// needs a select between two loads.  RS slots hold any subproblem whose
// chunks fit RS - 1 full slots.
template <typename K, int L, int RS>
__device__ __forceinline__ void prefetch_split(const SegPlan& p, const K* keys, uint64_t nkeys,
                                               u32x4 (&rk)[RS]) {
    const int t = threadIdx.x;
    const char* base = reinterpret_cast<const char*>(keys);
    const uint64_t bytes = nkeys * sizeof(K);
    const uint64_t wa0 = (uint64_t)p.ka_al * sizeof(K), wb0 = (uint64_t)p.kb_al * sizeof(K);
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(base + wa0, wa0 < bytes ? bytes - wa0 : 0);
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(base + wb0, wb0 < bytes ? bytes - wb0 : 0);
    const int sA = (p.nca + L - 1) / L;
#pragma unroll
    for (int i = 0; i < RS; ++i) {
        const bool isA = i < sA;
        const int q = (isA ? i : i - sA) * L + t;
        const int nq = isA ? p.nca : p.ncb;
        rk[i] = buf_load16(isA ? rA : rB, q < nq ? (uint32_t)q * 16u : kOffNone);
    }
}

// Registers -> LDS for prefetch_split's slot layout; the successor slots
// are patched by the lanes that wrote their chunks.
template <typename K, int L, int RS>
__device__ __forceinline__ void commit_split(const SegPlan& p, const u32x4 (&rk)[RS], K* sKey) {
    constexpr int V = Vec<K>::N;
    const int t = threadIdx.x;
    const int sA = (p.nca + L - 1) / L;
#pragma unroll
    for (int i = 0; i < RS; ++i) {
        const bool isA = i < sA;
        const int q = (isA ? i : i - sA) * L + t;
        if (q < (isA ? p.nca : p.ncb))
            *reinterpret_cast<u32x4*>(sKey + (isA ? q * V : p.wa + q * V)) = rk[i];
    }
    if (!p.succA && t == p.qsA % L) sKey[p.offA + p.a] = KeyMax<K>::v;
    if (!p.succB && t == (p.qsB - p.nca) % L) sKey[p.wa + p.offB + p.b] = KeyMax<K>::v;
}

// A successor slot whose segment ends its source array must hold the key
// type's maximum.  The lane that wrote the chunk holding the slot overwrites
// it after its own chunk write, so no other lane races on it.
template <typename K, int L>
__device__ __forceinline__ void fix_successors(const SegPlan& p, K* sKey) {
    const int t = threadIdx.x;
    if (!p.succA && t == p.qsA % L) sKey[p.offA + p.a] = KeyMax<K>::v;
    if (!p.succB && t == p.qsB % L) sKey[p.wa + p.offB + p.b] = KeyMax<K>::v;
}

// Wait until at most N vector memory operations of this wave are in flight,
// without waiting on the other counters (gfx9 s_waitcnt encoding: vmcnt in
// bits 3:0 and 15:14, expcnt in 6:4, lgkmcnt in 11:8).  Loads complete in
// issue order, so after wait_vm<N> every load issued before the last N
// operations has landed.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit field");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// Registers -> LDS.  The caller has waited for the loads that filled rk / rp.
template <typename K, bool PAY, int L, int R>
__device__ __forceinline__ void commit(const SegPlan& p, const u32x4 (&rk)[R],
                                       const u32x4 (&rp)[R], K* sKey, uint32_t* sPay) {
    constexpr int V = Vec<K>::N;
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int q = r * L + t;
        if (q < p.nca + p.ncb)
            *reinterpret_cast<u32x4*>(sKey + (q < p.nca ? q * V : p.wa + (q - p.nca) * V)) = rk[r];
    }
    fix_successors<K, L>(p, sKey);
    if (PAY) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int q = r * L + t;
            if (q < p.ncpa + p.ncpb)
                *reinterpret_cast<u32x4*>(sPay + (q < p.ncpa ? q * 4 : p.waP + (q - p.ncpa) * 4)) = rp[r];
        }
    }
}

// Direct staging (no register prefetch) for subproblems too large for the
// register-pipelined path: chunk loop straight from global memory to LDS.
template <typename K, bool PAY, int L>
__device__ __forceinline__ void stage_direct(const SegPlan& p, const K* keys, uint64_t nkeys,
                                             const uint32_t* pay, K* sKey, uint32_t* sPay) {
    constexpr int V = Vec<K>::N;
    const int t = threadIdx.x;
    const __amdgpu_buffer_rsrc_t rA = make_rsrc(keys + p.ka_al, (nkeys - p.ka_al) * sizeof(K));
    const __amdgpu_buffer_rsrc_t rB = make_rsrc(keys + p.kb_al, (nkeys - p.kb_al) * sizeof(K));
    for (int q = t; q < p.nca + p.ncb; q += L) {
        if (q < p.nca) *reinterpret_cast<u32x4*>(sKey + q * V) = buf_load16(rA, q * 16);
        else *reinterpret_cast<u32x4*>(sKey + p.wa + (q - p.nca) * V) = buf_load16(rB, (q - p.nca) * 16);
    }
    // the successor slots belong to chunks this lane may not have written:
    // order the patch after every chunk write
    __syncthreads();
    if (t == 0) {
        if (!p.succA) sKey[p.offA + p.a] = KeyMax<K>::v;
        if (!p.succB) sKey[p.wa + p.offB + p.b] = KeyMax<K>::v;
    }
    if (PAY) {
        const __amdgpu_buffer_rsrc_t qA = make_rsrc(pay + (p.ka_al + p.offA - p.offPA),
                                                    (nkeys - (p.ka_al + p.offA - p.offPA)) * 4);
        const __amdgpu_buffer_rsrc_t qB = make_rsrc(pay + (p.kb_al + p.offB - p.offPB),
                                                    (nkeys - (p.kb_al + p.offB - p.offPB)) * 4);
        for (int q = t; q < p.ncpa + p.ncpb; q += L) {
            if (q < p.ncpa) *reinterpret_cast<u32x4*>(sPay + q * 4) = buf_load16(qA, q * 16);
            else *reinterpret_cast<u32x4*>(sPay + p.waP + (q - p.ncpa) * 4) = buf_load16(qB, (q - p.ncpa) * 16);
        }
    }
}

// Sequential stable merges of a lane's two subproblems (A slots from ia, B
// slots from ib, len outputs at slots from co, payload outputs from cp), in
// one loop: the two chains of dependent LDS reads are independent, so each
// step waits once for both.
//
// Uniform form (sentinels valid): every lane of the wave runs the same number
// of steps, the largest of the two lengths maximised over the wave.  A lane
// that is done keeps merging: its start (ia, ib) is a prefix state of the
// stable merge (the outputs before its c_off are exactly A[0, a_lo) and
// B[0, b_lo)), so its extra outputs are the true next outputs -- the same
// values the lanes owning those slots write -- or lie past the subproblem, in
// slack slots nobody reads.  Reads stay valid until the lane has output the
// whole subproblem: the successors stand in for the element after each
// segment.
template <typename K, bool PAY, bool DIRECT>
__device__ __forceinline__ void lane_merge_uniform2(const K* sKey, K* sOut, uint32_t* sIdx,
                                                    int dPay, const uint32_t* sPay, int dA, int dB,
                                                    int ia1, int ib1, int len1, int co1,
                                                    int cp1, int ia2, int ib2, int len2, int co2,
                                                    int cp2) {
    const int len = len1 > len2 ? len1 : len2;
    if (!__any(len > 0)) return;
    if constexpr (!PAY || DIRECT) {
        // walk LDS pointers rather than slot indices, which saves the
        // index-to-address step on every read; with DIRECT payloads the
        // payload of the taken key is read dPay slots further on
        const K *pa1 = sKey + ia1, *pb1 = sKey + ib1, *pa2 = sKey + ia2, *pb2 = sKey + ib2;
        K *po1 = sOut + co1, *po2 = sOut + co2;
        uint32_t* pp1 = DIRECT ? sIdx + cp1 : nullptr;
        uint32_t* pp2 = DIRECT ? sIdx + cp2 : nullptr;
        K ka1 = *pa1, kb1 = *pb1, ka2 = *pa2, kb2 = *pb2;
        int k = 0;
        do {
            const bool t1 = kb1 < ka1;
            const bool t2 = kb2 < ka2;
            const K* s1 = t1 ? pb1 : pa1;
            const K* s2 = t2 ? pb2 : pa2;
            po1[k] = t1 ? kb1 : ka1;
            po2[k] = t2 ? kb2 : ka2;
            if constexpr (DIRECT) {
                pp1[k] = reinterpret_cast<const uint32_t*>(s1)[dPay];
                pp2[k] = reinterpret_cast<const uint32_t*>(s2)[dPay];
            }
            const K kn1 = s1[1];
            const K kn2 = s2[1];
            pb1 = t1 ? s1 + 1 : pb1;
            pa1 = t1 ? pa1 : s1 + 1;
            kb1 = t1 ? kn1 : kb1;
            ka1 = t1 ? ka1 : kn1;
            pb2 = t2 ? s2 + 1 : pb2;
            pa2 = t2 ? pa2 : s2 + 1;
            kb2 = t2 ? kn2 : kb2;
            ka2 = t2 ? ka2 : kn2;
            ++k;
        } while (__any(k < len));
        return;
    }
    K ka1 = sKey[ia1], kb1 = sKey[ib1];
    K ka2 = sKey[ia2], kb2 = sKey[ib2];
    int k = 0;
    do {
        const bool t1 = kb1 < ka1;
        const bool t2 = kb2 < ka2;
        const int s1 = t1 ? ib1 : ia1;
        const int s2 = t2 ? ib2 : ia2;
        sOut[co1 + k] = t1 ? kb1 : ka1;
        sOut[co2 + k] = t2 ? kb2 : ka2;
        if (PAY) {
            // the payload of key slot s sits at payload slot s + dA (A) or
            // s + dB (B); past the end of a lane's range the value read is
            // never written back
            sIdx[cp1 + k] = sPay[s1 + (t1 ? dB : dA)];
            sIdx[cp2 + k] = sPay[s2 + (t2 ? dB : dA)];
        }
        const int n1 = s1 + 1, n2 = s2 + 1;
        const K kn1 = sKey[n1];
        const K kn2 = sKey[n2];
        ib1 = t1 ? n1 : ib1;
        ia1 = t1 ? ia1 : n1;
        kb1 = t1 ? kn1 : kb1;
        ka1 = t1 ? ka1 : kn1;
        ib2 = t2 ? n2 : ib2;
        ia2 = t2 ? ia2 : n2;
        kb2 = t2 ? kn2 : kb2;
        ka2 = t2 ? ka2 : kn2;
        ++k;
    } while (__any(k < len));
}

// Batcher's odd-even merge network on v[LO..HI] (HI inclusive) at stride R:
// with both halves sorted, the compare-exchanges leave the whole range
// sorted.  Fully unrolled: every index is a compile-time constant, so the
// values stay in registers.
template <typename K>
__device__ __forceinline__ void cmp_exchange(K& x, K& y) {
    const K lo = y < x ? y : x;
    const K hi = y < x ? x : y;
    x = lo;
    y = hi;
}

template <int I, int END, int STEP, int R>
struct CmpExchangeRun {
    template <typename K>
    static __device__ __forceinline__ void run(K* v) {
        if constexpr (I < END) {
            cmp_exchange(v[I], v[I + R]);
            CmpExchangeRun<I + STEP, END, STEP, R>::run(v);
        }
    }
};

template <int LO, int HI, int R>
struct OddEvenMerge {
    template <typename K>
    static __device__ __forceinline__ void run(K* v) {
        constexpr int STEP = 2 * R;
        if constexpr (STEP < HI - LO) {
            OddEvenMerge<LO, HI, STEP>::run(v);
            OddEvenMerge<LO + R, HI, STEP>::run(v);
            CmpExchangeRun<LO + R, HI - R, STEP, R>::template run<K>(v);
        } else {
            cmp_exchange(v[LO], v[LO + R]);
        }
    }
};

// Bounds-checked form: each lane stops after its own la + lb outputs.
template <typename K, bool PAY, bool DIRECT>
__device__ __forceinline__ void lane_merge_checked(const K* sKey, K* sOut, uint32_t* sIdx, int dPay,
                                                   const uint32_t* sPay, int dA, int dB,
                                                   int ia, int la, int ib, int lb, int co, int cp) {
    const int len = la + lb;
    const int ea = ia + la, eb = ib + lb;
    K ka = sKey[ia];
    K kb = sKey[ib];
    for (int k = 0; k < len; ++k) {
        const bool takeB = (ib < eb) && (ia >= ea || kb < ka);
        const int src = takeB ? ib : ia;
        sOut[co + k] = takeB ? kb : ka;
        if constexpr (DIRECT) sIdx[cp + k] = reinterpret_cast<const uint32_t*>(sKey)[src + dPay];
        else if (PAY) sIdx[cp + k] = sPay[src + (takeB ? dB : dA)];
        const int nxt = src + 1;
        const K kn = sKey[nxt];
        if (takeB) { ib = nxt; kb = kn; }
        else { ia = nxt; ka = kn; }
    }
}

// Lane-level split and per-lane merges of a staged subproblem.  Entered by
// the whole workgroup after a barrier that follows commit / stage_direct;
// ends after a barrier, with output k in sOut[offC + k] (and, with payloads,
// its payload in sIdx[offCP + k]).  The staging buffers are free afterwards.
// LEAN = the caller has registers to spare: both lane-level searches run
// together and lane blocks use select arithmetic (otherwise the searches run
// one after the other and the block arithmetic branches, to stay within the
// payload kernels' register budget).
// Lane-level cross ranks (Steps 1-2 inside the workgroup) of a staged
// subproblem: lane t writes xbar_t to sXb[t] and ybar_t to sYb[t], lane 0
// also sXb[L] = b and sYb[L] = a; ends at a barrier.  The searches are short
// chains of LDS reads that end at that barrier: they run above the merges
// of other workgroups.
template <typename K, int L, bool LEAN>
__device__ __forceinline__ void lane_split(const SegPlan& p, const K* sKey,
                                           const LaneBlocks<L, LEAN>& LA,
                                           const LaneBlocks<L, LEAN>& LB, int* sXb, int* sYb) {
    const int t = threadIdx.x;
    const int a = p.a, b = p.b;
    const int baseA = p.offA, baseB = p.wa + p.offB;
    __builtin_amdgcn_s_setprio(1);
    {
        const int xt = LA.start(t), yt = LB.start(t);
        // lanes without a block start search with the successor slot's key
        // and discard the result
        int rx, ry;
        paired_bounds_any<K, LEAN>(sKey + baseB, b, sKey[baseA + (xt < a ? xt : a)], sKey + baseA, a,
                             sKey[baseB + (yt < b ? yt : b)], rx, ry);
        sXb[t] = xt < a ? rx : b;
        sYb[t] = yt < b ? ry : a;
        if (t == 0) {
            sXb[L] = b;
            sYb[L] = a;
        }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
}

template <typename K, bool PAY, int L, bool LEAN = !PAY>
__device__ __forceinline__ void merge_lanes(const SegPlan& p, const K* sKey, const uint32_t* sPay,
                                            K* sOut, uint32_t* sIdx, int* sXb, int* sYb) {
    const int t = threadIdx.x;
    const int a = p.a, b = p.b, s = p.s;
    const int baseA = p.offA, baseB = p.wa + p.offB;
    // 32-bit keys: payload slot = key slot + dPay (the payload windows share
    // the key windows' geometry, and dPay is the distance between the two
    // arrays in LDS); 64-bit keys: payload slot = key slot + dA in A's window
    // and + dB in B's (payload chunks hold twice as many elements as key
    // chunks).  Either way the merges write the payloads themselves.
    constexpr bool DIRECT = PAY && sizeof(K) == 4;
    const int dPay = DIRECT ? (int)(sPay - reinterpret_cast<const uint32_t*>(sKey)) : 0;
    const int dA = p.offPA - p.offA;
    const int dB = (p.waP + p.offPB) - (p.wa + p.offB);

    // ---- lane-level cross ranks (Steps 1-2 inside the workgroup) ----------
    const LaneBlocks<L, LEAN> LA(a), LB(b);
    lane_split<K, L, LEAN>(p, sKey, LA, LB, sXb, sYb);

    // the sentinel loop is exact unless the A successor is the type maximum
    // and the B part holds that maximum too
    const bool fast = p.succA || b == 0 || sKey[baseB + b - 1] != KeyMax<K>::v;

    // ---- per-lane stable sequential merges (Steps 3-4 inside the WG) ------
    // lane t is the processing element of A block t (Step 3) and of B block
    // t (Step 4); a descriptor outside the segment would be a bug and merges
    // nothing
    // (no arrays indexed by a loop variable here: they would live in scratch
    // memory, i.e. extra HBM traffic)
    const Piece<int> p3 = step3_piece<int>(LA, LB, sXb, sYb, t);
    const Piece<int> p4 = step4_piece<int>(LA, LB, sXb, sYb, t);
    auto valid = [&](const Piece<int>& q) {
        return 0 <= q.a_lo && q.a_lo <= q.a_hi && q.a_hi <= a && 0 <= q.b_lo && q.b_lo <= q.b_hi &&
               q.b_hi <= b && 0 <= q.c_off && q.c_off + (q.a_hi - q.a_lo) + (q.b_hi - q.b_lo) <= s;
    };
    const bool ok3 = valid(p3), ok4 = valid(p4);
    const int la3 = ok3 ? p3.a_hi - p3.a_lo : 0, lb3 = ok3 ? p3.b_hi - p3.b_lo : 0;
    const int la4 = ok4 ? p4.a_hi - p4.a_lo : 0, lb4 = ok4 ? p4.b_hi - p4.b_lo : 0;
    if (fast) {
        lane_merge_uniform2<K, PAY, DIRECT>(sKey, sOut, sIdx, dPay, sPay, dA, dB, baseA + p3.a_lo,
                                            baseB + p3.b_lo, la3 + lb3, p.offC + p3.c_off,
                                            p.offCP + p3.c_off, baseA + p4.a_lo, baseB + p4.b_lo,
                                            la4 + lb4, p.offC + p4.c_off, p.offCP + p4.c_off);
    } else {
        lane_merge_checked<K, PAY, DIRECT>(sKey, sOut, sIdx, dPay, sPay, dA, dB, baseA + p3.a_lo, la3,
                                           baseB + p3.b_lo, lb3, p.offC + p3.c_off,
                                           p.offCP + p3.c_off);
        lane_merge_checked<K, PAY, DIRECT>(sKey, sOut, sIdx, dPay, sPay, dA, dB, baseA + p4.a_lo, la4,
                                           baseB + p4.b_lo, lb4, p.offC + p4.c_off,
                                           p.offCP + p4.c_off);
    }
    __syncthreads();

}

// Lane-level split and per-lane merges of a staged subproblem whose outputs
// go straight to memory: output k to out[c0 + k] (and its payload to
// out_pay[c0 + k]).  Each lane merges exactly its two pieces (no uniform
// trip count, which would write past a piece), so no output buffer is
// needed in LDS.  Entered after the barrier that follows staging; the
// staging buffers may be reused only after a further barrier.
template <typename K, bool PAY, int L>
__device__ __forceinline__ void merge_lanes_to_memory(const SegPlan& p, const K* sKey,
                                                      const uint32_t* sPay, int* sXb, int* sYb,
                                                      K* out, uint32_t* out_pay) {
    const int t = threadIdx.x;
    const int a = p.a, b = p.b, s = p.s;
    const int baseA = p.offA, baseB = p.wa + p.offB;
    constexpr bool DIRECT = PAY && sizeof(K) == 4;
    const int dPay = DIRECT ? (int)(sPay - reinterpret_cast<const uint32_t*>(sKey)) : 0;
    const int dA = p.offPA - p.offA;
    const int dB = (p.waP + p.offPB) - (p.wa + p.offB);
    const LaneBlocks<L, true> LA(a), LB(b);
    lane_split<K, L, true>(p, sKey, LA, LB, sXb, sYb);
    const Piece<int> p3 = step3_piece<int>(LA, LB, sXb, sYb, t);
    const Piece<int> p4 = step4_piece<int>(LA, LB, sXb, sYb, t);
    auto valid = [&](const Piece<int>& q) {
        return 0 <= q.a_lo && q.a_lo <= q.a_hi && q.a_hi <= a && 0 <= q.b_lo && q.b_lo <= q.b_hi &&
               q.b_hi <= b && 0 <= q.c_off && q.c_off + (q.a_hi - q.a_lo) + (q.b_hi - q.b_lo) <= s;
    };
    const bool ok3 = valid(p3), ok4 = valid(p4);
    // slot k of the merges' output indexing (offC / offCP + output index) is
    // out[c0 - offC + k] (out_pay[c0 - offCP + k])
    K* gOut = out + (p.c0 - p.offC);
    uint32_t* gPay = PAY ? out_pay + (p.c0 - p.offCP) : nullptr;
    lane_merge_checked<K, PAY, DIRECT>(sKey, gOut, gPay, dPay, sPay, dA, dB, baseA + p3.a_lo,
                                       ok3 ? p3.a_hi - p3.a_lo : 0, baseB + p3.b_lo,
                                       ok3 ? p3.b_hi - p3.b_lo : 0, p.offC + p3.c_off,
                                       p.offCP + p3.c_off);
    lane_merge_checked<K, PAY, DIRECT>(sKey, gOut, gPay, dPay, sPay, dA, dB, baseA + p4.a_lo,
                                       ok4 ? p4.a_hi - p4.a_lo : 0, baseB + p4.b_lo,
                                       ok4 ? p4.b_hi - p4.b_lo : 0, p.offC + p4.c_off,
                                       p.offCP + p4.c_off);
}

// One output array of a subproblem, LDS -> HBM: aligned 16-byte stores for
// whole chunks, element stores at the two partial ends.  RW = number of
// output chunks per thread, unrolled (0 = a loop, for large subproblems).
template <typename E, int L, int RW>
__device__ __forceinline__ void write_out(const E* sArr, int off, int s, E* base_out) {
    // base_out = output position of sArr[0]; elements [off, off + s) are real;
    // chunks of V = 16 / sizeof(E) elements aligned to base_out
    constexpr int V = 16 / sizeof(E);
    const int t = threadIdx.x;
    const int q0 = (off + V - 1) / V, q1 = (off + s) / V;   // full chunks [q0, q1)
    // the merged stream is written once and not read back soon:
    // non-temporal stores keep it from evicting the cached lines that the
    // cross-rank searches reuse
    auto chunk = [&](int q) {
        __builtin_nontemporal_store(*reinterpret_cast<const u32x4*>(sArr + q * V),
                                    reinterpret_cast<u32x4*>(base_out + q * V));
    };
    if (RW > 0) {
        // all LDS reads first (a chunk past the end re-reads chunk q0 and is
        // not stored), so one wait covers them, then the stores
        u32x4 v[RW > 0 ? RW : 1];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int q = q0 + r * L + t;
            v[r] = *reinterpret_cast<const u32x4*>(sArr + (q < q1 ? q : q0) * V);
        }
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int q = q0 + r * L + t;
            if (q < q1) __builtin_nontemporal_store(v[r], reinterpret_cast<u32x4*>(base_out + q * V));
        }
    } else {
        for (int q = q0 + t; q < q1; q += L) chunk(q);
    }
    // the elements outside the full chunks: at most V - 1 at each end
    if (t < 2 * V) {
        int k;
        if (q1 < q0) k = t < V ? off + t : off + s;   // no full chunk: head covers all
        else k = t < V ? off + t : q1 * V + (t - V);
        const bool head = t < V && k < (q1 < q0 ? off + s : q0 * V);
        const bool tail = t >= V && q1 >= q0 && k < off + s;
        if (head || tail) base_out[k] = sArr[k];
    }
}

// Write-back of merged outputs: aligned 16-byte stores for whole chunks,
// element stores at the two partial ends.  Reads only sOut / sIdx, so it
// may run after the staging buffers have been refilled.  RW = number of
// output chunks per thread, unrolled (0 = a loop, for large subproblems).
template <typename K, bool PAY, int L, int RW>
__device__ __forceinline__ void write_back(const SegPlan& p, const K* sOut, const uint32_t* sIdx,
                                           K* out, uint32_t* out_pay) {
    if (p.s == 0) return;
    write_out<K, L, RW>(sOut, p.offC, p.s, out + (p.c0 - p.offC));
    if (PAY) write_out<uint32_t, L, RW>(sIdx, p.offCP, p.s, out_pay + (p.c0 - p.offCP));
}

// LDS carve-up shared by the merge kernels.
template <typename K, bool PAY, int L>
struct SmemPtrs {
    K* sKey;
    uint32_t* sPay;
    K* sOut;
    uint32_t* sIdx;
    int* sXb;
    int* sYb;
    __device__ SmemPtrs(char* smem, uint32_t cap) {
        using M = MergeSmem<K, PAY, L>;
        char* p = smem;
        sKey = reinterpret_cast<K*>(p);
        p += M::key_slots(cap) * sizeof(K);
        sOut = reinterpret_cast<K*>(p);
        p += M::out_slots(cap) * sizeof(K);
        sPay = nullptr;
        sIdx = nullptr;
        if (PAY) {
            sPay = reinterpret_cast<uint32_t*>(p);
            p += M::pay_slots(cap) * 4;
            sIdx = reinterpret_cast<uint32_t*>(p);
            p += M::out_slots(cap) * 4;
        }
        sXb = reinterpret_cast<int*>(p);
        sYb = sXb + (L + 1);
    }
};

// A descriptor is usable if it lies inside the arrays and fits the LDS.
__device__ __forceinline__ bool desc_ok(const PieceDesc& d, int64_t nkeys, int64_t nout,
                                        uint32_t cap) {
    const int64_t a = piece_a(d), b = piece_b(d);
    return a + b <= (int64_t)cap && d.ka0 >= 0 && d.ka0 + a <= nkeys && d.kb0 >= 0 &&
           d.kb0 + b <= nkeys && d.out0 >= 0 && d.out0 + a + b <= nout;
}

}  // namespace sm
