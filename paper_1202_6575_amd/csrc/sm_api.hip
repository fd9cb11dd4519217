// sm_api.hip -- the C ABI of libstablemerge.so (declared in include/stablemerge.h).
//
// Host-side argument checks, workspace layouts and launch sequences.
// Plain merge: Steps 1-2 (partition kernel), the single synchronisation
// (the kernel boundary), Steps 3-4 (case selection, then the merges).  When
// forced block counts make subproblems larger than one workgroup stages,
// each subproblem becomes a job of the batch engine, which splits it again
// by the same method (a stable merge of a subproblem is the subproblem's
// part of the stable merge, Observation 1).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "stablemerge.h"
#include "sm_batch.h"
#include "sm_device.h"
#include "sm_launch.h"
#include "sm_sort.h"
#include "sm_learned.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t key_bytes(int dtype) { return sm::dtype_bytes(dtype); }

bool dtype_ok(int dtype) { return sm::dtype_known(dtype); }

// sm_options.reserved must be zero (room for later options).
bool options_ok(const sm_options* opt) {
    if (!opt) return true;
    for (int32_t r : opt->reserved)
        if (r != 0) return false;
    return true;
}

// The kernel dtype code: the public code plus the requested order.
int kernel_dtype(int dtype, const sm_options* opt) {
    return sm::kernel_dtype(dtype, opt && opt->descending);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

bool overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Block length in elements when none is given: a subproblem then holds up to
// twice this, and one merge workgroup stages it in LDS.  Keys only, and 64-bit
// keys with payloads: the largest length (measured on MI355X) at which four
// merge workgroups still share a compute unit's 160 KiB of LDS.  32-bit keys
// with payloads: 1408, three workgroups per compute unit, which measured
// faster than 1152 (four per unit) in merges and in the sort's passes.
int32_t default_tile(int dtype, bool pay) {
    if (key_bytes(dtype) == 8) return pay ? 1024 : 1152;
    return pay ? 1408 : 2368;
}

int32_t pick_tile(int dtype, bool pay, const sm_options* opt) {
    return opt && opt->tile != 0 ? opt->tile : default_tile(dtype, pay);
}

int check_tile(int dtype, bool pay, int32_t tile) {
    if (tile < 1 || tile > (1 << 16)) return fail(SM_ERR_ARG, "tile must be in [1, 65536]");
    if (sm::merge_lds_bytes(dtype, pay, sm::merge_cap_for_tile(tile)) > sm::kMaxLds)
        return fail(SM_ERR_ARG, "tile %d is too large for one workgroup's LDS", tile);
    return SM_OK;
}

// Workspace of stable_merge: xbar[p_a+1] and ybar[p_b+1] (int64), a status
// word, p_a + p_b subproblem descriptors, and when the subproblems are
// merged as jobs, the batch engine's workspace.  stable_merge_pieces uses the
// part from the descriptors on.
size_t ranks_bytes(int64_t pa, int64_t pb) { return align256((size_t)(pa + 1 + pb + 1) * 8); }

struct Plan {
    int64_t p_a, p_b;
    int32_t tile;
    uint32_t cap;  // capacity (elements) of one merge workgroup's subproblem
    bool hier;     // subproblems exceed cap: merge them as jobs of the engine
    sm::BatchLayout layout;
    size_t off_flag, off_desc, off_batch, ws_bytes;
};

int check_sizes(int64_t n, int64_t m, int dtype) {
    if (n < 0 || m < 0)
        return fail(SM_ERR_ARG, "n and m must be >= 0 (n=%lld, m=%lld)", (long long)n, (long long)m);
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if ((uint64_t)(n + m) > (1ull << 40)) return fail(SM_ERR_ARG, "n + m too large");
    return SM_OK;
}

// Block counts, subproblem capacity and workspace layout of one merge.
int make_plan(int64_t n, int64_t m, int dtype, bool pay, int64_t pa, int64_t pb, int32_t tile,
              Plan* pl) {
    int rc = check_sizes(n, m, dtype);
    if (rc != SM_OK) return rc;
    if (pa < 0 || pb < 0) return fail(SM_ERR_ARG, "p_a and p_b must be >= 0");
    rc = check_tile(dtype, pay, tile);
    if (rc != SM_OK) return rc;
    if (pa == 0) pa = n > 0 ? (n + tile - 1) / tile : 1;
    if (pb == 0) pb = m > 0 ? (m + tile - 1) / tile : 1;
    if (pa > (1ll << 31) - 2 || pb > (1ll << 31) - 2 || pa + pb > (1ll << 31) - 2)
        return fail(SM_ERR_ARG, "too many blocks (p_a=%lld, p_b=%lld)", (long long)pa,
                    (long long)pb);
    // a subproblem holds at most one block of A and one block of B
    const int64_t la = (n + pa - 1) / pa, lb = (m + pb - 1) / pb;
    if (la >= (1ll << 30) || lb >= (1ll << 30))
        return fail(SM_ERR_ARG, "blocks of 2^30 or more elements; use more blocks");
    // subproblems that one workgroup stages are merged directly, larger ones
    // are split again with blocks of `tile` elements
    const int64_t sub = la + lb > 0 ? la + lb : 1;
    pl->p_a = pa;
    pl->p_b = pb;
    pl->tile = tile;
    pl->hier = sub >= (1 << 20) || sm::merge_lds_bytes(dtype, pay, (uint32_t)sub) > sm::kMaxLds;
    pl->cap = pl->hier ? sm::merge_cap_for_tile(tile) : (uint32_t)sub;
    size_t off = ranks_bytes(pa, pb);
    pl->off_flag = off;
    off += 256;
    pl->off_desc = off;
    off += align256((size_t)(pa + pb) * sm::kPieceDescBytes);
    pl->off_batch = off;
    if (pl->hier) {
        pl->layout = sm::batch_layout(pa + pb, n + m, tile);
        if (pl->layout.p_max > (1ll << 31) - 2)
            return fail(SM_ERR_ARG, "too many second-level subproblems; use a larger tile");
        off += pl->layout.bytes;
    }
    pl->ws_bytes = off;
    return SM_OK;
}

// Checks shared by the entry points that write a merged array.
int check_buffers(const void* keys, const uint32_t* payloads, int64_t total, void* out_keys,
                  uint32_t* out_payloads, int dtype) {
    const bool pay = payloads != nullptr;
    if ((payloads == nullptr) != (out_payloads == nullptr))
        return fail(SM_ERR_ARG, "payloads and out_payloads must both be NULL or both non-NULL");
    if (!keys || !out_keys) return fail(SM_ERR_ARG, "keys and out_keys must not be NULL");
    if (!aligned16(keys) || !aligned16(out_keys) ||
        (pay && (!aligned16(payloads) || !aligned16(out_payloads))))
        return fail(SM_ERR_ARG, "device arrays must be 16-byte aligned");
    const size_t kb = (size_t)total * key_bytes(dtype);
    if (overlap(out_keys, kb, keys, kb) ||
        (pay && (overlap(out_payloads, (size_t)total * 4, payloads, (size_t)total * 4) ||
                 overlap(out_payloads, (size_t)total * 4, keys, kb) ||
                 overlap(out_keys, kb, payloads, (size_t)total * 4))))
        return fail(SM_ERR_ALIAS, "outputs overlap inputs; C must be a separate array");
    return SM_OK;
}

int check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (!ws || ws_bytes < need)
        return fail(SM_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws ? ws_bytes : (size_t)0);
    if (!aligned16(ws)) return fail(SM_ERR_ARG, "workspace must be 16-byte aligned");
    return SM_OK;
}

// The workspace holds cross ranks and descriptors that the kernels write
// while reading the inputs and writing the outputs: it must not share a byte
// with any of the caller's arrays.
int check_ws_alias(const void* ws, size_t need, const void* keys, const uint32_t* payloads,
                   int64_t total, const void* out_keys, const uint32_t* out_payloads, int dtype,
                   const void* extra0 = nullptr, size_t extra0_bytes = 0,
                   const void* extra1 = nullptr, size_t extra1_bytes = 0) {
    const size_t kb = (size_t)total * key_bytes(dtype), pb = (size_t)total * 4;
    if (overlap(ws, need, keys, kb) || overlap(ws, need, out_keys, kb) ||
        overlap(ws, need, payloads, payloads ? pb : 0) ||
        overlap(ws, need, out_payloads, out_payloads ? pb : 0) ||
        overlap(ws, need, extra0, extra0_bytes) || overlap(ws, need, extra1, extra1_bytes))
        return fail(SM_ERR_ALIAS, "workspace overlaps an input or output array");
    return SM_OK;
}

// Steps 3-4 and the merges, once Steps 1-2 have written xbar / ybar.
// `tail` is the workspace from the descriptors on; dtype is a kernel code.
int cases_and_merge(const Plan& pl, int dtype, const void* keys, const uint32_t* payloads,
                    int64_t n, int64_t m, const int64_t* xbar, const int64_t* ybar,
                    void* out_keys, uint32_t* out_payloads, char* tail, hipStream_t st) {
    sm::PieceDesc* desc = reinterpret_cast<sm::PieceDesc*>(tail);
    const int64_t P = pl.p_a + pl.p_b;
    hipError_t e;
    // the small-block merge has an ascending form only
    if (!pl.hier && pl.cap <= sm::kFineCap && !(dtype & sm::kDescending)) {
        e = sm::launch_fine_merge(dtype, keys, payloads, n, m, pl.p_a, pl.p_b, xbar, ybar, out_keys,
                                  out_payloads, st);
        if (e != hipSuccess) return hip_fail(e, "merge launch");
        return SM_OK;
    }
    // a few large subproblems: Steps 3-4 inside the merge workgroups
    if (!pl.hier && sm::merge_cases_direct_applies(dtype, payloads != nullptr, pl.cap, P)) {
        e = sm::launch_merge_cases_direct(dtype, keys, payloads, n, m, pl.p_a, pl.p_b, xbar, ybar,
                                          out_keys, out_payloads, pl.cap, st);
        if (e != hipSuccess) return hip_fail(e, "merge launch");
        return SM_OK;
    }
    e = sm::launch_cases(n, m, pl.p_a, pl.p_b, xbar, ybar, desc, st);
    if (e != hipSuccess) return hip_fail(e, "cases launch");
    if (!pl.hier)
        e = sm::launch_merge_desc(dtype, keys, payloads, n + m, out_keys, out_payloads, n + m, desc,
                                  P, nullptr, sm::merge_pack_cap(dtype, payloads != nullptr, pl.cap),
                                  st, /*packed=*/true);
    else
        e = sm::launch_batch(dtype, keys, payloads, n + m, out_keys, out_payloads, n + m, desc, P,
                             pl.tile, tail + (pl.off_batch - pl.off_desc), pl.layout, st);
    if (e != hipSuccess) return hip_fail(e, "merge launch");
    return SM_OK;
}

// Steps 1-4 of one merge once its plan and buffers have been checked; `w`
// is device memory of at least pl.ws_bytes bytes, in any state (every
// kernel writes what it later reads).
int merge_run(const Plan& pl, const void* keys, const uint32_t* payloads, int64_t n, int64_t m,
              void* out_keys, uint32_t* out_payloads, int dtype, char* w, const sm_options* opt,
              hipStream_t st) {
    int64_t* xbar = reinterpret_cast<int64_t*>(w);
    int64_t* ybar = xbar + (pl.p_a + 1);
    int* flag = reinterpret_cast<int*>(w + pl.off_flag);
    hipError_t e;

    const int kd = kernel_dtype(dtype, opt);
    if (opt && opt->validate) {
        int host_flag = 0;
        e = sm::launch_clear(flag, 1, st);
        if (e == hipSuccess) e = sm::launch_validate(kd, keys, n, m, flag, st);
        if (e != hipSuccess) return hip_fail(e, "validate launch");
        e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "validate readback");
        if (host_flag) return fail(SM_ERR_UNSORTED, "A or B is not sorted in the requested order");
    }

    e = sm::launch_partition(kd, keys, n, m, pl.p_a, pl.p_b, xbar, ybar, st);
    if (e != hipSuccess) return hip_fail(e, "partition launch");
    return cases_and_merge(pl, kd, keys, payloads, n, m, xbar, ybar, out_keys, out_payloads,
                           w + pl.off_desc, st);
}

// The scratch memory of stable_merge_noalloc: one copy per device, held from
// the library's first use on that device until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device memory: every
// host use goes through the device address that hipGetSymbolAddress returns
// for the current device, looked up once per device and kept.
}  // namespace

static __device__ __align__(256) char scratch[SM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(SM_ERR_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) & 255))
            return fail(SM_ERR_HIP, "scratch address is null or misaligned");
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return SM_OK;
}

}  // namespace

extern "C" {

const char* sm_last_error(void) { return g_err; }

int sm_version(void) { return 200; }

size_t stable_merge_workspace_bytes(int64_t n, int64_t m, int dtype, int has_payload,
                                    const sm_options* opt) {
    Plan pl;
    if (!dtype_ok(dtype) || !options_ok(opt)) return 0;
    const bool pay = has_payload != 0;
    if (make_plan(n, m, dtype, pay, opt ? opt->p_a : 0, opt ? opt->p_b : 0,
                  pick_tile(dtype, pay, opt), &pl) != SM_OK)
        return 0;
    return pl.ws_bytes;
}

int stable_merge_partition(const void* keys, int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                           int dtype, int64_t* xbar, int64_t* ybar, void* stream) {
    int rc = check_sizes(n, m, dtype);
    if (rc != SM_OK) return rc;
    if (p_a < 1 || p_b < 1) return fail(SM_ERR_ARG, "p_a and p_b must be >= 1");
    if (p_a + p_b > (1ll << 40)) return fail(SM_ERR_ARG, "too many blocks");
    if (!xbar || !ybar) return fail(SM_ERR_ARG, "xbar and ybar must not be NULL");
    if (n + m > 0 && !keys) return fail(SM_ERR_ARG, "keys must not be NULL");
    if (reinterpret_cast<uintptr_t>(keys) % key_bytes(dtype))
        return fail(SM_ERR_ARG, "keys misaligned");
    hipError_t e = sm::launch_partition(dtype, keys, n, m, p_a, p_b, xbar, ybar,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "partition launch");
    return SM_OK;
}

size_t stable_merge_pieces_workspace_bytes(int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                                           int dtype, int has_payload) {
    Plan pl;
    if (!dtype_ok(dtype) || p_a < 1 || p_b < 1) return 0;
    const bool pay = has_payload != 0;
    if (make_plan(n, m, dtype, pay, p_a, p_b, default_tile(dtype, pay), &pl) != SM_OK) return 0;
    return pl.ws_bytes - pl.off_desc;
}

int stable_merge_pieces(const void* keys, const uint32_t* payloads, int64_t n, int64_t m,
                        int64_t p_a, int64_t p_b, const int64_t* xbar, const int64_t* ybar,
                        void* out_keys, uint32_t* out_payloads, int dtype, void* ws,
                        size_t ws_bytes, void* stream) {
    if (p_a < 1 || p_b < 1) return fail(SM_ERR_ARG, "p_a and p_b must be >= 1");
    const bool pay = payloads != nullptr;
    Plan pl;
    int rc = make_plan(n, m, dtype, pay, p_a, p_b, default_tile(dtype, pay), &pl);
    if (rc != SM_OK) return rc;
    if (n + m == 0) return SM_OK;
    if (!xbar || !ybar) return fail(SM_ERR_ARG, "xbar and ybar must not be NULL");
    rc = check_buffers(keys, payloads, n + m, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    rc = check_ws(ws, ws_bytes, pl.ws_bytes - pl.off_desc);
    if (rc != SM_OK) return rc;
    rc = check_ws_alias(ws, pl.ws_bytes - pl.off_desc, keys, payloads, n + m, out_keys,
                        out_payloads, dtype, xbar, (size_t)(p_a + 1) * 8, ybar,
                        (size_t)(p_b + 1) * 8);
    if (rc != SM_OK) return rc;
    return cases_and_merge(pl, dtype, keys, payloads, n, m, xbar, ybar, out_keys, out_payloads,
                           static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

int stable_merge(const void* keys, const uint32_t* payloads, int64_t n, int64_t m, void* out_keys,
                 uint32_t* out_payloads, int dtype, void* ws, size_t ws_bytes,
                 const sm_options* opt, void* stream) {
    const bool pay = payloads != nullptr;
    if (!options_ok(opt)) return fail(SM_ERR_ARG, "sm_options.reserved must be zero");
    Plan pl;
    int rc = make_plan(n, m, dtype, pay, opt ? opt->p_a : 0, opt ? opt->p_b : 0,
                       pick_tile(dtype, pay, opt), &pl);
    if (rc != SM_OK) return rc;
    const int64_t total = n + m;
    if (total == 0) return SM_OK;
    rc = check_buffers(keys, payloads, total, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    rc = check_ws(ws, ws_bytes, pl.ws_bytes);
    if (rc != SM_OK) return rc;
    rc = check_ws_alias(ws, pl.ws_bytes, keys, payloads, total, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    return merge_run(pl, keys, payloads, n, m, out_keys, out_payloads, dtype,
                     static_cast<char*>(ws), opt, static_cast<hipStream_t>(stream));
}

int stable_merge_noalloc(const void* keys, const uint32_t* payloads, int64_t n, int64_t m,
                         void* out_keys, uint32_t* out_payloads, int dtype,
                         const sm_options* opt, void* stream) {
    const bool pay = payloads != nullptr;
    if (!options_ok(opt)) return fail(SM_ERR_ARG, "sm_options.reserved must be zero");
    if (opt && opt->validate)
        return fail(SM_ERR_ARG, "validate reads a status word back to the host; "
                                "stable_merge_noalloc does not offer it");
    Plan pl;
    int rc = make_plan(n, m, dtype, pay, opt ? opt->p_a : 0, opt ? opt->p_b : 0,
                       pick_tile(dtype, pay, opt), &pl);
    if (rc != SM_OK) return rc;
    const int64_t total = n + m;
    if (total == 0) return SM_OK;
    rc = check_buffers(keys, payloads, total, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    if (pl.ws_bytes > (size_t)SM_NOALLOC_SCRATCH_BYTES)
        return fail(SM_ERR_WORKSPACE,
                    "this merge needs %zu bytes of scratch, above the built-in %zu; "
                    "use stable_merge with a workspace, or a larger tile",
                    pl.ws_bytes, (size_t)SM_NOALLOC_SCRATCH_BYTES);
    char* w = nullptr;
    rc = scratch_on_current_device(&w);
    if (rc != SM_OK) return rc;
    return merge_run(pl, keys, payloads, n, m, out_keys, out_payloads, dtype, w, opt,
                     static_cast<hipStream_t>(stream));
}

size_t stable_merge_batched_workspace_bytes(int64_t count, int64_t total, int dtype,
                                            int has_payload, const sm_options* opt) {
    if (!dtype_ok(dtype) || !options_ok(opt) || count < 0 || total < 0 || total > (1ll << 40))
        return 0;
    const bool pay = has_payload != 0;
    const int32_t tile = pick_tile(dtype, pay, opt);
    if (check_tile(dtype, pay, tile) != SM_OK) return 0;
    const sm::BatchLayout L = sm::batch_layout(count, total, tile);
    return align256((size_t)count * sm::kPieceDescBytes) + L.bytes;
}

int stable_merge_batched(const void* keys, const uint32_t* payloads, const int64_t* offsets,
                         const int64_t* n_a, int64_t count, int64_t total, void* out_keys,
                         uint32_t* out_payloads, int dtype, void* ws, size_t ws_bytes,
                         const sm_options* opt, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (count < 0 || total < 0 || total > (1ll << 40))
        return fail(SM_ERR_ARG, "count and total must be >= 0 (count=%lld, total=%lld)",
                    (long long)count, (long long)total);
    if (count > (1ll << 31) - 2) return fail(SM_ERR_ARG, "too many pairs");
    if (!options_ok(opt)) return fail(SM_ERR_ARG, "sm_options.reserved must be zero");
    const bool pay = payloads != nullptr;
    const int32_t tile = pick_tile(dtype, pay, opt);
    int rc = check_tile(dtype, pay, tile);
    if (rc != SM_OK) return rc;
    if (count == 0 || total == 0) return SM_OK;
    if (!offsets || !n_a) return fail(SM_ERR_ARG, "offsets and n_a must not be NULL");
    rc = check_buffers(keys, payloads, total, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    const sm::BatchLayout L = sm::batch_layout(count, total, tile);
    if (L.p_max > (1ll << 31) - 2)
        return fail(SM_ERR_ARG, "too many subproblems for one launch; use a larger tile");
    const size_t off_eng = align256((size_t)count * sm::kPieceDescBytes);
    rc = check_ws(ws, ws_bytes, off_eng + L.bytes);
    if (rc != SM_OK) return rc;
    rc = check_ws_alias(ws, off_eng + L.bytes, keys, payloads, total, out_keys, out_payloads,
                        dtype, offsets, (size_t)(count + 1) * 8, n_a, (size_t)count * 8);
    if (rc != SM_OK) return rc;

    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    sm::PieceDesc* jobs = reinterpret_cast<sm::PieceDesc*>(w);
    int* flag = reinterpret_cast<int*>(w + off_eng + L.off_flag);
    hipError_t e = sm::launch_clear(flag, 1, st);
    if (e == hipSuccess) e = sm::launch_jobs_from_pairs(offsets, n_a, count, total, jobs, flag, st);
    if (e != hipSuccess) return hip_fail(e, "pair descriptor launch");
    if (opt && opt->validate) {
        int host_flag = 0;
        e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "validate readback");
        if (host_flag) return fail(SM_ERR_ARG, "offsets / n_a describe an invalid pair");
        e = sm::launch_batch_validate(kernel_dtype(dtype, opt), keys, offsets, n_a, count, total,
                                      flag, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "validate readback");
        if (host_flag)
            return fail(SM_ERR_UNSORTED, "an A or B of the batch is not sorted in the requested order");
    }
    e = sm::launch_batch(kernel_dtype(dtype, opt), keys, payloads, total, out_keys, out_payloads,
                         total, jobs, count, tile, w + off_eng, L, st);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return SM_OK;
}

namespace {

int sort_plan(int64_t N, int dtype, bool pay, const sm_options* opt, int* run, int32_t* tile,
              sm::SortLayout* L, int64_t seg_count = 0, int64_t max_len = 0) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (N < 0 || N >= (1ll << 31)) return fail(SM_ERR_ARG, "N must be in [0, 2^31)");
    if (!options_ok(opt)) return fail(SM_ERR_ARG, "sm_options.reserved must be zero");
    *run = opt && opt->run != 0 ? opt->run : 512;
    if (!sm::sort_run_ok(*run, dtype))
        return fail(SM_ERR_ARG, "run must be 256, 512, 1024, 2048 or (32-bit keys) 4096");
    *tile = pick_tile(dtype, pay, opt);
    int rc = check_tile(dtype, pay, *tile);
    if (rc != SM_OK) return rc;
    *L = sm::sort_layout(N, dtype, pay, *run, *tile, seg_count, max_len);
    if (L->batch.p_max > (1ll << 31) - 2)
        return fail(SM_ERR_ARG, "too many subproblems per pass; use a larger tile");
    return SM_OK;
}

}  // namespace

size_t stable_merge_sort_workspace_bytes(int64_t N, int dtype, int has_payload,
                                         const sm_options* opt) {
    int run;
    int32_t tile;
    sm::SortLayout L;
    if (sort_plan(N, dtype, has_payload != 0, opt, &run, &tile, &L) != SM_OK) return 0;
    return L.bytes;
}

namespace {

// Argument checks shared by the two sorts (after sort_plan).
int check_sort_arrays(const void* keys, const uint32_t* payloads, int64_t N, void* out_keys,
                      uint32_t* out_payloads, int dtype) {
    const bool pay = payloads != nullptr;
    if ((payloads == nullptr) != (out_payloads == nullptr))
        return fail(SM_ERR_ARG, "payloads and out_payloads must both be NULL or both non-NULL");
    if (!keys || !out_keys) return fail(SM_ERR_ARG, "keys and out_keys must not be NULL");
    if (!aligned16(keys) || !aligned16(out_keys) ||
        (pay && (!aligned16(payloads) || !aligned16(out_payloads))))
        return fail(SM_ERR_ARG, "device arrays must be 16-byte aligned");
    const size_t kb = (size_t)N * key_bytes(dtype), pb = (size_t)N * 4;
    // the same array in and out is an in-place sort; a partial overlap is not
    if ((out_keys != keys && overlap(out_keys, kb, keys, kb)) ||
        (pay && ((out_payloads != payloads && overlap(out_payloads, pb, payloads, pb)) ||
                 overlap(out_payloads, pb, keys, kb) || overlap(out_keys, kb, payloads, pb) ||
                 overlap(out_keys, kb, out_payloads, pb))))
        return fail(SM_ERR_ALIAS, "outputs overlap inputs other than in place");
    return SM_OK;
}

int check_sort_buffers(const void* keys, const uint32_t* payloads, int64_t N, void* out_keys,
                       uint32_t* out_payloads, int dtype, const void* ws, size_t ws_bytes,
                       size_t need) {
    const bool pay = payloads != nullptr;
    const size_t kb = (size_t)N * key_bytes(dtype), pb = (size_t)N * 4;
    int rc = check_sort_arrays(keys, payloads, N, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    rc = check_ws(ws, ws_bytes, need);
    if (rc != SM_OK) return rc;
    const char* w = static_cast<const char*>(ws);
    if (overlap(w, need, keys, kb) || overlap(w, need, out_keys, kb) ||
        (pay && (overlap(w, need, payloads, pb) || overlap(w, need, out_payloads, pb))))
        return fail(SM_ERR_ALIAS, "workspace overlaps the keys or payloads");
    return SM_OK;
}

// The segmented sort's workspace: the sort's, then one status word.
size_t seg_flag_offset(const sm::SortLayout& L) { return align256(L.bytes); }

}  // namespace

static int sort_impl(const void* keys, const uint32_t* payloads, int64_t N, void* out_keys,
                     uint32_t* out_payloads, int dtype, void* ws, size_t ws_bytes,
                     const sm_options* opt, void* stream, const sm::LearnedSearch* ls) {
    const bool pay = payloads != nullptr;
    int run;
    int32_t tile;
    sm::SortLayout L;
    int rc = sort_plan(N, dtype, pay, opt, &run, &tile, &L);
    if (rc != SM_OK) return rc;
    if ((payloads == nullptr) != (out_payloads == nullptr))
        return fail(SM_ERR_ARG, "payloads and out_payloads must both be NULL or both non-NULL");
    if (N == 0) return SM_OK;
    rc = check_sort_buffers(keys, payloads, N, out_keys, out_payloads, dtype, ws, ws_bytes,
                            L.bytes);
    if (rc != SM_OK) return rc;
    hipError_t e = sm::launch_sort(kernel_dtype(dtype, opt), keys, payloads, N, out_keys,
                                   out_payloads, run, tile, static_cast<char*>(ws), L,
                                   static_cast<hipStream_t>(stream), nullptr, 0, ls);
    if (e != hipSuccess) return hip_fail(e, "sort launch");
    return SM_OK;
}

int stable_merge_sort(const void* keys, const uint32_t* payloads, int64_t N, void* out_keys,
                      uint32_t* out_payloads, int dtype, void* ws, size_t ws_bytes,
                      const sm_options* opt, void* stream) {
    return sort_impl(keys, payloads, N, out_keys, out_payloads, dtype, ws, ws_bytes, opt, stream,
                     nullptr);
}

int stable_merge_sort_runs(const void* keys, const uint32_t* payloads, int64_t N,
                           void* out_keys, uint32_t* out_payloads, int dtype, int run,
                           void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (N < 0 || N > (1ll << 38)) return fail(SM_ERR_ARG, "N must be in [0, 2^38]");
    if (!sm::sort_run_ok(run, dtype))
        return fail(SM_ERR_ARG, "run must be 256, 512, 1024, 2048 or (32-bit keys) 4096");
    if (N == 0) return SM_OK;
    int rc = check_sort_arrays(keys, payloads, N, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    hipError_t e = sm::launch_sort_runs(dtype, keys, payloads, N, out_keys, out_payloads, run,
                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "run formation launch");
    return SM_OK;
}

int stable_merge_sort_learned(const void* keys, const uint32_t* payloads, int64_t N,
                              void* out_keys, uint32_t* out_payloads, int dtype,
                              const float* model, float step_frac, uint64_t* counters, void* ws,
                              size_t ws_bytes, const sm_options* opt, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (!model) return fail(SM_ERR_ARG, "model must not be NULL");
    if (!(step_frac >= 0.0f && step_frac <= 1.0f))
        return fail(SM_ERR_ARG, "step_frac must be in [0, 1]");
    if (opt && opt->descending)
        return fail(SM_ERR_ARG, "the learned sort is ascending only");
    const sm::LearnedSearch ls{model, step_frac,
                               reinterpret_cast<unsigned long long*>(counters)};
    return sort_impl(keys, payloads, N, out_keys, out_payloads, dtype, ws, ws_bytes, opt, stream,
                     &ls);
}

size_t stable_merge_segmented_sort_workspace_bytes(int64_t count, int64_t N, int64_t max_len,
                                                   int dtype, int has_payload,
                                                   const sm_options* opt) {
    int run;
    int32_t tile;
    sm::SortLayout L;
    if (count < 1 || max_len < 0 || max_len > N) return 0;
    if (sort_plan(N, dtype, has_payload != 0, opt, &run, &tile, &L, count, max_len) != SM_OK)
        return 0;
    return seg_flag_offset(L) + 256;
}

int stable_merge_segmented_sort(const void* keys, const uint32_t* payloads,
                                const int64_t* offsets, int64_t count, int64_t N,
                                int64_t max_len, void* out_keys, uint32_t* out_payloads,
                                int dtype, void* ws, size_t ws_bytes, const sm_options* opt,
                                void* stream) {
    const bool pay = payloads != nullptr;
    if (count < 1) return fail(SM_ERR_ARG, "count must be >= 1");
    if (count > (1ll << 31)) return fail(SM_ERR_ARG, "count must be below 2^31");
    if (max_len < 0 || max_len > N) return fail(SM_ERR_ARG, "0 <= max_len <= N required");
    int run;
    int32_t tile;
    sm::SortLayout L;
    int rc = sort_plan(N, dtype, pay, opt, &run, &tile, &L, count, max_len);
    if (rc != SM_OK) return rc;
    if ((payloads == nullptr) != (out_payloads == nullptr))
        return fail(SM_ERR_ARG, "payloads and out_payloads must both be NULL or both non-NULL");
    if (!offsets) return fail(SM_ERR_ARG, "offsets must not be NULL");
    if (N == 0) return SM_OK;
    const size_t need = seg_flag_offset(L) + 256;
    rc = check_sort_buffers(keys, payloads, N, out_keys, out_payloads, dtype, ws, ws_bytes, need);
    if (rc != SM_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (opt && opt->validate) {
        int* flag = reinterpret_cast<int*>(static_cast<char*>(ws) + seg_flag_offset(L));
        int host_flag = 0;
        hipError_t e = sm::launch_clear(flag, 1, st);
        if (e == hipSuccess) e = sm::launch_seg_check(offsets, count, N, max_len, flag, st);
        if (e == hipSuccess) e = hipMemcpyAsync(&host_flag, flag, sizeof(int),
                                                hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "segment check");
        if (host_flag)
            return fail(SM_ERR_ARG, "offsets must run from 0 to N without decreasing, with no "
                                    "segment longer than max_len");
    }
    hipError_t e = sm::launch_sort(kernel_dtype(dtype, opt), keys, payloads, N, out_keys,
                                   out_payloads, run, tile, static_cast<char*>(ws), L, st, offsets,
                                   count);
    if (e != hipSuccess) return hip_fail(e, "segmented sort launch");
    return SM_OK;
}

size_t sm_mlp_grad_workspace_bytes(int64_t samples) {
    return samples < 0 ? 0 : sm::mlp_grad_ws_bytes(samples);
}

int sm_mlp_grad(const float* params, const void* keys, const float* target, int64_t samples,
                int dtype, float* grad, float* loss, void* ws, size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (samples < 1 || samples > (1ll << 34)) return fail(SM_ERR_ARG, "samples must be in [1, 2^34]");
    if (!params || !keys || !target || !grad) return fail(SM_ERR_ARG, "NULL pointer");
    int rc = check_ws(ws, ws_bytes, sm::mlp_grad_ws_bytes(samples));
    if (rc != SM_OK) return rc;
    hipError_t e = sm::launch_mlp_grad(dtype, params, keys, target, samples, grad, loss, ws,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SM_OK : hip_fail(e, "mlp grad launch");
}

int sm_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step, float lr,
                float beta1, float beta2, float eps, void* stream) {
    if (!params || !m || !v || !grad) return fail(SM_ERR_ARG, "NULL pointer");
    if (step < 1) return fail(SM_ERR_ARG, "step must be >= 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
        return fail(SM_ERR_ARG, "need 0 <= beta1, beta2 < 1 and eps > 0");
    hipError_t e = sm::launch_mlp_adam(params, m, v, grad, step, lr, beta1, beta2, eps,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SM_OK : hip_fail(e, "adam launch");
}

int sm_mlp_init(const void* sorted_keys, const float* target, int64_t samples, int dtype,
                float* params, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (samples < 0 || (samples > 0 && (!sorted_keys || !target)) || !params)
        return fail(SM_ERR_ARG, "bad sample or NULL pointer");
    hipError_t e = sm::launch_mlp_init(dtype, sorted_keys, target, samples, params,
                                       static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SM_OK : hip_fail(e, "init launch");
}

int sm_mlp_predict(const float* params, const void* keys, int64_t q, int dtype, int64_t len,
                   int64_t* rhat, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (q < 0 || len < 0 || len > (1ll << 40)) return fail(SM_ERR_ARG, "bad sizes");
    if (q > 0 && (!params || !keys || !rhat)) return fail(SM_ERR_ARG, "NULL pointer");
    hipError_t e = sm::launch_mlp_predict(dtype, params, keys, q, len, rhat,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SM_OK : hip_fail(e, "predict launch");
}

size_t sm_rank_model_workspace_bytes(int64_t samples, int dtype) {
    if (!dtype_ok(dtype) || samples < 1 || samples > (1ll << 34)) return 0;
    return sm::rank_model_layout(samples, dtype).bytes;
}

int sm_rank_model_train(const void* X, int64_t len, const void* Q, int64_t q_len, int dtype,
                        int is_high, int64_t samples, int64_t steps, float lr, uint64_t seed,
                        float* params, float* loss, void* ws, size_t ws_bytes, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (len < 1 || q_len < 1 || len > (1ll << 40) || q_len > (1ll << 40))
        return fail(SM_ERR_ARG, "the searched and the query arrays must be non-empty");
    if (samples < 1 || samples > (1ll << 34) || steps < 0 || !(lr > 0.0f))
        return fail(SM_ERR_ARG, "samples >= 1, steps >= 0 and lr > 0 required");
    if (!X || !Q || !params) return fail(SM_ERR_ARG, "NULL pointer");
    const sm::RankModelLayout L = sm::rank_model_layout(samples, dtype);
    int rc = check_ws(ws, ws_bytes, L.bytes);
    if (rc != SM_OK) return rc;
    hipError_t e = sm::launch_rank_model_train(dtype, X, len, Q, q_len, is_high != 0, samples, steps,
                                               lr, seed, params, loss, static_cast<char*>(ws), L,
                                               static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SM_OK : hip_fail(e, "training launch");
}

int stable_merge_rank_search(const void* X, int64_t len, const void* queries, int64_t q, int dtype,
                             int is_high, const int64_t* guess, int64_t step0, int64_t window,
                             int64_t* ranks, int32_t* probes, int32_t* fallback, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (len < 0 || q < 0 || len > (1ll << 40)) return fail(SM_ERR_ARG, "bad sizes");
    if (step0 < 1 || window < 0 || window > (1ll << 40))
        return fail(SM_ERR_ARG, "step0 >= 1 and 0 <= window <= 2^40 required");
    if (q > 0 && (!queries || !guess || !ranks || (len > 0 && !X)))
        return fail(SM_ERR_ARG, "NULL pointer");
    hipError_t e = sm::launch_rank_search(dtype, X, len, queries, q, is_high != 0, guess, step0,
                                          window, ranks, probes, fallback,
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SM_OK : hip_fail(e, "search launch");
}

int stable_merge_partition_learned(const void* keys, int64_t n, int64_t m, int64_t p_a,
                                   int64_t p_b, int dtype, const float* model_b,
                                   const float* model_a, int64_t step0_a, int64_t step0_b,
                                   int64_t window, int64_t* xbar, int64_t* ybar, uint64_t* hist,
                                   uint64_t* counters, void* stream) {
    int rc = check_sizes(n, m, dtype);
    if (rc != SM_OK) return rc;
    if (p_a < 1 || p_b < 1 || p_a + p_b > (1ll << 40)) return fail(SM_ERR_ARG, "bad block counts");
    if (step0_a < 1 || step0_b < 1 || window < 0 || window > (1ll << 40))
        return fail(SM_ERR_ARG, "step0 >= 1 and 0 <= window <= 2^40 required");
    if (!xbar || !ybar || !hist || !counters || !model_a || !model_b)
        return fail(SM_ERR_ARG, "NULL pointer");
    if (n + m > 0 && !keys) return fail(SM_ERR_ARG, "keys must not be NULL");
    if (reinterpret_cast<uintptr_t>(keys) % key_bytes(dtype))
        return fail(SM_ERR_ARG, "keys misaligned");
    hipError_t e = sm::launch_learned_partition(dtype, keys, n, m, p_a, p_b, model_b, model_a,
                                                step0_a, step0_b, window, xbar, ybar, hist,
                                                counters, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SM_OK : hip_fail(e, "learned partition launch");
}

size_t stable_merge_learned_workspace_bytes(int64_t n, int64_t m, int64_t block, int dtype,
                                            int has_payload) {
    if (!dtype_ok(dtype) || n < 0 || m < 0 || block < 1 || block > (1ll << 20)) return 0;
    const int64_t p_a = n > 0 ? (n + block - 1) / block : 1;
    const int64_t p_b = m > 0 ? (m + block - 1) / block : 1;
    const size_t merge_ws = stable_merge_pieces_workspace_bytes(n, m, p_a, p_b, dtype, has_payload);
    if (merge_ws == 0 && n + m > 0) return 0;
    return ranks_bytes(p_a, p_b) + merge_ws;
}

int stable_merge_learned(const void* keys, const uint32_t* payloads, int64_t n, int64_t m,
                         void* out_keys, uint32_t* out_payloads, int dtype, const float* model_b,
                         const float* model_a, int64_t step0_a, int64_t step0_b, int64_t block,
                         int64_t window, uint64_t* hist, uint64_t* counters, void* ws,
                         size_t ws_bytes, void* stream) {
    int rc = check_sizes(n, m, dtype);
    if (rc != SM_OK) return rc;
    if (block < 1 || block > (1ll << 20)) return fail(SM_ERR_ARG, "1 <= block <= 2^20 required");
    if (n + m == 0) return SM_OK;
    rc = check_buffers(keys, payloads, n + m, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    const size_t need = stable_merge_learned_workspace_bytes(n, m, block, dtype, payloads != nullptr);
    if (need == 0) return fail(SM_ERR_ARG, "sizes not supported");
    rc = check_ws(ws, ws_bytes, need);
    if (rc != SM_OK) return rc;
    rc = check_ws_alias(ws, need, keys, payloads, n + m, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    const int64_t p_a = n > 0 ? (n + block - 1) / block : 1;
    const int64_t p_b = m > 0 ? (m + block - 1) / block : 1;
    int64_t* xbar = static_cast<int64_t*>(ws);
    int64_t* ybar = xbar + (p_a + 1);
    const size_t off = ranks_bytes(p_a, p_b);
    rc = stable_merge_partition_learned(keys, n, m, p_a, p_b, dtype, model_b, model_a, step0_a,
                                        step0_b, window, xbar, ybar, hist, counters, stream);
    if (rc != SM_OK) return rc;
    return stable_merge_pieces(keys, payloads, n, m, p_a, p_b, xbar, ybar, out_keys, out_payloads,
                               dtype, static_cast<char*>(ws) + off, ws_bytes - off, stream);
}

// ---------------------------------------------------------------------------
// Rank-model handles: a trained network together with what it was trained
// for (key type, which rank, feature kind), so that it can be kept, saved
// and loaded as a unit.  The parameters live in 98 device floats owned by
// the handle: the 97 parameters, then the last training loss.
// ---------------------------------------------------------------------------
}  // extern "C"

struct sm_predictor {
    uint32_t magic;
    int dtype;
    int is_high;
    int device;
    int64_t trained_len;
    float* dev;            // 97 parameters, then the loss
    hipStream_t stream;    // stream of the last training run
};

namespace {

constexpr uint32_t kPredMagic = 0x4D524D53u;   // "SMRM" read little-endian
constexpr uint32_t kBlobVersion = 1;
constexpr int32_t kFeatureLog2 = 1;            // phi = log2(u + 1) / bits
constexpr size_t kBlobParamsOff = 40;
constexpr size_t kBlobChecksumOff = kBlobParamsOff + 4 * SM_MLP_PARAMS;
static_assert(kBlobChecksumOff + 4 == SM_PREDICTOR_BLOB_BYTES, "blob layout");

uint32_t fnv1a(const unsigned char* b, size_t n) {
    uint32_t h = 2166136261u;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 16777619u;
    }
    return h;
}

template <typename T>
void put(unsigned char* b, size_t off, T v) { memcpy(b + off, &v, sizeof v); }
template <typename T>
T get(const unsigned char* b, size_t off) {
    T v;
    memcpy(&v, b + off, sizeof v);
    return v;
}

bool pred_ok(const sm_predictor* p) { return p && p->magic == kPredMagic && p->dev; }

int pred_new(sm_predictor** out, int dtype, int is_high, int64_t trained_len,
             const float* host_vals) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    float* d = nullptr;
    e = hipMalloc(&d, (SM_MLP_PARAMS + 1) * sizeof(float));
    if (e != hipSuccess) return hip_fail(e, "predictor allocation");
    e = hipMemcpy(d, host_vals, (SM_MLP_PARAMS + 1) * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return hip_fail(e, "predictor upload");
    }
    sm_predictor* p = new (std::nothrow) sm_predictor;
    if (!p) {
        (void)hipFree(d);
        return fail(SM_ERR_ARG, "out of host memory");
    }
    p->magic = kPredMagic;
    p->dtype = dtype;
    p->is_high = is_high;
    p->device = dev;
    p->trained_len = trained_len;
    p->dev = d;
    p->stream = nullptr;
    *out = p;
    return SM_OK;
}

// Wait for the last training run, then copy the parameters and the loss.
int pred_download(const sm_predictor* p, float* host_vals) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e == hipSuccess)
        e = hipMemcpy(host_vals, p->dev, (SM_MLP_PARAMS + 1) * sizeof(float),
                      hipMemcpyDeviceToHost);
    return e == hipSuccess ? SM_OK : hip_fail(e, "predictor download");
}

}  // namespace

extern "C" {

int sm_predictor_create(sm_predictor** out, int dtype, int is_high) {
    if (!out) return fail(SM_ERR_ARG, "out must not be NULL");
    *out = nullptr;
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    float zeros[SM_MLP_PARAMS + 1] = {};
    zeros[SM_MLP_PARAMS] = 1.0f;   // an untrained model: loss 1 (error of the whole array)
    return pred_new(out, dtype, is_high != 0, 0, zeros);
}

int sm_predictor_destroy(sm_predictor* p) {
    if (!p) return SM_OK;
    if (p->magic != kPredMagic) return fail(SM_ERR_ARG, "not a predictor handle");
    p->magic = 0;
    const hipError_t e = hipFree(p->dev);
    delete p;
    return e == hipSuccess ? SM_OK : hip_fail(e, "predictor free");
}

int sm_predictor_train(sm_predictor* p, const void* X, int64_t len, const void* Q, int64_t q_len,
                       int64_t samples, int64_t steps, float lr, uint64_t seed, void* ws,
                       size_t ws_bytes, void* stream) {
    if (!pred_ok(p)) return fail(SM_ERR_ARG, "not a predictor handle");
    const int rc = sm_rank_model_train(X, len, Q, q_len, p->dtype, p->is_high, samples, steps, lr,
                                       seed, p->dev, p->dev + SM_MLP_PARAMS, ws, ws_bytes, stream);
    if (rc != SM_OK) return rc;
    p->trained_len = len;
    p->stream = static_cast<hipStream_t>(stream);
    return SM_OK;
}

const float* sm_predictor_params(const sm_predictor* p) { return pred_ok(p) ? p->dev : nullptr; }

int sm_predictor_info(const sm_predictor* p, int* dtype, int* is_high, int64_t* trained_len,
                      float* loss) {
    if (!pred_ok(p)) return fail(SM_ERR_ARG, "not a predictor handle");
    if (dtype) *dtype = p->dtype;
    if (is_high) *is_high = p->is_high;
    if (trained_len) *trained_len = p->trained_len;
    if (loss) {
        float v[SM_MLP_PARAMS + 1];
        const int rc = pred_download(p, v);
        if (rc != SM_OK) return rc;
        *loss = v[SM_MLP_PARAMS];
    }
    return SM_OK;
}

int sm_predictor_save(const sm_predictor* p, void* host_buf, size_t bytes) {
    if (!pred_ok(p)) return fail(SM_ERR_ARG, "not a predictor handle");
    if (!host_buf || bytes < SM_PREDICTOR_BLOB_BYTES)
        return fail(SM_ERR_ARG, "the buffer must hold SM_PREDICTOR_BLOB_BYTES (%d) bytes",
                    SM_PREDICTOR_BLOB_BYTES);
    float v[SM_MLP_PARAMS + 1];
    const int rc = pred_download(p, v);
    if (rc != SM_OK) return rc;
    unsigned char b[SM_PREDICTOR_BLOB_BYTES] = {};
    put<uint32_t>(b, 0, kPredMagic);
    put<uint32_t>(b, 4, kBlobVersion);
    put<int32_t>(b, 8, p->dtype);
    put<int32_t>(b, 12, p->is_high);
    put<int32_t>(b, 16, kFeatureLog2);
    put<int32_t>(b, 20, SM_MLP_HIDDEN);
    put<int32_t>(b, 24, SM_MLP_PARAMS);
    put<float>(b, 28, v[SM_MLP_PARAMS]);
    put<int64_t>(b, 32, p->trained_len);
    memcpy(b + kBlobParamsOff, v, 4 * SM_MLP_PARAMS);
    put<uint32_t>(b, kBlobChecksumOff, fnv1a(b, kBlobChecksumOff));
    memcpy(host_buf, b, SM_PREDICTOR_BLOB_BYTES);
    return SM_OK;
}

int sm_predictor_load(sm_predictor** out, const void* host_buf, size_t bytes) {
    if (!out) return fail(SM_ERR_ARG, "out must not be NULL");
    *out = nullptr;
    if (!host_buf || bytes < SM_PREDICTOR_BLOB_BYTES)
        return fail(SM_ERR_ARG, "a predictor blob has SM_PREDICTOR_BLOB_BYTES (%d) bytes",
                    SM_PREDICTOR_BLOB_BYTES);
    const unsigned char* b = static_cast<const unsigned char*>(host_buf);
    if (get<uint32_t>(b, 0) != kPredMagic) return fail(SM_ERR_ARG, "not a predictor blob");
    if (get<uint32_t>(b, 4) != kBlobVersion)
        return fail(SM_ERR_ARG, "predictor blob version %u is not supported",
                    get<uint32_t>(b, 4));
    if (get<uint32_t>(b, kBlobChecksumOff) != fnv1a(b, kBlobChecksumOff))
        return fail(SM_ERR_ARG, "predictor blob checksum mismatch");
    const int dtype = get<int32_t>(b, 8), is_high = get<int32_t>(b, 12);
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "predictor blob names dtype %d", dtype);
    if ((is_high != 0 && is_high != 1) || get<int32_t>(b, 16) != kFeatureLog2 ||
        get<int32_t>(b, 20) != SM_MLP_HIDDEN || get<int32_t>(b, 24) != SM_MLP_PARAMS)
        return fail(SM_ERR_ARG, "predictor blob describes a different network");
    const int64_t len = get<int64_t>(b, 32);
    if (len < 0) return fail(SM_ERR_ARG, "predictor blob has a negative array length");
    float v[SM_MLP_PARAMS + 1];
    memcpy(v, b + kBlobParamsOff, 4 * SM_MLP_PARAMS);
    v[SM_MLP_PARAMS] = get<float>(b, 28);
    return pred_new(out, dtype, is_high, len, v);
}

}  // extern "C"
