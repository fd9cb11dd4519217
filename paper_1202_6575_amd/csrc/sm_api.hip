// sm_api.hip -- the C ABI of libstablemerge.so (declared in include/stablemerge.h).
//
// Host-side argument checks, workspace layout and the launch sequence of the
// plain stable merge: Steps 1-2 (partition kernel), the single
// synchronisation (the kernel boundary), Steps 3-4 (merge kernel).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "stablemerge.h"
#include "sm_device.h"
#include "sm_launch.h"

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

size_t key_bytes(int dtype) { return dtype == SM_UINT64 ? 8 : 4; }

bool dtype_ok(int dtype) { return dtype == SM_INT32 || dtype == SM_UINT32 || dtype == SM_UINT64; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

bool overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Default top-level block length in elements (the subproblem capacity is
// about twice this).
int32_t default_tile(int dtype, bool pay) {
    if (dtype == SM_UINT64) return pay ? 1024 : 2048;
    return pay ? 2048 : 2048;
}

// Workspace layout of stable_merge: xbar[p_a+1], ybar[p_b+1] (int64), a
// status word, then p_a + p_b subproblem descriptors.
size_t ranks_bytes(int64_t pa, int64_t pb) {
    return ((size_t)(pa + 1 + pb + 1) * sizeof(int64_t) + 255) & ~(size_t)255;
}

struct Plan {
    int64_t p_a, p_b;
    uint32_t cap;
    uint32_t lds;
    size_t ws_bytes;
};

// Chooses block counts and checks that one workgroup can hold a subproblem.
int make_plan(int64_t n, int64_t m, int dtype, bool pay, const sm_options* opt, Plan* pl) {
    if (n < 0 || m < 0) return fail(SM_ERR_ARG, "n and m must be >= 0 (n=%lld, m=%lld)",
                                    (long long)n, (long long)m);
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if ((uint64_t)(n + m) > (1ull << 40)) return fail(SM_ERR_ARG, "n + m too large");
    int64_t pa = opt ? opt->p_a : 0, pb = opt ? opt->p_b : 0;
    int32_t tile = opt && opt->tile > 0 ? opt->tile : default_tile(dtype, pay);
    if (pa < 0 || pb < 0) return fail(SM_ERR_ARG, "p_a and p_b must be >= 0");
    if (tile < 1) return fail(SM_ERR_ARG, "tile must be >= 1");
    if (pa == 0) pa = n > 0 ? (n + tile - 1) / tile : 1;
    if (pb == 0) pb = m > 0 ? (m + tile - 1) / tile : 1;
    if (pa > (1ll << 31) - 2 || pb > (1ll << 31) - 2 || pa + pb > (1ll << 31) - 2)
        return fail(SM_ERR_ARG, "too many blocks (p_a=%lld, p_b=%lld)", (long long)pa,
                    (long long)pb);
    // every subproblem holds at most ceil(n/p_a) + ceil(m/p_b) elements
    const int64_t cap = (n + pa - 1) / pa + (m + pb - 1) / pb;
    const uint32_t lds = sm::merge_lds_bytes(dtype, pay, (uint32_t)(cap < (1 << 20) ? cap : (1 << 20)));
    if (cap >= (1 << 20) || lds > sm::kMaxLds)
        return fail(SM_ERR_ARG,
                    "subproblems of up to %lld elements do not fit one workgroup's LDS "
                    "(%u bytes > %u); use more blocks",
                    (long long)cap, lds, sm::kMaxLds);
    pl->p_a = pa;
    pl->p_b = pb;
    pl->cap = (uint32_t)(cap > 0 ? cap : 1);
    pl->lds = lds;
    pl->ws_bytes = ranks_bytes(pa, pb) + 256 + (size_t)(pa + pb) * sm::kPieceDescBytes;
    return SM_OK;
}


// Checks shared by stable_merge and stable_merge_pieces.
int check_buffers(const void* keys, const uint32_t* payloads, int64_t total, void* out_keys,
                  uint32_t* out_payloads, int dtype) {
    const bool pay = payloads != nullptr;
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

}  // namespace

extern "C" {

const char* sm_last_error(void) { return g_err; }

int sm_version(void) { return 100; }

size_t stable_merge_workspace_bytes(int64_t n, int64_t m, int dtype, int has_payload,
                                    const sm_options* opt) {
    Plan pl;
    if (make_plan(n, m, dtype, has_payload != 0, opt, &pl) != SM_OK) return 0;
    return pl.ws_bytes;
}

int stable_merge_partition(const void* keys, int64_t n, int64_t m, int64_t p_a, int64_t p_b,
                           int dtype, int64_t* xbar, int64_t* ybar, void* stream) {
    if (!dtype_ok(dtype)) return fail(SM_ERR_DTYPE, "unknown dtype %d", dtype);
    if (n < 0 || m < 0) return fail(SM_ERR_ARG, "n and m must be >= 0");
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


size_t stable_merge_pieces_workspace_bytes(int64_t p_a, int64_t p_b) {
    if (p_a < 1 || p_b < 1 || p_a + p_b > (1ll << 40)) return 0;
    return (size_t)(p_a + p_b) * sm::kPieceDescBytes;
}

int stable_merge_pieces(const void* keys, const uint32_t* payloads, int64_t n, int64_t m,
                        int64_t p_a, int64_t p_b, const int64_t* xbar, const int64_t* ybar,
                        void* out_keys, uint32_t* out_payloads, int dtype, void* ws,
                        size_t ws_bytes, void* stream) {
    if ((payloads == nullptr) != (out_payloads == nullptr))
        return fail(SM_ERR_ARG, "payloads and out_payloads must both be NULL or both non-NULL");
    if (p_a < 1 || p_b < 1) return fail(SM_ERR_ARG, "p_a and p_b must be >= 1");
    sm_options o;
    memset(&o, 0, sizeof o);
    o.p_a = p_a;
    o.p_b = p_b;
    Plan pl;
    int rc = make_plan(n, m, dtype, payloads != nullptr, &o, &pl);
    if (rc != SM_OK) return rc;
    if (n + m == 0) return SM_OK;
    if (!xbar || !ybar) return fail(SM_ERR_ARG, "xbar and ybar must not be NULL");
    rc = check_buffers(keys, payloads, n + m, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    const size_t need = (size_t)(pl.p_a + pl.p_b) * sm::kPieceDescBytes;
    if (!ws || ws_bytes < need)
        return fail(SM_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws ? ws_bytes : (size_t)0);
    if (!aligned16(ws)) return fail(SM_ERR_ARG, "workspace must be 16-byte aligned");
    hipError_t e = sm::launch_merge(dtype, keys, payloads, n, m, pl.p_a, pl.p_b, xbar, ybar,
                                    static_cast<sm::PieceDesc*>(ws), out_keys, out_payloads,
                                    pl.cap, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "merge launch");
    return SM_OK;
}

int stable_merge(const void* keys, const uint32_t* payloads, int64_t n, int64_t m, void* out_keys,
                 uint32_t* out_payloads, int dtype, void* ws, size_t ws_bytes,
                 const sm_options* opt, void* stream) {
    const bool pay = payloads != nullptr;
    if ((payloads == nullptr) != (out_payloads == nullptr))
        return fail(SM_ERR_ARG, "payloads and out_payloads must both be NULL or both non-NULL");
    Plan pl;
    int rc = make_plan(n, m, dtype, pay, opt, &pl);
    if (rc != SM_OK) return rc;
    const int64_t total = n + m;
    if (total == 0) return SM_OK;
    rc = check_buffers(keys, payloads, total, out_keys, out_payloads, dtype);
    if (rc != SM_OK) return rc;
    if (!ws || ws_bytes < pl.ws_bytes)
        return fail(SM_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", pl.ws_bytes,
                    ws ? ws_bytes : (size_t)0);
    if (!aligned16(ws)) return fail(SM_ERR_ARG, "workspace must be 16-byte aligned");

    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t* xbar = static_cast<int64_t*>(ws);
    int64_t* ybar = xbar + (pl.p_a + 1);
    int* flag = reinterpret_cast<int*>(static_cast<char*>(ws) + ranks_bytes(pl.p_a, pl.p_b));
    sm::PieceDesc* desc = reinterpret_cast<sm::PieceDesc*>(static_cast<char*>(ws) +
                                                           ranks_bytes(pl.p_a, pl.p_b) + 256);
    hipError_t e;

    if (opt && opt->validate) {
        int host_flag = 0;
        e = hipMemsetAsync(flag, 0, sizeof(int), st);
        if (e != hipSuccess) return hip_fail(e, "validate memset");
        e = sm::launch_validate(dtype, keys, n, m, flag, st);
        if (e != hipSuccess) return hip_fail(e, "validate launch");
        e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "validate readback");
        if (host_flag) return fail(SM_ERR_UNSORTED, "A or B is not non-decreasing");
    }

    e = sm::launch_partition(dtype, keys, n, m, pl.p_a, pl.p_b, xbar, ybar, st);
    if (e != hipSuccess) return hip_fail(e, "partition launch");
    e = sm::launch_merge(dtype, keys, payloads, n, m, pl.p_a, pl.p_b, xbar, ybar, desc, out_keys,
                         out_payloads, pl.cap, st);
    if (e != hipSuccess) return hip_fail(e, "merge launch");
    return SM_OK;
}

}  // extern "C"
