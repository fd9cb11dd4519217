// sm_launch.h -- host-side launchers of the stable-merge kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sm {

// Every `dtype` below is a kernel dtype code (sm_keys.h): a public key type
// code, with kDescending set for descending order where a launcher supports
// it (the small-block merge and the learned kernels do not).

// Workgroup size of the merge kernels: p = 256 lane-level processing elements.
constexpr int kMergeThreads = 256;
// Largest dynamic LDS a merge workgroup may use (gfx950: 160 KiB per CU).
constexpr uint32_t kMaxLds = 160 * 1024;
// LDS allocation unit of one workgroup (128 of them make up kMaxLds)
constexpr uint32_t kLdsGranule = 1280;

// LDS bytes a merge workgroup needs for subproblems of up to cap elements.
uint32_t merge_lds_bytes(int dtype, bool pay, uint32_t cap);

// Steps 1-2: xbar[0..p_a], ybar[0..p_b] (int64, device).
hipError_t launch_partition(int dtype, const void* keys, int64_t n, int64_t m,
                            int64_t p_a, int64_t p_b, int64_t* xbar, int64_t* ybar,
                            hipStream_t st);

// Block starts up to which Steps 1-2 run as group searches, kSearchGroup
// lanes per search.
constexpr int64_t kGroupSearchMax = 2048;
constexpr int kSearchGroup = 16;

struct PieceDesc;

// Workgroup size of the merge that takes its subproblem straight from the
// cross ranks (a few large subproblems), and the subproblem count, per
// compute unit, up to which it is used.
constexpr int kWideMergeThreads = 1024;
constexpr int kWideMergeMaxWgPerCu = 4;

// Whether launch_merge_cases_direct serves P subproblems of up to cap
// elements: few of them (at most kWideMergeMaxWgPerCu per compute unit),
// each larger than the register-pipelined merges stage or fewer than the
// compute units, within one workgroup's registers and LDS.
bool merge_cases_direct_applies(int dtype, bool pay, uint32_t cap, int64_t P);

// Steps 3-4 and the merges in one launch, one kWideMergeThreads workgroup per
// subproblem: each computes its own descriptor from xbar / ybar, stages its
// inputs in LDS and writes its merged outputs straight to memory.
hipError_t launch_merge_cases_direct(int dtype, const void* keys, const uint32_t* pay, int64_t n,
                                     int64_t m, int64_t p_a, int64_t p_b, const int64_t* xbar,
                                     const int64_t* ybar, void* out_keys, uint32_t* out_pay,
                                     uint32_t cap, hipStream_t st);

// Steps 3-4 case selection alone.
hipError_t launch_cases(int64_t n, int64_t m, int64_t p_a, int64_t p_b, const int64_t* xbar,
                        const int64_t* ybar, PieceDesc* desc, hipStream_t st);

// Merges of P subproblem descriptors (keys / payload positions index arrays
// of nkeys elements; outputs index arrays of nout elements).  If P_dev is
// not null the count is read from device memory and P is its upper bound.
hipError_t launch_merge_desc(int dtype, const void* keys, const uint32_t* pay, int64_t nkeys,
                             void* out_keys, uint32_t* out_pay, int64_t nout,
                             const PieceDesc* desc, int64_t P, const int64_t* P_dev, uint32_t cap,
                             hipStream_t st, bool packed = false);

// Steps 3-4 plus the merges for small blocks: one lane per subproblem, no
// descriptors (subproblems of at most kFineCap elements).
hipError_t launch_fine_merge(int dtype, const void* keys, const uint32_t* pay, int64_t n,
                            int64_t m, int64_t p_a, int64_t p_b, const int64_t* xbar,
                            const int64_t* ybar, void* out_keys, uint32_t* out_pay,
                            hipStream_t st);
constexpr uint32_t kFineCap = 64;

// Subproblem capacity (elements) that one merge workgroup can stage for a
// key type, in the register-pipelined kernel at the default tile.
uint32_t merge_cap_for_tile(int32_t tile);

// Capacity for packed steps over subproblems of at most `cap` elements: the
// largest that keeps the merge workgroup's LDS granules and register slots
// (and so the workgroups per compute unit) as they are for `cap`.
uint32_t merge_pack_cap(int dtype, bool pay, uint32_t cap);

// Number of compute units of the current device.
int device_cu_count();

constexpr size_t kPieceDescBytes = 32;

// Sets *flag (device int) to 1 if keys[0, n) or keys[n, n + m) is not
// sorted in the order of the kernel dtype code; *flag must be 0 before the
// launch.
hipError_t launch_validate(int dtype, const void* keys, int64_t n, int64_t m, int* flag,
                           hipStream_t st);

}  // namespace sm
