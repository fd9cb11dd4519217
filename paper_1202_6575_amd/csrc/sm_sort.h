// sm_sort.h -- host side of the stable merge sort (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "sm_batch.h"

namespace sm {

// Workspace of one sort: a second key (and payload) buffer of N elements,
// the jobs of the largest pass, and the batch engine's state for it.
struct SortLayout {
    int passes;
    int64_t count_max;
    size_t off_tmp_keys, off_tmp_pay, off_jobs, off_batch, bytes;
    BatchLayout batch;
};

// Run lengths the run-formation kernel is built for (4096 for 32-bit keys).
bool sort_run_ok(int run, int dtype);

// Number of merge passes after runs of `run` elements: ceil(log2(N / run)).
int sort_passes(int64_t N, int run);

SortLayout sort_layout(int64_t N, int dtype, bool pay, int run, int64_t tile);

// Run formation, then the merge passes; the result lands in out_keys /
// out_pay, which may be the input arrays themselves.
hipError_t launch_sort(int dtype, const void* keys, const uint32_t* pay, int64_t N, void* out_keys,
                       uint32_t* out_pay, int run, int64_t tile, char* ws, const SortLayout& L,
                       hipStream_t st);

}  // namespace sm
