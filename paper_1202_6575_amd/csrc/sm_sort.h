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

// seg_count > 0: the segmented sort of seg_count segments no longer than
// max_len each.
SortLayout sort_layout(int64_t N, int dtype, bool pay, int run, int64_t tile,
                       int64_t seg_count = 0, int64_t max_len = 0);

// Run formation, then the merge passes; the result lands in out_keys /
// out_pay, which may be the input arrays themselves.
// With seg_offsets (device, seg_count + 1 entries from 0 to N) every
// segment is sorted on its own: runs start at segment starts and every merge
// pass pairs runs within a segment.
// With `ls` every merge pass finds its cross ranks from learned guesses.
hipError_t launch_sort(int dtype, const void* keys, const uint32_t* pay, int64_t N, void* out_keys,
                       uint32_t* out_pay, int run, int64_t tile, char* ws, const SortLayout& L,
                       hipStream_t st, const int64_t* seg_offsets = nullptr,
                       int64_t seg_count = 0, const LearnedSearch* ls = nullptr);

// Run formation alone: every run of `run` consecutive elements stably
// sorted into out (out may be keys itself).
hipError_t launch_sort_runs(int dtype, const void* keys, const uint32_t* pay, int64_t N,
                            void* out_keys, uint32_t* out_pay, int run, hipStream_t st);

// Sets *bad (device int, cleared beforehand) unless the offsets run from 0
// to N without decreasing and no segment is longer than max_len.
hipError_t launch_seg_check(const int64_t* offsets, int64_t count, int64_t N, int64_t max_len,
                            int* bad, hipStream_t st);

}  // namespace sm
