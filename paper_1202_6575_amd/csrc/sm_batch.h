// sm_batch.h -- host side of the job engine (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace sm {

struct PieceDesc;

// Device workspace of one batch of `count` jobs over `total` elements with
// blocks of `tile` elements: byte offsets of each array, the bounds on the
// number of subproblems (p_max) and cross ranks (s_max), total bytes.
struct BatchLayout {
    int64_t count, nblocks, p_max, s_max;
    size_t off_pstart, off_sstart, off_bsum_p, off_bsum_s, off_totals, off_flag, off_ranks,
        off_desc, bytes;
};

BatchLayout batch_layout(int64_t count, int64_t total, int64_t tile);

// Jobs of independent pairs (offsets[count + 1], n_a[count]) into `jobs`;
// *bad (device int, cleared beforehand) is set for an inconsistent pair.
hipError_t launch_jobs_from_pairs(const int64_t* offsets, const int64_t* n_a, int64_t count,
                                  int64_t total, PieceDesc* jobs, int* bad, hipStream_t st);

// Sets *bad if some A or B of a batch of valid pairs is not non-decreasing.
hipError_t launch_batch_validate(int dtype, const void* keys, const int64_t* offsets,
                                 const int64_t* n_a, int64_t count, int64_t total, int* bad,
                                 hipStream_t st);

// Zero n device ints with a kernel (graph-capture safe).
hipError_t launch_clear(int* p, int n, hipStream_t st);

// Cross ranks from a learned starting point (ascending key types only):
// `model` (97 device floats) maps a key to its normalised rank in any
// sorted array drawn from the keys' distribution; the search for the rank
// of x in an array of len elements starts at model(x) * len and steps away
// by the largest power of two <= max(1, step_frac * len), doubling, before
// bisecting.  counters (device, may be null) accumulate [searches, probes].
struct LearnedSearch {
    const float* model;
    float step_frac;
    unsigned long long* counters;
};

// plan + scan, partition, cases and merge for `count` jobs; with `ls` the
// partition searches start at learned guesses (the ranks are the same).
hipError_t launch_batch(int dtype, const void* keys, const uint32_t* pay, int64_t nkeys,
                        void* out_keys, uint32_t* out_pay, int64_t nout, const PieceDesc* jobs,
                        int64_t count, int64_t tile, char* ws, const BatchLayout& L,
                        hipStream_t st, const LearnedSearch* ls = nullptr);

// partition, cases and merge for jobs whose plan is already in the
// workspace: subproblem and cross-rank starts at L.off_pstart / L.off_sstart
// (count + 1 each, exclusive, the last one the total) and the two totals at
// L.off_totals.  uni_p, uni_s > 0: every job but the last has exactly uni_p
// subproblems and uni_s cross ranks, so a flat index finds its job by
// division; 0: by search over the starts.
hipError_t launch_batch_planned(int dtype, const void* keys, const uint32_t* pay, int64_t nkeys,
                                void* out_keys, uint32_t* out_pay, int64_t nout,
                                const PieceDesc* jobs, int64_t count, int64_t tile, char* ws,
                                const BatchLayout& L, hipStream_t st, const LearnedSearch* ls,
                                int64_t uni_p, int64_t uni_s);

}  // namespace sm
