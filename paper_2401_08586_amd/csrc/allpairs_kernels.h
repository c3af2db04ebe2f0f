// All-list neighbour search for small sets (launchers; the C ABI is in capi.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nnps {

struct ApBox {
    double lo[3], hi[3];
};

// Largest set the all-list path takes (its work grows as n^2).
constexpr int kAllPairsMaxN = 65536;
// The allocation-free all-list search keeps its per-slice row counts in a static device
// array: kApStaticCounts is the largest nslice * n of allpairs_plan over n <= kAllPairsMaxN
// (589,248 at n = 65,472; 2.25 MiB), followed by kApStaticFlags error words.
constexpr int64_t kApStaticCounts = 589248;
constexpr int kApStaticFlags = 64;
// Looks up, once per device (the device must be current), the address of that device's
// copy of the static array; returns the lookup's status.
hipError_t allpairs_static_scratch_init(int device);
// The address found by allpairs_static_scratch_init(device), or nullptr.
int* allpairs_static_scratch(int device);

// Work split: rows in groups of 64 (one wavefront, one row per lane) times slices of the
// candidate range, so that even small sets give the chip thousands of wavefronts.
struct ApPlan {
    int n = 0;
    int slice = 0;   // candidates per slice (a multiple of 64)
    int nslice = 0;  // slices per row
};
ApPlan allpairs_plan(int n);

// Count: cnt[s * n + i] = neighbours of row i in slice s; row_ptr[1..n] = row totals, then
// their inclusive scan (row_ptr[0] = 0); *err |= 1 for a position outside [lo, hi] or not
// finite. cnt holds nslice * n ints.
hipError_t launch_allpairs_count(int dim, const ApPlan& p, const double* pos, double R2, const ApBox& box, int* cnt,
                                 int64_t* row_ptr, int* err, hipStream_t st);
// Fill: row i's pairs of slice s at row_ptr[i] + sum_{t < s} cnt[t * n + i], ascending j,
// never at or past min(row_ptr[i + 1], cap); a slice whose pairs do not match its count
// sets kApErrFill in *err.
constexpr int kApErrFill = 1;
hipError_t launch_allpairs_fill(int dim, const ApPlan& p, const double* pos, double R2, const int* cnt,
                                const int64_t* row_ptr, int32_t* col, float* dist, int64_t cap, int* err,
                                hipStream_t st);

}  // namespace nnps
