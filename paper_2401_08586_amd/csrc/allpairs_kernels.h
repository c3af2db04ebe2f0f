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

hipError_t launch_allpairs_count(int dim, int n, const double* pos, double R2, const ApBox& box, int64_t* row_ptr,
                                 int* err, hipStream_t st);
hipError_t launch_allpairs_fill(int dim, int n, const double* pos, double R2, const ApBox& box,
                                const int64_t* row_ptr, int32_t* col, float* dist, hipStream_t st);

}  // namespace nnps
