// SPH kernels that consume the neighbour list (launchers; the C ABI is in capi.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nnps {

// A row whose bounds fall outside [0, ncol] or decrease, or a column index outside [0, n),
// sets kErrBadList in *err (the sums skip what lies outside).
constexpr int kErrBadList = 2;
hipError_t launch_sph_gradient(int dim, int64_t n, double h, const double* pos, const double* f, const double* vol,
                               const int64_t* row_ptr, const int32_t* col, int64_t ncol, double* grad,
                               double* grad_norm, int* err, hipStream_t st);

}  // namespace nnps
