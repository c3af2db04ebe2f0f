// SPH kernels that consume the neighbour list (launchers; the C ABI is in capi.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nnps {

hipError_t launch_sph_gradient(int dim, int64_t n, double h, const double* pos, const double* f, const double* vol,
                               const int64_t* row_ptr, const int32_t* col, int64_t ncol, double* grad,
                               double* grad_norm, hipStream_t st);

}  // namespace nnps
