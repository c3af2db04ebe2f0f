// SPH gradient of a scalar field over the CSR neighbour list, in binary64: the standard
// kernel-gradient sum (SPH method section, Eq. 2) with the cubic B-spline kernel (Eq. 3),
// and the normalised, volume-free first-order operator of the appendix (Eq. A5).
//
// Sixteen lanes per row, four rows per wavefront: lane k of a row takes the row's entries
// k, k + 16, ...; the partial sums are combined over the 16 lanes by a butterfly. Rows of
// one wavefront are consecutive particles, so their neighbour lists overlap in cache.
// For each neighbour j of i:
//   dx = x_j - x_i (per axis), r = sqrt(dx0^2 + dx1^2 [+ dx2^2]), q = r / h (as r (1/h)),
//   dW/dq = -2q + 1.5q^2 (q < 1), -0.5(2 - q)^2 (1 <= q < 2), 0 beyond,
//   dW/dx_i = alpha_d / h * dW/dq * (x_i - x_j) / r   (0 when r = 0; as a product with 1/r),
// with alpha_d = 15 / (7 pi h^2) in 2D and 3 / (2 pi h^3) in 3D. Outputs per axis:
//   grad      = sum_j V_j f_j dW/dx_i                                  (Eq. 2)
//   grad_norm = sum_j (f_j - f_i) dW/dx_i / sum_j (x_j - x_i) dW/dx_i   (Eq. A5; 0 when the
//               denominator is 0)
#include "sph_kernels.h"

namespace nnps {

constexpr int kGradThreads = 256;
constexpr int kRowLanes = 16;  // lanes per row

__device__ __forceinline__ double row_sum_f64(double v)
{
#pragma unroll
    for (int o = kRowLanes / 2; o > 0; o >>= 1) v = __dadd_rn(v, __shfl_xor(v, o, 64));
    return v;
}

// dW/dq of the cubic B-spline without alpha_d (Eq. 3 differentiated in q = r / h)
__device__ __forceinline__ double bspline_dwdq(double q)
{
    if (q < 1.0) return __dadd_rn(__dmul_rn(-2.0, q), __dmul_rn(1.5, __dmul_rn(q, q)));
    if (q < 2.0) {
        const double t = __dsub_rn(2.0, q);
        return __dmul_rn(-0.5, __dmul_rn(t, t));
    }
    return 0.0;
}

template <int DIM>
__global__ void __launch_bounds__(kGradThreads)
k_sph_gradient(int64_t n, double inv_h, double alpha_h, const double* __restrict__ pos, const double* __restrict__ f,
               const double* __restrict__ vol, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
               int64_t ncol, double* __restrict__ grad, double* __restrict__ grad_norm, int* __restrict__ err)
{
    const int64_t i = (static_cast<int64_t>(blockIdx.x) * kGradThreads + threadIdx.x) / kRowLanes;
    const int sub = threadIdx.x & (kRowLanes - 1);
    if (i >= n) return;  // whole 16-lane groups leave together
    double xi[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) xi[a] = pos[i * DIM + a];
    const double fi = f[i];
    // row bounds clamped to the column array, column indices outside [0, n) skipped: a
    // list inconsistent with ncol or n cannot make the kernel read outside its arrays, and
    // it is reported (kErrBadList) instead of passing silently
    const int64_t r0 = row_ptr[i], r1 = row_ptr[i + 1];
    const int64_t rs = min(max(r0, int64_t(0)), ncol);
    const int64_t re = min(max(r1, rs), ncol);
    bool bad = sub == 0 && (rs != r0 || re != r1);
    double s[DIM], num[DIM], den[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) s[a] = num[a] = den[a] = 0.0;
    for (int64_t k = rs + sub; k < re; k += kRowLanes) {
        const int64_t j = col[k];
        if (j < 0 || j >= n) {
            bad = true;
            continue;
        }
        double dx[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) dx[a] = __dsub_rn(pos[j * DIM + a], xi[a]);
        double r2 = __dmul_rn(dx[0], dx[0]);
#pragma unroll
        for (int a = 1; a < DIM; ++a) r2 = __dadd_rn(r2, __dmul_rn(dx[a], dx[a]));
        const double r = __dsqrt_rn(r2);
        const double inv_r = r > 0.0 ? __ddiv_rn(1.0, r) : 0.0;
        const double g = __dmul_rn(__dmul_rn(alpha_h, bspline_dwdq(__dmul_rn(r, inv_h))), inv_r);
        const double fj = f[j];
        const double vfj = __dmul_rn(vol ? vol[j] : 1.0, fj);
        const double df = __dsub_rn(fj, fi);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double dw = -__dmul_rn(g, dx[a]);  // dW/dx_i along axis a
            s[a] = __dadd_rn(s[a], __dmul_rn(vfj, dw));
            num[a] = __dadd_rn(num[a], __dmul_rn(df, dw));
            den[a] = __dadd_rn(den[a], __dmul_rn(dx[a], dw));
        }
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        s[a] = row_sum_f64(s[a]);
        num[a] = row_sum_f64(num[a]);
        den[a] = row_sum_f64(den[a]);
    }
    if (bad) atomicOr(err, kErrBadList);
    if (sub == 0) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (grad) grad[i * DIM + a] = s[a];
            if (grad_norm) grad_norm[i * DIM + a] = den[a] != 0.0 ? __ddiv_rn(num[a], den[a]) : 0.0;
        }
    }
}

hipError_t launch_sph_gradient(int dim, int64_t n, double h, const double* pos, const double* f, const double* vol,
                               const int64_t* row_ptr, const int32_t* col, int64_t ncol, double* grad,
                               double* grad_norm, int* err, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const double pi = 3.14159265358979323846;
    const double alpha = dim == 2 ? 15.0 / (7.0 * pi * h * h) : 3.0 / (2.0 * pi * h * h * h);
    const double alpha_h = alpha / h;
    const int64_t rows_per_block = kGradThreads / kRowLanes;
    const dim3 g(static_cast<unsigned>((n + rows_per_block - 1) / rows_per_block)), b(kGradThreads);
    if (dim == 2)
        hipLaunchKernelGGL(k_sph_gradient<2>, g, b, 0, st, n, 1.0 / h, alpha_h, pos, f, vol, row_ptr, col, ncol,
                           grad, grad_norm, err);
    else
        hipLaunchKernelGGL(k_sph_gradient<3>, g, b, 0, st, n, 1.0 / h, alpha_h, pos, f, vol, row_ptr, col, ncol,
                           grad, grad_norm, err);
    return hipGetLastError();
}

}  // namespace nnps
