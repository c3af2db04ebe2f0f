// All-list neighbour search for small sets (SPH method section, Fig. 3a: every particle
// tested against every other; the paper finds it faster than cell lists below about 1e4
// particles). Binary64 throughout, with the same predicate as the cell-list paths
// (r2 = ((dx0^2) + dx1^2) + dx2^2 in that order, no contraction, r2 <= R^2), so rows and
// distances are bit-identical to the FP64 cell list.
//
// One thread per target row; candidates are staged in LDS tiles of kApTile positions
// that every thread of the workgroup reads in the same order (broadcast reads), so rows
// come out in ascending index with no sort. Three launches: counts into row_ptr[1..n],
// an in-place scan by one workgroup, and the fill.
#include "allpairs_kernels.h"

namespace nnps {

constexpr int kApThreads = 256;
constexpr int kApTile = 256;
constexpr int kApScanThreads = 1024;

template <int DIM>
__device__ __forceinline__ double ap_r2(const double* pi, const double* pj)
{
    const double d0 = __dsub_rn(pj[0], pi[0]);
    const double d1 = __dsub_rn(pj[1], pi[1]);
    double r2 = __dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1));
    if (DIM == 3) {
        const double d2 = __dsub_rn(pj[2], pi[2]);
        r2 = __dadd_rn(r2, __dmul_rn(d2, d2));
    }
    return r2;
}

// FILL = false: row_ptr[i + 1] = |N(i)| and *err |= 1 for a position outside [lo, hi] or
// not finite. FILL = true: the row's (col, dist) pairs at row_ptr[i].. in ascending j.
template <int DIM, bool FILL>
__global__ void __launch_bounds__(kApThreads)
k_allpairs(int n, const double* __restrict__ pos, double R2, ApBox box, int64_t* __restrict__ row_ptr,
           int32_t* __restrict__ col, float* __restrict__ dist, int* __restrict__ err)
{
    __shared__ double tile[kApTile * DIM];
    const int i = blockIdx.x * kApThreads + threadIdx.x;
    const bool active = i < n;
    double pi[3] = {0.0, 0.0, 0.0};
    if (active) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) pi[k] = pos[static_cast<size_t>(i) * DIM + k];
        if (!FILL) {
            bool bad = false;
#pragma unroll
            for (int k = 0; k < DIM; ++k) bad |= !(pi[k] >= box.lo[k] && pi[k] <= box.hi[k]);
            if (bad) atomicOr(err, 1);
        }
    }
    int64_t w = FILL && active ? row_ptr[i] : 0;
    int cnt = 0;
    for (int t0 = 0; t0 < n; t0 += kApTile) {
        const int m = min(kApTile, n - t0);
        __syncthreads();
        for (int e = threadIdx.x; e < m * DIM; e += kApThreads) tile[e] = pos[static_cast<size_t>(t0) * DIM + e];
        __syncthreads();
        if (!active) continue;
        for (int e = 0; e < m; ++e) {
            const int j = t0 + e;
            const double r2 = ap_r2<DIM>(pi, tile + e * DIM);
            if (r2 <= R2 && j != i) {
                if (FILL) {
                    col[w] = j;
                    dist[w] = static_cast<float>(__dsqrt_rn(r2));
                    ++w;
                } else {
                    ++cnt;
                }
            }
        }
    }
    if (!FILL && active) row_ptr[i + 1] = cnt;
}

// One workgroup: row_ptr[0] = 0 and row_ptr[1..n] (counts) replaced by their inclusive
// prefix sums, so row_ptr[n] = nnz.
__global__ void __launch_bounds__(kApScanThreads)
k_allpairs_scan(int n, int64_t* __restrict__ row_ptr)
{
    __shared__ int64_t part[kApScanThreads];
    const int per = (n + kApScanThreads - 1) / kApScanThreads;
    const int a = min(n, static_cast<int>(threadIdx.x) * per), b = min(n, a + per);
    int64_t s = 0;
    for (int k = a; k < b; ++k) s += row_ptr[k + 1];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread sums
    for (int o = 1; o < kApScanThreads; o <<= 1) {
        const int64_t v = threadIdx.x >= static_cast<unsigned>(o) ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int k = a; k < b; ++k) {
        run += row_ptr[k + 1];
        row_ptr[k + 1] = run;
    }
    if (threadIdx.x == 0) row_ptr[0] = 0;
}

hipError_t launch_allpairs_count(int dim, int n, const double* pos, double R2, const ApBox& box, int64_t* row_ptr,
                                 int* err, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 g((n + kApThreads - 1) / kApThreads), b(kApThreads);
    if (dim == 2)
        hipLaunchKernelGGL((k_allpairs<2, false>), g, b, 0, st, n, pos, R2, box, row_ptr, nullptr, nullptr, err);
    else
        hipLaunchKernelGGL((k_allpairs<3, false>), g, b, 0, st, n, pos, R2, box, row_ptr, nullptr, nullptr, err);
    hipLaunchKernelGGL(k_allpairs_scan, dim3(1), dim3(kApScanThreads), 0, st, n, row_ptr);
    return hipGetLastError();
}

hipError_t launch_allpairs_fill(int dim, int n, const double* pos, double R2, const ApBox& box,
                                const int64_t* row_ptr, int32_t* col, float* dist, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 g((n + kApThreads - 1) / kApThreads), b(kApThreads);
    int64_t* rp = const_cast<int64_t*>(row_ptr);  // read only when filling
    if (dim == 2)
        hipLaunchKernelGGL((k_allpairs<2, true>), g, b, 0, st, n, pos, R2, box, rp, col, dist, nullptr);
    else
        hipLaunchKernelGGL((k_allpairs<3, true>), g, b, 0, st, n, pos, R2, box, rp, col, dist, nullptr);
    return hipGetLastError();
}

}  // namespace nnps
