// All-list neighbour search for small sets (SPH method section, Fig. 3a: every particle
// tested against every other; the paper finds it faster than cell lists below about 1e4
// particles). Binary64 throughout, with the same predicate as the cell-list paths
// (r2 = ((dx0^2) + dx1^2) + dx2^2 in that order, no contraction, r2 <= R^2), so rows and
// distances are bit-identical to the FP64 cell list.
//
// A workgroup is one wavefront: 64 rows (one per lane) against one slice of the candidate
// range. The slice's positions pass through LDS 64 at a time (one coalesced load per
// lane); every lane then reads them in the same order (broadcast reads), so each row's
// entries come out in ascending j with no sort. Slices give small sets enough wavefronts
// to fill the chip. Launches: count, row totals, scan, and (after the caller has sized
// the outputs) the fill.
#include "allpairs_kernels.h"

#include <algorithm>
#include <mutex>

namespace nnps {

// Device scratch of the allocation-free all-list search: the per-slice row counts of the
// largest admissible set (kApStaticCounts ints), then kApStaticFlags error words. Every
// device the library runs on holds its own copy until the process ends; host code must
// never pass this name to a kernel (it is a host-side stand-in): it uses the per-device
// address looked up below.
static __device__ __align__(256) int scratch[kApStaticCounts + kApStaticFlags];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

hipError_t allpairs_static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? static_cast<int*>(p) : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_err[device];
}

int* allpairs_static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

constexpr int kApRows = 64;
constexpr int kApMinSlice = 256;
constexpr int kApTargetWaves = 8192;  // about 8 wavefronts per SIMD
constexpr int kApScanThreads = 1024;

ApPlan allpairs_plan(int n)
{
    ApPlan p;
    p.n = n;
    if (n == 0) return p;
    const int row_groups = (n + kApRows - 1) / kApRows;
    int want = std::max(1, std::min((n + kApMinSlice - 1) / kApMinSlice,
                                    (kApTargetWaves + row_groups - 1) / row_groups));
    int slice = (n + want - 1) / want;
    slice = (slice + 63) / 64 * 64;
    p.slice = slice;
    p.nslice = (n + slice - 1) / slice;
    return p;
}

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

// grid (row groups, slices), 64 threads. The fill writes slice s of row i into
// [w, w + cnt[s][i]) with w = row_ptr[i] + sum_{t < s} cnt[t][i], and never at or past
// min(row_ptr[i + 1], cap): a slice that finds more or fewer pairs than its count (the
// positions or row pointers changed since the count) sets bit kApErrFill of *err.
template <int DIM, bool FILL>
__global__ void __launch_bounds__(kApRows)
k_allpairs(int n, int slice, const double* __restrict__ pos, double R2, ApBox box, int* __restrict__ cnt,
           const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col, float* __restrict__ dist,
           int64_t cap, int* __restrict__ err)
{
    __shared__ double tile[kApRows * DIM];
    const int lane = threadIdx.x;
    const int i = blockIdx.x * kApRows + lane;
    const int s = blockIdx.y;
    const int j0 = s * slice, j1 = min(n, j0 + slice);
    const bool active = i < n;
    double pi[3] = {0.0, 0.0, 0.0};
    if (active) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) pi[k] = pos[static_cast<size_t>(i) * DIM + k];
        if (!FILL && s == 0) {
            bool bad = false;
#pragma unroll
            for (int k = 0; k < DIM; ++k) bad |= !(pi[k] >= box.lo[k] && pi[k] <= box.hi[k]);
            if (bad) atomicOr(err, 1);
        }
    }
    int64_t w = 0, wend = 0;
    if (FILL && active) {
        w = row_ptr[i];
        for (int t = 0; t < s; ++t) w += cnt[static_cast<size_t>(t) * n + i];
        wend = min(min(w + cnt[static_cast<size_t>(s) * n + i], row_ptr[i + 1]), cap);
    }
    int c = 0;
    for (int t0 = j0; t0 < j1; t0 += kApRows) {
        const int m = min(kApRows, j1 - t0);
        __syncthreads();
        if (lane < m) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) tile[lane * DIM + k] = pos[static_cast<size_t>(t0 + lane) * DIM + k];
        }
        __syncthreads();
        if (!active) continue;
        for (int e = 0; e < m; ++e) {
            const int j = t0 + e;
            const double r2 = ap_r2<DIM>(pi, tile + e * DIM);
            if (r2 <= R2 && j != i) {
                if (FILL) {
                    if (w < wend) {
                        col[w] = j;
                        dist[w] = static_cast<float>(__dsqrt_rn(r2));
                    }
                    ++w;
                } else {
                    ++c;
                }
            }
        }
    }
    if (!FILL && active) cnt[static_cast<size_t>(s) * n + i] = c;
    if (FILL && active && w != wend) atomicOr(err, kApErrFill);
}

// row_ptr[i + 1] = sum over slices of cnt[s * n + i]
__global__ void __launch_bounds__(256)
k_allpairs_rows(int n, int nslice, const int* __restrict__ cnt, int64_t* __restrict__ row_ptr)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int64_t t = 0;
    for (int s = 0; s < nslice; ++s) t += cnt[static_cast<size_t>(s) * n + i];
    row_ptr[i + 1] = t;
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

hipError_t launch_allpairs_count(int dim, const ApPlan& p, const double* pos, double R2, const ApBox& box, int* cnt,
                                 int64_t* row_ptr, int* err, hipStream_t st)
{
    if (p.n == 0) return hipSuccess;
    const dim3 g((p.n + kApRows - 1) / kApRows, p.nslice), b(kApRows);
    if (dim == 2)
        hipLaunchKernelGGL((k_allpairs<2, false>), g, b, 0, st, p.n, p.slice, pos, R2, box, cnt, nullptr, nullptr,
                           nullptr, int64_t(0), err);
    else
        hipLaunchKernelGGL((k_allpairs<3, false>), g, b, 0, st, p.n, p.slice, pos, R2, box, cnt, nullptr, nullptr,
                           nullptr, int64_t(0), err);
    hipLaunchKernelGGL(k_allpairs_rows, dim3((p.n + 255) / 256), dim3(256), 0, st, p.n, p.nslice, cnt, row_ptr);
    hipLaunchKernelGGL(k_allpairs_scan, dim3(1), dim3(kApScanThreads), 0, st, p.n, row_ptr);
    return hipGetLastError();
}

hipError_t launch_allpairs_fill(int dim, const ApPlan& p, const double* pos, double R2, const int* cnt,
                                const int64_t* row_ptr, int32_t* col, float* dist, int64_t cap, int* err,
                                hipStream_t st)
{
    if (p.n == 0) return hipSuccess;
    const dim3 g((p.n + kApRows - 1) / kApRows, p.nslice), b(kApRows);
    int* c = const_cast<int*>(cnt);  // read only when filling
    if (dim == 2)
        hipLaunchKernelGGL((k_allpairs<2, true>), g, b, 0, st, p.n, p.slice, pos, R2, ApBox{}, c, row_ptr, col, dist,
                           cap, err);
    else
        hipLaunchKernelGGL((k_allpairs<3, true>), g, b, 0, st, p.n, p.slice, pos, R2, ApBox{}, c, row_ptr, col, dist,
                           cap, err);
    return hipGetLastError();
}

}  // namespace nnps
