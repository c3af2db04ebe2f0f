// Internal definitions shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnps {

// Targets per work block: one wavefront, one target per lane.
constexpr int kWave = 64;
// Candidate positions staged in LDS per chunk in the count pass (even).
constexpr int kStage = 512;
// Fill pass: largest candidate union of a block (staged whole and ranked by original
// index) and largest number of CSR entries of a block; blocks above either limit send
// their rows to the long-row path.
constexpr int kUnion2 = 512;
constexpr int kUnion3 = 1024;
constexpr int kFlat2 = 2048;
constexpr int kFlat3 = 4608;
// Accepted-candidate bits the count pass keeps per target, indexed by the candidate's
// position in the block's union (32 positions per word), stored word-major so a
// wavefront's stores coalesce. Blocks with a larger union take the long-row path.
constexpr int kCandWords2 = kUnion2 / 32;
constexpr int kCandWords3 = kUnion3 / 32;
// Fixed-point positions are stored per particle, padded to a power of two of int64.
__host__ __device__ constexpr int x_stride(int dim) { return dim == 3 ? 4 : 2; }
// Largest x-span (cells) of a work block; keeps staged cell offsets exact in FP16.
constexpr int kMaxXWin = 256;
// Dense-cell path: candidates staged per chunk, targets per work unit (a workgroup of
// four wavefronts, 64 targets each) and the default thresholds.
constexpr int kDenseChunk = 1024;
// The FP16 passes stage fewer candidates per chunk, so that the fill's tables (records,
// FP64 positions and the per-wavefront queues of accepted candidates) still fit four
// workgroups per CU (a multiple of 128); the count uses the same chunks, so that the
// accepted bits it keeps per target and chunk are the fill's.
constexpr int kDenseChunkF16 = 896;
// Default bound on the device scratch for those bits (MiB).
constexpr int kDenseBitsMiB = 16384;
constexpr int kDenseQueue = 512;  // per-wavefront queue of a row's accepted candidates in a chunk
constexpr int kDenseThreads = 256;
constexpr int kDenseBitsThreads = 512;  // the dense fill that takes the count's kept bits
constexpr int kDenseSlice = 256;
constexpr int kDenseUnion3 = 512;
constexpr int kDenseUnion2 = 160;
constexpr int kDenseGrid = 1280;  // five workgroups on each of the 256 compute units
constexpr int64_t kDenseMaxEntries = int64_t(1) << 28;
constexpr int kDenseStats = 6;  // candidates, band, false pos, false neg, outside disagree, rows

// Per-block descriptors the count pass leaves for the fill (ints per block), and the
// spare descriptors of the last round over the XCDs.
constexpr int kBlockDescInts = 24;
constexpr int kXcdPad = 8;

// Device error flags.
constexpr int kErrDomain = 1;
constexpr int kErrCapacity = 2;
constexpr int kErrLongRow = 4;

// Statistic slots (int64 on the device).
enum StatSlot {
    kStCandidates = 0,
    kStBand,
    kStFalsePos,
    kStFalseNeg,
    kStOutsideDisagree,
    kStHeavy,
    kStDenseRows,
    kStCount
};

// Everything a kernel needs to know about one particle set's grid and thresholds.
struct Frame {
    int dim;
    int mode;
    int n;
    int F;              // fixed-point fraction bits per cell width
    int nc[3];          // cells per axis (1 for unused axes)
    int ncell;
    double lo[3], hi[3];
    double w;           // cell width
    double s;           // 2^F / w
    double R2;          // fl(R*R)
    float dist_scale;   // (float)(w * 2^-F)
    int xwin;           // largest x-span of a work block, in cells
    int bmax;           // most targets of a work block (<= 64)
    uint16_t t_lo, t_hi, t_mid;  // FP16 thresholds on r2 = 4|delta|^2 (bit patterns)
    float t32_lo, t32_hi, t32_mid;  // FP32 thresholds on the same r2
};

// One particle set of a launch. All sets of a launch share one global particle index
// space (set s owns [poff, poff + n)) and one global cell index space ([coff, coff +
// ncell)), so one sort and one kernel launch per pass cover every set.
struct SetDesc {
    Frame fr;                // fr.n = this set's particle count
    int poff, coff;          // first global particle / cell index
    const double* pos;       // caller's positions [n][dim] (float64)
    const double* disp;      // incremental update: displacements [n][dim] added to pos, or null
    int64_t* row_ptr;        // caller's CSR row pointers [n + 1]
    int32_t* col;            // caller's CSR column indices (set-local)
    float* dist;             // caller's CSR distances
    int64_t capacity;        // entries available in col and dist
};

// Index of the set owning global index v, given offs[0..nsets] ascending.
__device__ __forceinline__ int find_set(const int* __restrict__ offs, int nsets, int v)
{
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace nnps
