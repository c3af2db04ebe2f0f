// Internal definitions shared by the HIP kernels and the C-ABI host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnps {

// Targets per work block: one wavefront, one target per lane.
constexpr int kWave = 64;
// Candidate positions staged in LDS per chunk (even).
constexpr int kStage = 1024;
// Per-lane row buffers in the fill pass (entries); longer rows take the long-row path.
constexpr int kCap2 = 32;
constexpr int kCap3 = 96;
// Longest row the long-row path sorts in LDS.
constexpr int kHeavySortMax = 4096;
// Block cuts every 512 cells along x, so the staged cell offsets stay exact in FP16.
constexpr int kXSpanShift = 9;

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
    kStCount
};

// Everything a kernel needs to know about the grid and the thresholds.
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
    uint16_t t_lo, t_hi, t_mid;  // FP16 thresholds on r2 = 4|delta|^2 (bit patterns)
};

}  // namespace nnps
