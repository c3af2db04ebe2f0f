// Launchers for the cell-build and search kernels (internal to the library).
#pragma once

#include "nnps_internal.h"

namespace nnps {

hipError_t launch_assign(const double* pos, const Frame& fr, int64_t* X, uint32_t* key,
                         int* cell_count, int* err, hipStream_t st);
hipError_t launch_scan_i32_i32(const int* in, int64_t m, int* out, int64_t* partial, hipStream_t st);
hipError_t launch_scan_u32_u32(const uint32_t* in, int64_t m, uint32_t* out, int64_t* partial,
                               hipStream_t st);
hipError_t launch_scan_i32_i64(const int* in, int64_t m, int64_t* out, int64_t* partial,
                               hipStream_t st);
int64_t scan_partials_needed(int64_t m);
int radix_tiles(int n);
size_t radix_table_entries(int n);
hipError_t launch_radix_sort(int n, int keybits, uint32_t* k0, int* v0, uint32_t* k1, int* v1,
                             uint32_t* table, int64_t* partial, hipStream_t st, uint32_t** kfinal,
                             int** vfinal);
hipError_t launch_pack(const Frame& fr, const int* perm, const int64_t* X, ushort4* q4,
                       const double* pos, double* spos, hipStream_t st);
hipError_t launch_blocks(const Frame& fr, const uint32_t* skey, const int* cell_start, int* flags,
                         int* bidx, int* bstart, int64_t* partial, hipStream_t st);

// Search passes. `nblk_max` bounds the number of blocks (the exact count is on the device).
struct SearchArgs {
    Frame fr;
    const double* pos;        // caller's positions [n][dim]
    const uint32_t* skey;     // sorted cell keys
    const int* perm;          // sorted -> original index
    const int* cell_start;    // [ncell + 1]
    const ushort4* q4;        // sorted FP16 relative coordinates (+ c_x mod 2^16)
    const double* spos;       // sorted FP64 positions [n][4] (baseline only)
    const int64_t* X;         // fixed-point positions [dim][n], original order
    const int* bstart;        // block starts [nblk + 1]
    const int* nblk;          // device pointer to the block count
    int* counts;              // per original index (count pass)
    const int64_t* row_ptr;   // fill pass
    int32_t* col;
    float* dist;
    int64_t capacity;
    int* heavy;               // sorted positions of long rows
    int* nheavy;
    unsigned long long* stats;      // [kStCount] totals
    unsigned long long* blk_stats;  // [nblk_max][5] per-block partial statistics
    uint32_t* cbits;                // accepted-candidate bits, word-major [words][n]
    int* err;
};

hipError_t launch_count(const SearchArgs& a, int nblk_max, hipStream_t st);
hipError_t launch_fill(const SearchArgs& a, int nblk_max, hipStream_t st);
hipError_t launch_long_rows(const SearchArgs& a, hipStream_t st);

}  // namespace nnps
