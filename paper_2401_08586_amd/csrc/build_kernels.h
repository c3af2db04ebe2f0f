// Launchers for the cell-build and search kernels (internal to the library).
#pragma once

#include "nnps_internal.h"

namespace nnps {

// What every kernel of one launch shares: the set table and the global index spaces.
struct Launch {
    int dim, mode;             // shared by all sets of a launch
    int nsets;
    int ntot;                  // total particles (sum of the sets' n)
    int ncell_tot;             // total cells
    const SetDesc* sets;       // [nsets] (device)
    const int* poffs;          // [nsets + 1] particle offsets (device)
    const int* coffs;          // [nsets + 1] cell offsets (device)
};

hipError_t launch_fill_i32(int* p, int64_t m, int v, hipStream_t st);
hipError_t launch_assign(const Launch& L, int64_t* X, uint32_t* key, int* cell_count, int* err, hipStream_t st);
hipError_t launch_scan_i32_i32(const int* in, int64_t m, int* out, int64_t* partial, hipStream_t st);
hipError_t launch_scan_i32_i64(const int* in, int64_t m, int64_t* out, int64_t* partial, hipStream_t st);
int64_t scan_partials_needed(int64_t m);
int radix_tiles(int n);
size_t radix_table_entries(int n);
hipError_t launch_radix_sort(int n, int keybits, uint32_t* k0, int* v0, uint32_t* k1, int* v1,
                             uint32_t* table, int64_t* partial, hipStream_t st, uint32_t** kfinal,
                             int** vfinal);
hipError_t launch_pack(const Launch& L, const uint32_t* skey, const int* perm, const int64_t* X, ushort4* q4,
                       double* spos, hipStream_t st);
hipError_t launch_blocks(const Launch& L, const uint32_t* skey, const int* cell_start, int* flags, int* bidx,
                         int* bstart, int* bset, int64_t* partial, hipStream_t st);
hipError_t launch_rowptr(const Launch& L, const int* counts, int64_t* rowg, int64_t* partial, int64_t* nnz,
                         hipStream_t st);

// Search passes over every block of every set. `nblk_max` bounds the number of blocks
// (the exact count is on the device).
struct SearchArgs {
    Launch L;
    const uint32_t* skey;     // sorted global cell keys
    const int* perm;          // sorted position -> global particle index
    const int* cell_start;    // [ncell_tot + 1]
    const ushort4* q4;        // sorted FP16 relative coordinates (+ c_x mod 2^16)
    const double* spos;       // sorted FP64 positions [ntot][4] (baseline only)
    const int64_t* X;         // fixed-point positions, global index, stride x_stride(dim)
    const int* bstart;        // block starts [nblk + 1]
    const int* bset;          // set of each block [nblk]
    const int* nblk;          // device pointer to the block count
    int* counts;              // per global particle (count pass)
    int* heavy;               // sorted positions of long rows
    int* nheavy;
    unsigned long long* stats;      // [kStCount] totals
    unsigned long long* blk_stats;  // [nblk_max][5] per-block partial statistics
    uint32_t* cbits;                // accepted-candidate bits, word-major [words][ntot]
    uint32_t* lrscratch;            // long-row path merge scratch, per workgroup
    int64_t lrscratch_words;        // its size per workgroup (32-bit words)
    int lr_keys;                    // keys a long-row workgroup sorts in LDS
    int* err;
};

hipError_t launch_count(const SearchArgs& a, int nblk_max, hipStream_t st);
hipError_t launch_fill(const SearchArgs& a, int nblk_max, hipStream_t st);
hipError_t launch_long_rows(const SearchArgs& a, int grid, hipStream_t st);

}  // namespace nnps
