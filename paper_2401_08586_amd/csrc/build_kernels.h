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
    const int* roffs;          // [nsets + 1] offsets of the sets' row segments (device)
    int nrows_tot;             // total row segments (x-lines cut into pieces of 64 cells)
};

hipError_t launch_fill_i32(int* p, int64_t m, int v, hipStream_t st);
hipError_t launch_fill2_i32(int* p, int64_t m, int* q, int64_t k, int v, hipStream_t st);
int row_segments(int ncx);  // pieces a row of ncx cells is walked in
hipError_t launch_assign(const Launch& L, double* X, uint32_t* key, int* slot, int* cell_count, int* err,
                         hipStream_t st);
hipError_t launch_place(int ntot, const uint32_t* key, const int* slot, const int* cell_start, uint32_t* skey,
                        int* perm, hipStream_t st);
hipError_t launch_scan_i32_i32(const int* in, int64_t m, int* out, int64_t* partial, hipStream_t st);
hipError_t launch_scan_i32_i64(const int* in, int64_t m, int64_t* out, int64_t* partial, hipStream_t st);
int64_t scan_partials_needed(int64_t m);
int radix_tiles(int n);
size_t radix_table_entries(int n);
hipError_t launch_pack(const Launch& L, const uint32_t* skey, const int* perm, const double* X, ushort4* q4,
                       double* spos, float4* rq, int* inv, hipStream_t st, uint32_t* skey_out = nullptr,
                       int* perm_out = nullptr);

// Incremental update of a built structure (see k_upd_move): device tables of one update.
struct Update {
    uint32_t* knew;           // [ntot] new cell key by particle
    uint32_t* mig;            // [ceil(ntot / 32)] bit s: the particle at old position s changed cell
    int* leave;               // [ncell_tot + 1] migrants out of each cell
    int* arrive;              // [ncell_tot + 1] migrants into each cell
                              // (leave, arrive and mig are one zeroed block: see update_of)
    int* aslot;               // [ntot] by particle: a migrant's arrival slot in its new cell
    int* cs_old;              // [ncell_tot + 1] cell starts before the update
    uint32_t* skey2;          // [ntot] new order: cell keys
    int* perm2;               // [ntot] new order: particle indices
};
// U1: move (when the set has displacements), fixed point, cells, migrant flags and counts.
hipError_t launch_update_move(const Launch& L, const uint32_t* skey, const int* inv, double* X, const Update& u,
                              int* err, hipStream_t st);
// U2: new cell occupancies and starts (cell_start is rewritten; the old one goes to cs_old).
hipError_t launch_update_cells(const Launch& L, int* cell_start, int* cnt, const Update& u, int64_t* partial,
                               hipStream_t st);
// U3: every particle's new sorted position (into skey2 / perm2).
hipError_t launch_update_place(const Launch& L, const uint32_t* skey, const int* perm, const int* cell_start,
                               const Update& u, hipStream_t st);
hipError_t launch_blocks(const Launch& L, const int* cell_start, const int* wdense, int* boff, int* bstart, int* bset,
                         int64_t* partial, hipStream_t st);

// Dense-cell path: device tables of one build. A cell is "dense" when its stencil holds
// more than `thresh` particles; runs of dense cells get no work blocks. Each dense cell g owns the list ulist[uoff[g] ..
// uoff[g] + usz[g]) of the sorted positions of the particles in its 3^d stencil, in
// ascending original index, and ceil(occupancy / kDenseSlice) work units.
struct DenseBuild {
    int thresh;             // stencil size above which a window is dense
    int64_t cap;            // capacity of the union lists (entries)
    int* usz;               // [ncell_tot] stencil size of dense cells, else 0
    int* wdense;            // [ncell_tot] 1 for every cell of a dense window
    int64_t* uoff;          // [ncell_tot + 1] exclusive scan of usz
    int* nsl;               // [ncell_tot] work units per cell
    int* unit_off;          // [ncell_tot + 1] exclusive scan of nsl
    int* ucell;             // [ntot] cell of each work unit
    int* dn;                // [1] entries in use; 0 when the dense path is off for the build
    int* ecnt;              // [ntot] dense stencils each particle belongs to
    int* epos;              // [ntot + 1] exclusive scan of ecnt
    uint32_t *uk0, *uk1;    // [cap] sort keys (dense cell)
    int *uv0, *uv1;         // [cap] sort values (sorted position)
    uint32_t* table;        // radix scratch
    int64_t* partial;       // scan scratch
    int* seen;              // [1] set to 1 when any cell is dense
    int* dbn;               // [ncell_tot] (target, chunk) pairs of each dense cell (FP16 chunks)
    int64_t* dboff;         // [ncell_tot + 1] exclusive scan of dbn
};
// Stencil sizes and the dense flag only (the path is not used by this build).
hipError_t launch_dense_detect(const Launch& L, const int* cell_start, const DenseBuild& d, hipStream_t st);
// Before the block table: stencil sizes, dense windows, union offsets and work units.
hipError_t launch_dense_cells(const Launch& L, const int* cell_start, const DenseBuild& d, hipStream_t st);
// After the sort and pack: the union lists. *ulist receives the sorted list array.
hipError_t launch_dense_unions(const Launch& L, const uint32_t* skey, const int* inv, const DenseBuild& d,
                               hipStream_t st, int** ulist);
// Row pointers of every set from the counts; also each particle's row start by sorted
// position (rsort[inv[i]]).
hipError_t launch_rowptr(const Launch& L, const int* counts, int64_t* rowg, int64_t* partial, int64_t* nnz,
                         const int* inv, int64_t* rsort, hipStream_t st);

// Search passes over every block of every set. `nblk_max` bounds the number of blocks
// (the exact count is on the device).
struct SearchArgs {
    Launch L;
    const uint32_t* skey;     // sorted global cell keys
    const int* perm;          // sorted position -> global particle index
    const int* cell_start;    // [ncell_tot + 1]
    const ushort4* q4;        // sorted FP16 relative coordinates (+ c_x mod 2^16)
    const double* spos;       // sorted FP64 positions [ntot][4] (FP64 and FP32 modes)
    const float4* rq;         // sorted FP32 relative coordinates + packed cell bits (FP32 mode)
    const double* X;          // fixed-point positions (exact integers), global index, stride x_stride(dim)
    const int* bstart;        // block starts [nblk + 1]
    const int* bset;          // set of each block [nblk]
    const int* nblk;          // device pointer to the block count
    int* counts;              // per global particle (count pass)
    int* counts_s;            // the same by sorted position (the fill reads them in block order)
    int64_t* rsort;           // each particle's row start in its set's output, by sorted position
    int* bdesc;               // [nblk_max][24] per-block descriptors the count pass leaves for the fill
    int* heavy;               // sorted positions of long rows
    int* nheavy;
    unsigned long long* stats;      // [kStCount] totals
    unsigned long long* blk_stats;  // [nblk_max][5] per-block partial statistics
    uint32_t* cbits;                // accepted-candidate bits, word-major [words][ntot]
    uint32_t* lrscratch;            // long-row path merge scratch, per workgroup
    int64_t lrscratch_words;        // its size per workgroup (32-bit words)
    int lr_keys;                    // keys a long-row workgroup sorts in LDS
    int* err;
    int* sink;                      // [2 * 64] per-lane dummy output slots
    int half;                       // 1: rows keep only neighbours of larger original index
    // dense-cell path (wdense == nullptr: off)
    const int* wdense;
    const int* usz;
    const int64_t* uoff;
    const int* ulist;
    const int* unit_off;
    const int* ucell;
    const int* dn;
    int* ucount;                    // work-unit counter (zeroed before each launch)
    unsigned long long* dstats;     // [dgrid][kDenseStats] per-workgroup statistics
    int dgrid;
    // FP16 dense passes: the count keeps each target's accepted bits per chunk (64 lanes x
    // 16 bits) at dbits[(dboff[cell] + target_in_cell * chunks + chunk) * 64 + lane] when
    // dboff[ncell_tot] * 64 <= dbits_cap, and the fill then reads them instead of testing
    const int64_t* dboff;
    uint16_t* dbits;
    int64_t dbits_cap;
};

hipError_t launch_count(const SearchArgs& a, int nblk_max, hipStream_t st);
hipError_t launch_fill(const SearchArgs& a, int nblk_max, hipStream_t st);
hipError_t launch_long_rows(const SearchArgs& a, int grid, hipStream_t st);
hipError_t launch_dense(const SearchArgs& a, bool fill, hipStream_t st);
hipError_t launch_stats(const SearchArgs& a, hipStream_t st);

}  // namespace nnps
