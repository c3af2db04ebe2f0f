// Cell build: FP64 cell assignment with a slot per particle in its cell, cell starts by a
// device-wide scan, a counting sort by cell, the FP16 relative-coordinate pack and the
// work-block table (the LDS radix sort serves the dense-cell lists).
//
// Paper: cell link list with cell size equal to the search radius (SPH method
// section, Fig. 3b); cell-relative coordinates (Eq. 5-6, Fig. 5); spatial sorting
// so that neighbouring threads work on neighbouring particles (Results, memory
// section and Table 6).
#include <algorithm>
#include <utility>

#include "build_kernels.h"

namespace nnps {

// ---------------------------------------------------------------------------
// Exact int64 -> float32 (one rounding) for |v| < 2^44: v = hi*2^20 + lo with
// hi exactly representable, lo < 2^20, and a single fused multiply-add rounds once.
__device__ __forceinline__ float exact_i64_to_f32(int64_t v)
{
    const int32_t hi = static_cast<int32_t>(v >> 20);
    const int32_t lo = static_cast<int32_t>(v & 0xFFFFF);
    return __builtin_fmaf(static_cast<float>(hi), 1048576.0f, static_cast<float>(lo));
}

// ---------------------------------------------------------------------------
// A1: cell assignment in FP64. X = rint((p - lo) * 2^F / w) (round half to even; an
// integer below 2^52, stored exactly as a double per particle with stride x_stride, so
// differences of two X are exact in binary64), cell = X >> F, global key = coff + cx + ncx (cy +
// ncy cz). Positions outside [lo, hi] (or NaN) raise the domain flag and are treated as
// lo so every index stays in range. Each particle also takes a slot in its cell (the
// cell's count before it), which places it in the sort by cell: runs of consecutive
// lanes with the same cell take their slots with one atomic, in lane order.
template <int DIM>
__global__ void __launch_bounds__(256)
k_assign(const SetDesc* __restrict__ sets, const int* __restrict__ poffs, int nsets, int ntot,
         double* __restrict__ X, uint32_t* __restrict__ key, int* __restrict__ slot, int* __restrict__ cell_count,
         int* __restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    bool bad = false;
    auto cell_of = [&](const SetDesc& sd) -> uint32_t {
        const Frame& fr = sd.fr;
        const int li = i - sd.poff;
        int64_t c[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double p = sd.pos[static_cast<size_t>(li) * DIM + k];
            if (!(p >= fr.lo[k] && p <= fr.hi[k])) {
                bad = true;
                p = fr.lo[k];
            }
            const double d = __dsub_rn(p, fr.lo[k]);
            const double t = rint(__dmul_rn(d, fr.s));  // an integer below 2^52
            X[static_cast<size_t>(i) * x_stride(DIM) + k] = t;
            c[k] = static_cast<int64_t>(t) >> fr.F;
        }
        return static_cast<uint32_t>(sd.coff + c[0] + fr.nc[0] * (c[1] + fr.nc[1] * c[2]));
    };
    // a wavefront inside one set reads the set's fields with scalar loads
    const int s = find_set(poffs, nsets, i);
    const int s0 = __builtin_amdgcn_readfirstlane(s);
    const uint32_t kk = __all(s == s0) ? cell_of(sets[s0]) : cell_of(sets[s]);
    key[i] = kk;
    // the active lanes are a prefix of the wavefront (i = base + lane, tail lanes returned)
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(static_cast<int>(kk), 1, 64);
    const uint64_t heads = __ballot(lane == 0 || static_cast<uint32_t>(prev) != kk);
    const int nact = __popcll(__ballot(1));
    const uint64_t upto = lane == 63 ? ~0ull : (2ull << lane) - 1ull;
    const int head = 63 - __clzll(heads & upto);  // first lane of this lane's run
    const uint64_t after = heads & ~upto;
    const int next = after ? __ffsll(static_cast<long long>(after)) - 1 : nact;
    int base = 0;
    if (head == lane) base = atomicAdd(&cell_count[kk], next - lane);
    slot[i] = __shfl(base, head, 64) + (lane - head);
    if (bad) atomicOr(err, kErrDomain);
}

// Counting sort by cell: particle i goes to cell_start[key] + slot.
__global__ void __launch_bounds__(256)
k_place(const uint32_t* __restrict__ key, const int* __restrict__ slot, const int* __restrict__ cell_start,
        int ntot, uint32_t* __restrict__ skey, int* __restrict__ perm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    const uint32_t kk = key[i];
    const int at = cell_start[kk] + slot[i];
    skey[at] = kk;
    perm[at] = i;
}

// Fill an int32 array with a value (a kernel rather than a memset node, so the sequence
// can be captured in a graph).
__global__ void __launch_bounds__(256)
k_fill_i32(int* __restrict__ p, int64_t m, int v)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < m;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// Two arrays in one launch.
__global__ void __launch_bounds__(256)
k_fill2_i32(int* __restrict__ p, int64_t m, int* __restrict__ q, int64_t k, int v)
{
    const int64_t i0 = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
    const int64_t step = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = i0; i < m; i += step) p[i] = v;
    for (int64_t i = i0; i < k; i += step) q[i] = v;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (int32 in, TOut out), three phases over tiles of
// kScanTile elements: tile sums, a scan of the tile sums, then each tile scanned
// with its offset. out[m] receives the total.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and the block total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* total, int64_t* sh /*[4]*/)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    int64_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        if (k < w) base += sh[k];
        tot += sh[k];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// A non-null `gate` pointing at 0 turns a scan kernel into a no-op (work that depends
// on a count known only on the device).
template <typename TIn>
__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const TIn* __restrict__ in, int64_t m, int64_t* __restrict__ partial, const int* gate)
{
    if (gate && *gate == 0) return;
    __shared__ int64_t sh[4];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    int64_t s = 0;
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t idx = base + r * kScanThreads + threadIdx.x;
        if (idx < m) s += static_cast<int64_t>(in[idx]);
    }
    int64_t tot;
    block_excl_scan(s, &tot, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One workgroup scans the tile sums in place (exclusive); partial[nt] = total.
__global__ void __launch_bounds__(kScanThreads)
k_scan_partials(int64_t* __restrict__ partial, int64_t nt, const int* gate)
{
    if (gate && *gate == 0) return;
    __shared__ int64_t sh[4];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < nt; b += kScanThreads) {
        const int64_t idx = b + threadIdx.x;
        const int64_t v = idx < nt ? partial[idx] : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan(v, &tot, sh);
        const int64_t c = carry;
        if (idx < nt) partial[idx] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[nt] = carry;
}

template <typename TIn, typename TOut>
__global__ void __launch_bounds__(kScanThreads)
k_scan_down(const TIn* __restrict__ in, int64_t m, const int64_t* __restrict__ partial,
            TOut* __restrict__ out, int64_t nt, const int* gate)
{
    if (gate && *gate == 0) return;
    __shared__ int64_t sh[4];
    // blocked layout: thread t owns kScanItems consecutive elements
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    TIn v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t idx = base + r;
        v[r] = idx < m ? in[idx] : TIn(0);
        s += static_cast<int64_t>(v[r]);
    }
    int64_t tot;
    int64_t run = block_excl_scan(s, &tot, sh) + partial[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t idx = base + r;
        if (idx < m) out[idx] = static_cast<TOut>(run);
        run += static_cast<int64_t>(v[r]);
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[m] = static_cast<TOut>(partial[nt]);
}

// The same final phase for up to kScanFold tiles, each workgroup summing the tile sums
// before its own (no separate scan of the tile sums; a single tile needs no tile sums).
constexpr int64_t kScanFold = 1024;

template <typename TIn, typename TOut>
__global__ void __launch_bounds__(kScanThreads)
k_scan_down_fold(const TIn* __restrict__ in, int64_t m, const int64_t* __restrict__ partial,
                 TOut* __restrict__ out, const int* gate)
{
    if (gate && *gate == 0) return;
    __shared__ int64_t sh[4];
    int64_t before = 0;
    for (int64_t t = threadIdx.x; t < blockIdx.x; t += kScanThreads) before += partial[t];
    int64_t offset;
    block_excl_scan(before, &offset, sh);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    TIn v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t idx = base + r;
        v[r] = idx < m ? in[idx] : TIn(0);
        s += static_cast<int64_t>(v[r]);
    }
    int64_t tot;
    int64_t run = block_excl_scan(s, &tot, sh) + offset;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t idx = base + r;
        if (idx < m) out[idx] = static_cast<TOut>(run);
        run += static_cast<int64_t>(v[r]);
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[m] = static_cast<TOut>(offset + tot);
}

template <typename T>
__global__ void k_zero_one(T* p) { *p = T(0); }

template <typename TIn, typename TOut>
hipError_t scan_exclusive(const TIn* in, int64_t m, TOut* out, int64_t* partial, hipStream_t st,
                          const int* gate = nullptr)
{
    const int64_t nt = (m + kScanTile - 1) / kScanTile;
    if (nt == 0) {
        // m == 0: out[0] = 0
        hipLaunchKernelGGL(k_zero_one<TOut>, dim3(1), dim3(1), 0, st, out);
        return hipGetLastError();
    }
    if (nt <= kScanFold) {
        if (nt > 1)
            hipLaunchKernelGGL(k_scan_reduce<TIn>, dim3(nt), dim3(kScanThreads), 0, st, in, m, partial, gate);
        hipLaunchKernelGGL((k_scan_down_fold<TIn, TOut>), dim3(nt), dim3(kScanThreads), 0, st, in, m, partial, out,
                           gate);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce<TIn>, dim3(nt), dim3(kScanThreads), 0, st, in, m, partial, gate);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, partial, nt, gate);
    hipLaunchKernelGGL((k_scan_down<TIn, TOut>), dim3(nt), dim3(kScanThreads), 0, st, in, m, partial,
                       out, nt, gate);
    return hipGetLastError();
}

int64_t scan_partials_needed(int64_t m) { return (m + kScanTile - 1) / kScanTile + 1; }

// ---------------------------------------------------------------------------
// A2: stable LSD radix sort of (key, index) pairs (the dense cells' union lists), up to
// 8 bits per pass. Tiles of kRsTile keys; each wave of a tile owns 1024 consecutive keys
// and ranks them 64 at a time: lanes holding the same digit find each other with one
// ballot per digit bit, and a per-wave LDS counter per digit keeps the order of rounds.
// Tile order, then wave, then round, then lane equals index order: the sort is stable.
// The tile is put in output order in LDS first, so a digit's run is written by
// consecutive threads.
constexpr int kRsThreads = 256;
constexpr int kRsRounds = 16;
constexpr int kRsTile = kRsThreads * kRsRounds;
constexpr int kRsMaxBits = 11;
// Digit width per pass: at most 8 bits, so a tile's keys fall into runs of 16 or more per
// digit on average and the scatter's stores fill whole cache lines (with 10- or 11-bit
// digits a tile has 2-4 keys per digit and nearly every store writes its own line).
constexpr int kRsPassBits = 8;

__global__ void __launch_bounds__(kRsThreads)
k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift, int bits,
             uint32_t* __restrict__ table, int ntiles, const int* ndev)
{
    // ndev: the number of keys is on the device (at most n; 0 skips the pass)
    if (ndev) {
        if (*ndev == 0) return;
        n = min(n, *ndev);
    }
    __shared__ uint32_t h[1 << kRsMaxBits];
    const int bins = 1 << bits;
    const uint32_t mask = bins - 1;
    for (int i = threadIdx.x; i < bins; i += kRsThreads) h[i] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRsTile;
    for (int r = 0; r < kRsRounds; ++r) {
        const int idx = base + r * kRsThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += kRsThreads) table[static_cast<size_t>(i) * ntiles + blockIdx.x] = h[i];
}

__global__ void __launch_bounds__(kRsThreads)
k_radix_scatter(const uint32_t* __restrict__ kin, const int* __restrict__ vin,
                uint32_t* __restrict__ kout, int* __restrict__ vout, int n, int shift, int bits,
                const uint32_t* __restrict__ offs, int ntiles, const int* ndev)
{
    if (ndev) {
        if (*ndev == 0) return;
        n = min(n, *ndev);
    }
    if (blockIdx.x * kRsTile >= n) return;  // a tile past the keys (the grid is sized for a bound)
    constexpr int MB = 1 << kRsPassBits;
    constexpr int NWV = kRsThreads / 64;
    static_assert(MB <= kRsThreads, "one thread per digit in the tile's digit scan");
    __shared__ uint32_t cw[NWV][MB];
    __shared__ uint32_t tstart[MB];  // the tile's first position of each digit
    __shared__ uint32_t wtot[NWV];
    __shared__ uint32_t sk[kRsTile];  // the tile's keys and values in output order
    __shared__ int sv[kRsTile];
    const int bins = 1 << bits;  // bits <= kRsPassBits
    const uint32_t mask = bins - 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < NWV * MB; i += kRsThreads) cw[i / MB][i % MB] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRsTile + w * (kRsRounds * 64);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t myk[kRsRounds];
    int myv[kRsRounds];
    uint32_t rank[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int idx = base + r * 64 + lane;
        const bool valid = idx < n;
        const uint32_t k = valid ? kin[idx] : 0u;
        const int v = valid ? (vin ? vin[idx] : idx) : 0;
        const uint32_t d = (k >> shift) & mask;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool set = (d >> b) & 1u;
            const uint64_t bb = __ballot(set);
            m &= set ? bb : ~bb;
        }
        const uint32_t rnk = __popcll(m & lt);
        const uint32_t cnt = __popcll(m);
        const uint32_t b0 = cw[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && rnk == 0) cw[w][d] = b0 + cnt;
        __builtin_amdgcn_wave_barrier();
        myk[r] = k;
        myv[r] = v;
        rank[r] = b0 + rnk;
    }
    __syncthreads();
    // per digit: each wavefront's offset inside the tile's run of that digit, and the run's
    // length; then the runs' starts (exclusive scan over the digits, one thread per digit)
    uint32_t len = 0;
    if (threadIdx.x < bins) {
#pragma unroll
        for (int k = 0; k < NWV; ++k) {
            const uint32_t t = cw[k][threadIdx.x];
            cw[k][threadIdx.x] = len;
            len += t;
        }
    }
    uint32_t inc = len;  // inclusive scan inside the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < w; ++k) before += wtot[k];
    if (threadIdx.x < bins) tstart[threadIdx.x] = before + inc - len;
    __syncthreads();
    // the tile in output order, in LDS
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const int idx = base + r * 64 + lane;
        if (idx < n) {
            const uint32_t d = (myk[r] >> shift) & mask;
            const uint32_t lp = tstart[d] + cw[w][d] + rank[r];
            sk[lp] = myk[r];
            sv[lp] = myv[r];
        }
    }
    __syncthreads();
    // consecutive threads write consecutive positions of a digit's run
    const int nvalid = min(kRsTile, n - static_cast<int>(blockIdx.x) * kRsTile);
    for (int i = threadIdx.x; i < nvalid; i += kRsThreads) {
        const uint32_t k = sk[i];
        const uint32_t d = (k >> shift) & mask;
        const uint32_t p = offs[static_cast<size_t>(d) * ntiles + blockIdx.x] + (static_cast<uint32_t>(i) - tstart[d]);
        kout[p] = k;
        vout[p] = sv[i];
    }
}

// ---------------------------------------------------------------------------
// A4: pack in sorted order. q_k = f16(f32(D_k) 2^(1-F)) with D_k = X_k - c_k 2^F - 2^(F-1),
// the Eq. 6 relative coordinate in [-1, 1]; the fourth half holds c_x mod 2^16.
// The FP64 baseline instead gets a sorted copy of the caller's positions.
template <int DIM>
__global__ void __launch_bounds__(256)
k_pack(const SetDesc* __restrict__ sets, const int* __restrict__ coffs, int nsets, int ntot,
       const uint32_t* __restrict__ skey, const int* __restrict__ perm, const double* __restrict__ X,
       ushort4* __restrict__ q4, double* __restrict__ spos, float4* __restrict__ rq, int* __restrict__ inv,
       uint32_t* __restrict__ skey_out, int* __restrict__ perm_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= ntot) return;
    const int o = perm[p];
    if (inv) inv[o] = p;
    // the incremental update places into a second pair of arrays: copied back here
    if (perm_out) {
        perm_out[p] = o;
        skey_out[p] = skey[p];
    }
    auto pack = [&](const SetDesc& sd) {
        const Frame& fr = sd.fr;
        if (spos) {
#pragma unroll
            for (int k = 0; k < DIM; ++k)
                spos[static_cast<size_t>(p) * 4 + k] = sd.pos[static_cast<size_t>(o - sd.poff) * DIM + k];
        }
        uint16_t h[4] = {0, 0, 0, 0};
        float q32[3] = {0.0f, 0.0f, 0.0f};
        uint32_t cbits = 0;
        const float scale = __builtin_ldexpf(1.0f, 1 - fr.F);
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            const int64_t x = static_cast<int64_t>(X[static_cast<size_t>(o) * x_stride(DIM) + k]);
            const int64_t c = x >> fr.F;
            const int64_t D = x - (c << fr.F) - (int64_t(1) << (fr.F - 1));
            q32[k] = exact_i64_to_f32(D) * scale;  // exact power-of-two scaling
            h[k] = __builtin_bit_cast(uint16_t, static_cast<_Float16>(q32[k]));
            if (k == 0) h[3] = static_cast<uint16_t>(c & 0xFFFF);
            cbits |= static_cast<uint32_t>(c & 1023) << (10 * k);
        }
        q4[p] = make_ushort4(h[0], h[1], h[2], h[3]);
        // FP32 mode: the coordinate in f32 and the cell indices mod 2^10 (a pair's cell
        // offsets are -1, 0 or 1 per axis, which their differences mod 2^10 recover)
        if (rq) rq[p] = make_float4(q32[0], q32[1], q32[2], __builtin_bit_cast(float, cbits));
    };
    // a wavefront inside one set reads the set's fields with scalar loads
    const int s = find_set(coffs, nsets, static_cast<int>(skey[p]));
    const int s0 = __builtin_amdgcn_readfirstlane(s);
    if (__all(s == s0)) pack(sets[s0]);
    else pack(sets[s]);
}

// ---------------------------------------------------------------------------
// Incremental update after the particles moved (Mixed-precision SPH framework section,
// Eq. 8-9, Fig. 6): a particle's relative coordinate advances by its displacement, and a
// particle leaving its cell migrates to the new one. Here the advance is made on the
// binary64 position (p = p + dp, one rounding, written back when a displacement array is
// given) and the fixed-point position and cell are recomputed from it exactly as the
// assignment computes them, so the relative coordinate carries no error from earlier
// steps and the structure equals a fresh build's up to the order inside cells. Only
// migrants are re-binned: the sorted order is kept, stayers keep their relative order in
// their cell, and each cell's migrants are appended after its stayers.

// U1 (per particle, in the caller's order so positions, displacements and fixed-point
// positions stream): move, recompute X and the cell. A displacement component that would
// take the particle out of [lo, hi] is applied with its sign flipped (a reflection at the
// box faces). A particle whose cell changed is a migrant: bit inv[i] of `mig` is set, it
// counts out of its old cell and takes an arrival slot in its new one. Every particle's
// new cell key is kept by particle index (knew).
template <int DIM>
__global__ void __launch_bounds__(256)
k_upd_move(const SetDesc* __restrict__ sets, const int* __restrict__ poffs, int nsets, int ntot,
           const uint32_t* __restrict__ skey, const int* __restrict__ inv, double* __restrict__ X,
           uint32_t* __restrict__ knew, uint32_t* __restrict__ mig, int* __restrict__ leave,
           int* __restrict__ arrive, int* __restrict__ aslot, int* __restrict__ err)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot) return;
    bool bad = false;
    auto cell_of = [&](const SetDesc& sd) -> uint32_t {
        // the set's fields in registers: read through the table they would be loaded again
        // after every store below (the compiler cannot tell the stores from the table)
        double lo[DIM], hi[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            lo[k] = sd.fr.lo[k];
            hi[k] = sd.fr.hi[k];
        }
        const double scale = sd.fr.s;
        const int F = sd.fr.F, ncx = sd.fr.nc[0], ncy = sd.fr.nc[1], coff = sd.coff;
        const int li = i - sd.poff;
        double* pos = const_cast<double*>(sd.pos);  // the caller lent them for the update
        const double* disp = sd.disp;
        double p[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) p[k] = pos[static_cast<size_t>(li) * DIM + k];
        if (disp) {
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                const double d = disp[static_cast<size_t>(li) * DIM + k];
                const double q = __dadd_rn(p[k], d);
                p[k] = (q >= lo[k] && q <= hi[k]) ? q : __dadd_rn(p[k], -d);
            }
#pragma unroll
            for (int k = 0; k < DIM; ++k) pos[static_cast<size_t>(li) * DIM + k] = p[k];
        }
        int64_t c[3] = {0, 0, 0};
        double t[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            double pk = p[k];
            if (!(pk >= lo[k] && pk <= hi[k])) {
                bad = true;
                pk = lo[k];
            }
            t[k] = rint(__dmul_rn(__dsub_rn(pk, lo[k]), scale));
            c[k] = static_cast<int64_t>(t[k]) >> F;
        }
#pragma unroll
        for (int k = 0; k < DIM; ++k) X[static_cast<size_t>(i) * x_stride(DIM) + k] = t[k];
        return static_cast<uint32_t>(coff + c[0] + ncx * (c[1] + ncy * c[2]));
    };
    // a wavefront inside one set reads the set's fields with scalar loads
    const int st = find_set(poffs, nsets, i);
    const int s0 = __builtin_amdgcn_readfirstlane(st);
    const uint32_t kn = __all(st == s0) ? cell_of(sets[s0]) : cell_of(sets[st]);
    knew[i] = kn;
    const int sp = inv[i];
    const uint32_t kold = skey[sp];
    if (kn != kold) {
        atomicOr(&mig[sp >> 5], 1u << (sp & 31));
        atomicAdd(&leave[kold], 1);
        aslot[i] = atomicAdd(&arrive[kn], 1);
    }
    if (bad) atomicOr(err, kErrDomain);
}

// U2 (per cell, and one more thread for the end): the new occupancy, old count - leavers
// + arrivals, as the scan's input, and a copy of the old cell starts (the scan writes the
// new ones in place).
__global__ void __launch_bounds__(256)
k_upd_counts(int ncell, const int* __restrict__ cell_start, const int* __restrict__ leave,
             const int* __restrict__ arrive, int* __restrict__ cnt, int* __restrict__ cs_old)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > ncell) return;
    const int a = cell_start[c];
    cs_old[c] = a;
    if (c < ncell) cnt[c] = cell_start[c + 1] - a - leave[c] + arrive[c];
}

// Set bits of `mig` at positions [a, b).
__device__ __forceinline__ int mig_bits(const uint32_t* __restrict__ mig, int a, int b)
{
    int n = 0;
    for (int w = a >> 5; (w << 5) < b; ++w) {
        uint32_t m = mig[w];
        const int lo = a - (w << 5), hi = b - (w << 5);  // bit range of this word, clipped below
        if (lo > 0) m &= ~0u << lo;
        if (hi < 32) m &= (1u << hi) - 1u;
        n += __builtin_popcount(m);
    }
    return n;
}

// U3 (per old sorted position s): the particle's new sorted position. A stayer keeps its
// rank among the stayers of its cell (its old offset less the leavers before it); a
// migrant goes after the stayers of its new cell, at its arrival slot.
__global__ void __launch_bounds__(256)
k_upd_place(int ntot, const uint32_t* __restrict__ skey, const int* __restrict__ perm,
            const uint32_t* __restrict__ knew, const uint32_t* __restrict__ mig, const int* __restrict__ leave,
            const int* __restrict__ aslot, const int* __restrict__ cs_old, const int* __restrict__ cs_new,
            uint32_t* __restrict__ skey2, int* __restrict__ perm2)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ntot) return;
    const int o = perm[s];
    const uint32_t kold = skey[s], kn = knew[o];
    int at;
    if (kn == kold) {
        const int a = cs_old[kold];
        const int lb = leave[kold] > 0 ? mig_bits(mig, a, s) : 0;
        at = cs_new[kold] + (s - a) - lb;
    } else {
        at = cs_new[kn] + (cs_old[kn + 1] - cs_old[kn] - leave[kn]) + aslot[o];
    }
    skey2[at] = kn;
    perm2[at] = o;
}

// ---------------------------------------------------------------------------
// Work blocks, one wavefront per segment of 64 cells of a row of cells of a set: walking
// the segment in x, a block is a run of at most fr.bmax consecutive sorted particles whose
// cells span at most fr.xwin cells; it starts where the previous one ended (so blocks are
// full unless the span, the segment or the row ends them). A run of dense cells (the
// dense-cell path's) is one block that the block kernels skip. The walk runs twice: the
// first counts each segment's blocks (nb[r]), the second, after an exclusive scan of the
// counts into boff, writes block boff[r] + j's first particle and set. Blocks come out in
// particle order, so block b ends where block b + 1 starts; bstart[total] = ntot.
constexpr int kRowSegment = 64;

template <bool WRITE>
__global__ void __launch_bounds__(256)
k_row_blocks(const SetDesc* __restrict__ sets, const int* __restrict__ roffs, int nsets, int nrows_tot, int ntot,
             const int* __restrict__ cell_start, const int* __restrict__ wdense, int* __restrict__ nb_or_boff,
             int* __restrict__ bstart, int* __restrict__ bset)
{
    const int r = blockIdx.x * (blockDim.x >> 6) + static_cast<int>(threadIdx.x >> 6);
    if (r >= nrows_tot) return;
    const int lane = threadIdx.x & 63;
    const int s = find_set(roffs, nsets, r);
    const SetDesc& sd = sets[s];
    const int ncx = sd.fr.nc[0];
    const int span = sd.fr.xwin;
    const int bmax = sd.fr.bmax;
    const int nseg = (ncx + kRowSegment - 1) / kRowSegment;
    const int rs = r - roffs[s];
    const int g0 = sd.coff + (rs / nseg) * ncx;
    const int base = (rs % nseg) * kRowSegment;
    const int b0 = WRITE ? nb_or_boff[r] : 0;
    if (WRITE && r == nrows_tot - 1 && lane == 0) bstart[nb_or_boff[nrows_tot]] = ntot;
    // wavefront-uniform walk state
    int bs = -1, xs = 0, nb = 0;
    bool dense_open = false;
    auto start = [&](int a) {
        if (WRITE && lane == 0) {
            bstart[b0 + nb] = a;
            bset[b0 + nb] = s;
        }
        ++nb;
    };
    {
        const int x = base + lane;
        int c0 = 0, c1 = 0, dn = 0;
        if (x < ncx) {
            c0 = cell_start[g0 + x];
            c1 = cell_start[g0 + x + 1];
            dn = wdense ? wdense[g0 + x] : 0;
        }
        const int m = min(kRowSegment, ncx - base);
        for (int i = 0; i < m; ++i) {
            const int a0 = __builtin_amdgcn_readlane(c0, i);
            const int a1 = __builtin_amdgcn_readlane(c1, i);
            const int ad = __builtin_amdgcn_readlane(dn, i);
            if (a1 == a0) continue;
            const int xx = base + i;
            if (ad) {
                if (bs < 0 || !dense_open) {
                    start(a0);
                    bs = a0;
                    dense_open = true;
                }
                continue;
            }
            if (bs < 0 || dense_open || xx - xs >= span) {
                start(a0);
                bs = a0;
                xs = xx;
                dense_open = false;
            }
            while (a1 - bs > bmax) {
                bs += bmax;
                start(bs);
                xs = xx;
            }
        }
    }
    if (!WRITE && lane == 0) nb_or_boff[r] = nb;
}

// Per-set CSR row pointers from the global exclusive scan of the counts (one thread per
// row boundary: set s has n_s + 1 of them), and each set's nnz.
__global__ void __launch_bounds__(256)
k_rowptr_scatter(const SetDesc* __restrict__ sets, const int* __restrict__ poffs, int nsets, int ntot,
                 const int64_t* __restrict__ rowg, int64_t* __restrict__ nnz, const int* __restrict__ inv,
                 int64_t* __restrict__ rsort)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntot + nsets) return;
    // boundary t belongs to the last set s with poffs[s] + s <= t
    int lo = 0, hi = nsets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (poffs[mid] + mid <= t) lo = mid;
        else hi = mid - 1;
    }
    const SetDesc& sd = sets[lo];
    const int i = t - (sd.poff + lo);  // 0 .. n_s
    const int64_t v = rowg[sd.poff + i] - rowg[sd.poff];
    if (sd.row_ptr) sd.row_ptr[i] = v;
    if (i == sd.fr.n) nnz[lo] = v;
    else rsort[inv[sd.poff + i]] = v;
}

// One set: its row pointers are the global exclusive scan of the counts, so the scan's
// final phase (as k_scan_down_fold) writes them, each particle's row start by sorted
// position, row_ptr[n] and nnz directly.
__global__ void __launch_bounds__(kScanThreads)
k_rowptr_fold1(const SetDesc* __restrict__ sets, const int* __restrict__ counts, int64_t m,
               const int64_t* __restrict__ partial, int64_t* __restrict__ nnz, const int* __restrict__ inv,
               int64_t* __restrict__ rsort)
{
    __shared__ int64_t sh[4];
    int64_t* row_ptr = sets[0].row_ptr;
    int64_t before = 0;
    for (int64_t t = threadIdx.x; t < blockIdx.x; t += kScanThreads) before += partial[t];
    int64_t offset;
    block_excl_scan(before, &offset, sh);
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t idx = base + r;
        v[r] = idx < m ? counts[idx] : 0;
        s += v[r];
    }
    int64_t tot;
    // the tile's exclusive prefixes pass through LDS, one pad entry per 16, so the writes
    // below go out lane by lane: coalesced row pointers and inverse-permutation reads
    __shared__ int64_t sloc[kScanTile + kScanTile / 16];
    int64_t run = block_excl_scan(s, &tot, sh);
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const int e = threadIdx.x * kScanItems + r;
        sloc[e + (e >> 4)] = run;
        run += v[r];
    }
    __syncthreads();
    const int64_t tile0 = static_cast<int64_t>(blockIdx.x) * kScanTile;
    for (int e = threadIdx.x; e < kScanTile; e += kScanThreads) {
        const int64_t idx = tile0 + e;
        if (idx < m) {
            const int64_t val = offset + sloc[e + (e >> 4)];
            if (row_ptr) row_ptr[idx] = val;
            rsort[inv[idx]] = val;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        if (row_ptr) row_ptr[m] = offset + tot;
        nnz[0] = offset + tot;
    }
}

// ---------------------------------------------------------------------------
// Dense-cell path tables. Where clustering piles hundreds or thousands of particles
// into a cell, every target of the cell tests the same stencil union, and its rows are
// long. A cell is dense when its stencil holds more than a threshold of particles. For such cells the search stages the union once per chunk for all the cell's
// targets, in ascending original index, so each row comes out sorted with no per-row
// sort. The union lists come from one stable sort: every particle, visited in original
// order, emits (dense cell, sorted position) for each dense cell whose stencil holds it.

// Global cell index -> local coordinates of its set.
struct CellXYZ {
    int x, y, z, ncx, ncy, ncz;
    __device__ __forceinline__ CellXYZ(const Frame& fr, int lk)
    {
        ncx = fr.nc[0];
        ncy = fr.nc[1];
        ncz = fr.nc[2];
        x = lk % ncx;
        const int row = lk / ncx;
        y = row % ncy;
        z = row / ncy;
    }
};

// Stencil size of every occupied cell; a cell is dense when it exceeds the threshold.
template <int DIM>
__global__ void __launch_bounds__(256)
k_dense_cells(const SetDesc* __restrict__ sets, const int* __restrict__ coffs, int nsets, int ncell_tot,
              const int* __restrict__ cell_start, int thresh, int* __restrict__ usz, int* __restrict__ wdense,
              int* __restrict__ seen)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ncell_tot) return;
    const SetDesc& sd = sets[find_set(coffs, nsets, g)];
    const CellXYZ c(sd.fr, g - sd.coff);
    const int* cs = cell_start + sd.coff;
    int u = 0;
    if (cell_start[g + 1] > cell_start[g]) {
        const int x0 = c.x > 0 ? c.x - 1 : 0;
        const int x1 = c.x + 1 < c.ncx ? c.x + 1 : c.ncx - 1;
        for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz) {
            const int zz = c.z + dz;
            if (zz < 0 || zz >= c.ncz) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = c.y + dy;
                if (yy < 0 || yy >= c.ncy) continue;
                const int rb = (zz * c.ncy + yy) * c.ncx;
                u += cs[rb + x1 + 1] - cs[rb + x0];
            }
        }
    }
    const bool dense = u > thresh;
    usz[g] = dense ? u : 0;
    wdense[g] = dense ? 1 : 0;
    if (dense) *seen = 1;  // every writer writes the same value
}

// After the scan of the stencil sizes: if the lists would not fit, the build falls back
// to the block path (every window normal); otherwise each dense cell gets its work
// units. dn receives the number of list entries in use (0 = path off).
__global__ void __launch_bounds__(256)
k_dense_units(int ncell_tot, const int* __restrict__ cell_start, const int64_t* __restrict__ uoff, int64_t cap,
              int* __restrict__ usz, int* __restrict__ wdense, int* __restrict__ nsl, int* __restrict__ dn,
              int* __restrict__ dbn)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ue = uoff[ncell_tot];
    const bool over = ue > cap;
    if (g == 0) *dn = over ? 0 : static_cast<int>(ue);
    if (g >= ncell_tot) return;
    if (over) {
        usz[g] = 0;
        wdense[g] = 0;
    }
    const int occ = cell_start[g + 1] - cell_start[g];
    const bool on = !over && usz[g] > 0;
    nsl[g] = on ? (occ + kDenseSlice - 1) / kDenseSlice : 0;
    dbn[g] = on ? occ * ((usz[g] + kDenseChunkF16 - 1) / kDenseChunkF16) : 0;
}

__global__ void __launch_bounds__(256)
k_dense_unit_cells(int ncell_tot, const int* __restrict__ nsl, const int* __restrict__ unit_off,
                   const int* __restrict__ dn, int* __restrict__ ucell)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ncell_tot || *dn == 0) return;
    const int k = nsl[g], u0 = unit_off[g];
    for (int s = 0; s < k; ++s) ucell[u0 + s] = g;
}

// Visit the dense cells whose stencil holds the particle at sorted position j. The 3^d
// stencil sizes are loaded together first (cells outside the grid read as 0), then the
// dense ones are visited in x-fastest order.
template <int DIM, typename F>
__device__ __forceinline__ void for_dense_stencils(const SetDesc* __restrict__ sets, const int* __restrict__ coffs,
                                                   int nsets, const uint32_t* __restrict__ skey,
                                                   const int* __restrict__ usz, int j, F&& f)
{
    constexpr int NS = DIM == 3 ? 27 : 9;
    const int gk = static_cast<int>(skey[j]);
    const SetDesc& sd = sets[find_set(coffs, nsets, gk)];
    const CellXYZ c(sd.fr, gk - sd.coff);
    int sz[NS];
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
        const int xx = c.x + dx, yy = c.y + dy, zz = c.z + dz;
        const bool in = xx >= 0 && xx < c.ncx && yy >= 0 && yy < c.ncy && zz >= 0 && zz < c.ncz;
        sz[t] = in ? usz[gk + dx + c.ncx * (dy + c.ncy * dz)] : 0;
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = DIM == 3 ? t / 9 - 1 : 0;
        if (sz[t] > 0) f(gk + dx + c.ncx * (dy + c.ncy * dz));
    }
}

template <int DIM>
__global__ void __launch_bounds__(256)
k_union_count(const SetDesc* __restrict__ sets, const int* __restrict__ coffs, int nsets, int ntot,
              const uint32_t* __restrict__ skey, const int* __restrict__ inv, const int* __restrict__ usz,
              const int* __restrict__ dn, int* __restrict__ ecnt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot || *dn == 0) return;
    int k = 0;
    for_dense_stencils<DIM>(sets, coffs, nsets, skey, usz, inv[i], [&](int) { ++k; });
    ecnt[i] = k;
}

template <int DIM>
__global__ void __launch_bounds__(256)
k_union_emit(const SetDesc* __restrict__ sets, const int* __restrict__ coffs, int nsets, int ntot,
             const uint32_t* __restrict__ skey, const int* __restrict__ inv, const int* __restrict__ usz,
             const int* __restrict__ dn, const int* __restrict__ epos, uint32_t* __restrict__ ukey,
             int* __restrict__ uval)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntot || *dn == 0) return;
    const int j = inv[i];
    int m = epos[i];
    for_dense_stencils<DIM>(sets, coffs, nsets, skey, usz, j, [&](int g2) {
        ukey[m] = static_cast<uint32_t>(g2);
        uval[m] = j;
        ++m;
    });
}

// ---------------------------------------------------------------------------
// Host-side launchers.
int row_segments(int ncx) { return (ncx + kRowSegment - 1) / kRowSegment; }

hipError_t launch_fill2_i32(int* p, int64_t m, int* q, int64_t k, int v, hipStream_t st)
{
    const int64_t n = std::max(m, k);
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill2_i32, dim3(blocks), dim3(256), 0, st, p, m, q, k, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t m, int v, hipStream_t st)
{
    if (m <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((m + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, st, p, m, v);
    return hipGetLastError();
}

hipError_t launch_place(int ntot, const uint32_t* key, const int* slot, const int* cell_start, uint32_t* skey,
                        int* perm, hipStream_t st)
{
    if (ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, dim3((ntot + 255) / 256), dim3(256), 0, st, key, slot, cell_start, ntot, skey, perm);
    return hipGetLastError();
}

hipError_t launch_assign(const Launch& L, double* X, uint32_t* key, int* slot, int* cell_count, int* err,
                         hipStream_t st)
{
    if (L.ntot == 0) return hipSuccess;
    const dim3 g((L.ntot + 255) / 256), b(256);
    if (L.dim == 2)
        hipLaunchKernelGGL(k_assign<2>, g, b, 0, st, L.sets, L.poffs, L.nsets, L.ntot, X, key, slot, cell_count, err);
    else
        hipLaunchKernelGGL(k_assign<3>, g, b, 0, st, L.sets, L.poffs, L.nsets, L.ntot, X, key, slot, cell_count, err);
    return hipGetLastError();
}

hipError_t launch_scan_i32_i32(const int* in, int64_t m, int* out, int64_t* partial, hipStream_t st)
{
    return scan_exclusive<int, int>(in, m, out, partial, st);
}

hipError_t launch_scan_i32_i64(const int* in, int64_t m, int64_t* out, int64_t* partial, hipStream_t st)
{
    return scan_exclusive<int, int64_t>(in, m, out, partial, st);
}

int radix_tiles(int n) { return (n + kRsTile - 1) / kRsTile; }

// Stable LSD sort of (key, value) pairs held in (k0, v0), with (k1, v1) as the second
// buffers; the number of pairs is read on the device (*ndev <= n; 0 skips the sort).
hipError_t radix_sort_kv_dev(int n, const int* ndev, int keybits, uint32_t* k0, int* v0, uint32_t* k1, int* v1,
                             uint32_t* table, int64_t* partial, hipStream_t st, uint32_t** kfinal, int** vfinal)
{
    const int ntiles = radix_tiles(n);
    const int passes = keybits <= 0 ? 1 : (keybits + kRsPassBits - 1) / kRsPassBits;
    const int bits = keybits <= 0 ? 1 : (keybits + passes - 1) / passes;
    if (bits > kRsPassBits) return hipErrorInvalidValue;  // cannot happen: passes fit the bound
    uint32_t *kin = k0, *kout = k1;
    int *vin = v0, *vout = v1;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * bits;
        hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kRsThreads), 0, st, kin, n, shift, bits,
                           table, ntiles, ndev);
        hipError_t e = scan_exclusive<uint32_t, uint32_t>(table, static_cast<int64_t>(ntiles) << bits,
                                                          table, partial, st, ndev);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kRsThreads), 0, st, kin, vin, kout,
                           vout, n, shift, bits, table, ntiles, ndev);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    *kfinal = kin;
    *vfinal = vin;
    return hipGetLastError();
}

size_t radix_table_entries(int n) { return static_cast<size_t>(radix_tiles(n)) << kRsMaxBits; }

hipError_t launch_pack(const Launch& L, const uint32_t* skey, const int* perm, const double* X, ushort4* q4,
                       double* spos, float4* rq, int* inv, hipStream_t st, uint32_t* skey_out, int* perm_out)
{
    if (L.ntot == 0) return hipSuccess;
    const dim3 g((L.ntot + 255) / 256), b(256);
    if (L.dim == 2)
        hipLaunchKernelGGL(k_pack<2>, g, b, 0, st, L.sets, L.coffs, L.nsets, L.ntot, skey, perm, X, q4, spos, rq, inv,
                           skey_out, perm_out);
    else
        hipLaunchKernelGGL(k_pack<3>, g, b, 0, st, L.sets, L.coffs, L.nsets, L.ntot, skey, perm, X, q4, spos, rq, inv,
                           skey_out, perm_out);
    return hipGetLastError();
}

hipError_t launch_update_move(const Launch& L, const uint32_t* skey, const int* inv, double* X, const Update& u,
                              int* err, hipStream_t st)
{
    if (L.ntot == 0) return hipSuccess;
    const dim3 g((L.ntot + 255) / 256), b(256);
    if (L.dim == 2)
        hipLaunchKernelGGL(k_upd_move<2>, g, b, 0, st, L.sets, L.poffs, L.nsets, L.ntot, skey, inv, X, u.knew, u.mig,
                           u.leave, u.arrive, u.aslot, err);
    else
        hipLaunchKernelGGL(k_upd_move<3>, g, b, 0, st, L.sets, L.poffs, L.nsets, L.ntot, skey, inv, X, u.knew, u.mig,
                           u.leave, u.arrive, u.aslot, err);
    return hipGetLastError();
}

hipError_t launch_update_cells(const Launch& L, int* cell_start, int* cnt, const Update& u, int64_t* partial,
                               hipStream_t st)
{
    const int nc = L.ncell_tot;
    hipLaunchKernelGGL(k_upd_counts, dim3((nc + 256) / 256), dim3(256), 0, st, nc, cell_start, u.leave, u.arrive,
                       cnt, u.cs_old);
    return scan_exclusive<int, int>(cnt, nc, cell_start, partial, st);
}

hipError_t launch_update_place(const Launch& L, const uint32_t* skey, const int* perm, const int* cell_start,
                               const Update& u, hipStream_t st)
{
    if (L.ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_upd_place, dim3((L.ntot + 255) / 256), dim3(256), 0, st, L.ntot, skey, perm, u.knew,
                       u.mig, u.leave, u.aslot, u.cs_old, cell_start, u.skey2, u.perm2);
    return hipGetLastError();
}

hipError_t launch_blocks(const Launch& L, const int* cell_start, const int* wdense, int* boff, int* bstart, int* bset,
                         int64_t* partial, hipStream_t st)
{
    if (L.ntot == 0) return launch_fill_i32(boff, static_cast<int64_t>(L.nrows_tot) + 1, 0, st);
    const dim3 g((L.nrows_tot + 3) / 4), b(256);
    hipLaunchKernelGGL(k_row_blocks<false>, g, b, 0, st, L.sets, L.roffs, L.nsets, L.nrows_tot, L.ntot, cell_start,
                       wdense, boff, bstart, bset);
    hipError_t e = scan_exclusive<int, int>(boff, L.nrows_tot, boff, partial, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_row_blocks<true>, g, b, 0, st, L.sets, L.roffs, L.nsets, L.nrows_tot, L.ntot, cell_start,
                       wdense, boff, bstart, bset);
    return hipGetLastError();
}

hipError_t launch_dense_detect(const Launch& L, const int* cell_start, const DenseBuild& d, hipStream_t st)
{
    const int nc = L.ncell_tot;
    hipError_t e = launch_fill_i32(d.seen, 1, 0, st);
    if (e != hipSuccess) return e;
    const dim3 g((nc + 255) / 256), b(256);
    if (L.dim == 2)
        hipLaunchKernelGGL(k_dense_cells<2>, g, b, 0, st, L.sets, L.coffs, L.nsets, nc, cell_start, d.thresh, d.usz,
                           d.wdense, d.seen);
    else
        hipLaunchKernelGGL(k_dense_cells<3>, g, b, 0, st, L.sets, L.coffs, L.nsets, nc, cell_start, d.thresh, d.usz,
                           d.wdense, d.seen);
    return hipGetLastError();
}

hipError_t launch_dense_cells(const Launch& L, const int* cell_start, const DenseBuild& d, hipStream_t st)
{
    const int nc = L.ncell_tot;
    const dim3 g((nc + 255) / 256), b(256);
    hipError_t e = launch_dense_detect(L, cell_start, d, st);
    if (e != hipSuccess) return e;
    e = scan_exclusive<int, int64_t>(d.usz, nc, d.uoff, d.partial, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dense_units, dim3((nc + 256) / 256), b, 0, st, nc, cell_start, d.uoff, d.cap, d.usz,
                       d.wdense, d.nsl, d.dn, d.dbn);
    e = scan_exclusive<int, int>(d.nsl, nc, d.unit_off, d.partial, st);
    if (e != hipSuccess) return e;
    e = scan_exclusive<int, int64_t>(d.dbn, nc, d.dboff, d.partial, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dense_unit_cells, g, b, 0, st, nc, d.nsl, d.unit_off, d.dn, d.ucell);
    return hipGetLastError();
}

hipError_t launch_dense_unions(const Launch& L, const uint32_t* skey, const int* inv, const DenseBuild& d,
                               hipStream_t st, int** ulist)
{
    *ulist = d.uv0;
    if (L.ntot == 0 || d.cap == 0) return hipSuccess;
    const dim3 g((L.ntot + 255) / 256), b(256);
    if (L.dim == 2)
        hipLaunchKernelGGL(k_union_count<2>, g, b, 0, st, L.sets, L.coffs, L.nsets, L.ntot, skey, inv, d.usz, d.dn,
                           d.ecnt);
    else
        hipLaunchKernelGGL(k_union_count<3>, g, b, 0, st, L.sets, L.coffs, L.nsets, L.ntot, skey, inv, d.usz, d.dn,
                           d.ecnt);
    hipError_t e = scan_exclusive<int, int>(d.ecnt, L.ntot, d.epos, d.partial, st, d.dn);
    if (e != hipSuccess) return e;
    if (L.dim == 2)
        hipLaunchKernelGGL(k_union_emit<2>, g, b, 0, st, L.sets, L.coffs, L.nsets, L.ntot, skey, inv, d.usz, d.dn,
                           d.epos, d.uk0, d.uv0);
    else
        hipLaunchKernelGGL(k_union_emit<3>, g, b, 0, st, L.sets, L.coffs, L.nsets, L.ntot, skey, inv, d.usz, d.dn,
                           d.epos, d.uk0, d.uv0);
    const int keybits = std::max(1, 32 - __builtin_clz(static_cast<unsigned>(std::max(L.ncell_tot - 1, 1))));
    uint32_t* kf = nullptr;
    e = radix_sort_kv_dev(static_cast<int>(d.cap), d.dn, keybits, d.uk0, d.uv0, d.uk1, d.uv1, d.table, d.partial,
                          st, &kf, ulist);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_rowptr(const Launch& L, const int* counts, int64_t* rowg, int64_t* partial, int64_t* nnz,
                         const int* inv, int64_t* rsort, hipStream_t st)
{
    const int64_t nt = (static_cast<int64_t>(L.ntot) + kScanTile - 1) / kScanTile;
    if (L.nsets == 1 && nt >= 1 && nt <= kScanFold) {
        if (nt > 1)
            hipLaunchKernelGGL(k_scan_reduce<int>, dim3(nt), dim3(kScanThreads), 0, st, counts,
                               static_cast<int64_t>(L.ntot), partial, nullptr);
        hipLaunchKernelGGL(k_rowptr_fold1, dim3(nt), dim3(kScanThreads), 0, st, L.sets, counts,
                           static_cast<int64_t>(L.ntot), partial, nnz, inv, rsort);
        return hipGetLastError();
    }
    hipError_t e = scan_exclusive<int, int64_t>(counts, L.ntot, rowg, partial, st);
    if (e != hipSuccess) return e;
    const int m = L.ntot + L.nsets;
    hipLaunchKernelGGL(k_rowptr_scatter, dim3((m + 255) / 256), dim3(256), 0, st, L.sets, L.poffs, L.nsets,
                       L.ntot, rowg, nnz, inv, rsort);
    return hipGetLastError();
}

}  // namespace nnps
