// Neighbour search over the sorted cell structure: the 3^d-cell stencil test in
// packed FP16 (relative coordinates, Eq. 6-7 with the factor 1/2 Eq. 7 drops), the
// FP64 guard-band recheck, the count pass and the fill pass with per-row ascending
// order and wave-cooperative CSR writes; plus the plain FP64 cell-list baseline.
//
// Work decomposition: a block is one wavefront of up to 64 consecutive sorted targets
// inside one (y, z) row of cells. Cells along x are contiguous in sorted order, so a
// target's candidates are 3^(d-1) contiguous runs ("row segments"), one per (dy, dz),
// each covering cells x-1..x+1. The block stages the union of its row segments in LDS
// (chunks of kStage positions) as pair records: two candidates' x, y, z and 2(c_x - base)
// per 16 bytes, so one packed-FP16 instruction tests two candidates.
#include "build_kernels.h"

namespace nnps {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2 as_h2(uint32_t u) { return __builtin_bit_cast(h2, u); }
__device__ __forceinline__ uint32_t as_u32(h2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ _Float16 as_f16(uint16_t u) { return __builtin_bit_cast(_Float16, u); }
__device__ __forceinline__ h2 splat(_Float16 v) { return h2{v, v}; }

__device__ __forceinline__ float exact_i64_to_f32_s(int64_t v)
{
    const int32_t hi = static_cast<int32_t>(v >> 20);
    const int32_t lo = static_cast<int32_t>(v & 0xFFFFF);
    return __builtin_fmaf(static_cast<float>(hi), 1048576.0f, static_cast<float>(lo));
}

// The binary64 predicate, in the fixed order and with no contraction.
template <int DIM>
__device__ __forceinline__ double r2_fp64(const double* pi, const double* pj)
{
    const double d0 = __dsub_rn(pj[0], pi[0]);
    const double d1 = __dsub_rn(pj[1], pi[1]);
    double r2 = __dmul_rn(d0, d0);
    r2 = __dadd_rn(r2, __dmul_rn(d1, d1));
    if (DIM == 3) {
        const double d2 = __dsub_rn(pj[2], pi[2]);
        r2 = __dadd_rn(r2, __dmul_rn(d2, d2));
    }
    return r2;
}

template <int DIM>
__device__ __forceinline__ bool recheck(const double* __restrict__ pos, const double* pi, int oj,
                                        double R2)
{
    double pj[3];
#pragma unroll
    for (int k = 0; k < DIM; ++k) pj[k] = pos[static_cast<size_t>(oj) * DIM + k];
    return r2_fp64<DIM>(pi, pj) <= R2;
}

// FP32 distance from the fixed-point positions: the int64 displacement is exact and
// is rounded once to FP32 (|dX| < 2^41 for any pair within the radius).
template <int DIM>
__device__ __forceinline__ float dist_fixed(const int64_t* __restrict__ X, int n, int oi, int oj,
                                           float scale)
{
    float s2 = 0.0f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const int64_t d = X[static_cast<size_t>(k) * n + oj] - X[static_cast<size_t>(k) * n + oi];
        const float f = exact_i64_to_f32_s(d);
        s2 = s2 + f * f;
    }
    return __builtin_sqrtf(s2) * scale;
}

template <int DIM>
__device__ __forceinline__ float dist_fp64(const double* __restrict__ pos, int oi, int oj)
{
    double pi[3], pj[3];
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        pi[k] = pos[static_cast<size_t>(oi) * DIM + k];
        pj[k] = pos[static_cast<size_t>(oj) * DIM + k];
    }
    return static_cast<float>(__dsqrt_rn(r2_fp64<DIM>(pi, pj)));
}

__device__ __forceinline__ int wave_excl_scan_i32(int v, int* total)
{
    const int lane = threadIdx.x & 63;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    *total = __shfl(inc, 63, 64);
    return inc - v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Geometry of one block and of one lane's row segments.
template <int DIM>
struct Geom {
    static constexpr int NSEG = DIM == 3 ? 9 : 3;
    static constexpr int SELF = DIM == 3 ? 4 : 1;  // segment with dy = dz = 0
    int p0, p1, p;
    bool active;
    int x, sx0;
    int U;
    int seg_g0[NSEG], seg_base[NSEG], la[NSEG], lb[NSEG];
    int pself;

    __device__ __forceinline__ void init(const SearchArgs& a, int b)
    {
        const Frame& fr = a.fr;
        const int lane = threadIdx.x & 63;
        p0 = a.bstart[b];
        p1 = a.bstart[b + 1];
        p = p0 + lane;
        active = p < p1;
        const uint32_t ncx = static_cast<uint32_t>(fr.nc[0]);
        const int ncy = fr.nc[1], ncz = fr.nc[2];
        const uint32_t k0 = a.skey[p0];
        const uint32_t row0 = k0 / ncx;
        const int xa = static_cast<int>(k0 - row0 * ncx);
        const int y0 = static_cast<int>(row0 % static_cast<uint32_t>(ncy));
        const int z0 = static_cast<int>(row0 / static_cast<uint32_t>(ncy));
        const uint32_t kl = a.skey[p1 - 1];
        const int xb = static_cast<int>(kl - (kl / ncx) * ncx);
        const uint32_t mk = a.skey[active ? p : p1 - 1];
        x = static_cast<int>(mk - (mk / ncx) * ncx);
        sx0 = xa > 0 ? xa - 1 : 0;
        const int sx1 = xb + 1 < static_cast<int>(ncx) ? xb + 1 : static_cast<int>(ncx) - 1;
        const int lx0 = x > 0 ? x - 1 : 0;
        const int lx1 = x + 1 < static_cast<int>(ncx) ? x + 1 : static_cast<int>(ncx) - 1;
        U = 0;
#pragma unroll
        for (int r = 0; r < NSEG; ++r) {
            const int dy = r % 3 - 1;
            const int dz = DIM == 3 ? r / 3 - 1 : 0;
            const int yy = y0 + dy, zz = z0 + dz;
            int g0 = 0, g1 = 0, ga = 0, gb = 0;
            if (yy >= 0 && yy < ncy && zz >= 0 && zz < ncz) {
                const int rb = (zz * ncy + yy) * static_cast<int>(ncx);
                g0 = a.cell_start[rb + sx0];
                g1 = a.cell_start[rb + sx1 + 1];
                ga = a.cell_start[rb + lx0];
                gb = a.cell_start[rb + lx1 + 1];
            }
            seg_g0[r] = g0;
            seg_base[r] = U;
            la[r] = U + (ga - g0);
            lb[r] = U + (gb - g0);
            U += g1 - g0;
        }
        pself = seg_base[SELF] + (p - seg_g0[SELF]);
    }

    // global sorted index of a logical (staged) position
    __device__ __forceinline__ int global_of(int r, int posl) const { return posl - seg_base[r] + seg_g0[r]; }

    __device__ __forceinline__ int global_of_any(int posl) const
    {
        int r = 0;
#pragma unroll
        for (int k = 1; k < NSEG; ++k)
            if (posl >= seg_base[k]) r = k;
        return global_of(r, posl);
    }
};

// Stage logical positions [cb, ce) as pair records; with ORIG also the original indices.
template <int DIM, bool ORIG>
__device__ __forceinline__ void stage(const SearchArgs& a, const Geom<DIM>& g, int cb, int ce,
                                      uint4* srec, int* sorig)
{
    const int lane = threadIdx.x & 63;
    const int m0 = cb >> 1, m1 = (ce + 1) >> 1;
    const uint16_t base16 = static_cast<uint16_t>(g.sx0 & 0xFFFF);
    for (int m = m0 + lane; m < m1; m += 64) {
        uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int posl = 2 * m + h;
            if (posl < ce) {
                const int gi = g.global_of_any(posl);
                const ushort4 v = a.q4[gi];
                const uint16_t rel = static_cast<uint16_t>(v.w - base16);
                const _Float16 cx2 = static_cast<_Float16>(2 * static_cast<int>(rel));
                const uint32_t sh = 16u * h;
                w0 |= static_cast<uint32_t>(v.x) << sh;
                w1 |= static_cast<uint32_t>(v.y) << sh;
                w2 |= static_cast<uint32_t>(v.z) << sh;
                w3 |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, cx2)) << sh;
                if (ORIG) sorig[posl - cb] = a.perm[gi];
            }
        }
        srec[m - m0] = make_uint4(w0, w1, w2, w3);
    }
}

// Per-lane constants of the FP16 test for row segment r.
template <int DIM>
struct Target16 {
    h2 qix, cx2i;
    _Float16 qiy, qiz;
    __device__ __forceinline__ void init(const ushort4& qi, int x, int sx0)
    {
        qix = splat(as_f16(qi.x));
        qiy = as_f16(qi.y);
        qiz = as_f16(qi.z);
        cx2i = splat(static_cast<_Float16>(2 * (x - sx0)));
    }
};

// The packed FP16 r2 for the pair record `rec` (two candidates); ay, az are
// RN16(q_i,y + 2dc_y), RN16(q_i,z + 2dc_z) for the segment.
template <int DIM>
__device__ __forceinline__ uint32_t r2_pair(const Target16<DIM>& t, h2 ay, h2 az, const uint4& rec)
{
    const h2 s = t.qix - as_h2(rec.x);
    const h2 dcx2 = t.cx2i - as_h2(rec.w);
    const h2 tx = s + dcx2;
    const h2 ty = ay - as_h2(rec.y);
    h2 r2;
    if (DIM == 3) {
        const h2 tz = az - as_h2(rec.z);
        r2 = tz * tz;
        r2 = __builtin_elementwise_fma(ty, ty, r2);
    } else {
        r2 = ty * ty;
    }
    r2 = __builtin_elementwise_fma(tx, tx, r2);
    return as_u32(r2);
}

struct Tally {
    int cnt = 0;
    unsigned long long cand = 0, band = 0, fpos = 0, fneg = 0, odis = 0;
};

// Classify one candidate (FP16 bits r2h at staged position posl of segment r);
// returns whether j is a neighbour. MODE 0: three-way test with FP64 recheck in the
// band; MODE 2: FP64 decides every candidate.
template <int DIM, int MODE>
__device__ __forceinline__ bool classify(const SearchArgs& a, const Geom<DIM>& g, const double* pi,
                                         int r, int posl, uint32_t r2h, Tally& t, const int* sorig,
                                         int cb, int* oj_out)
{
    const Frame& fr = a.fr;
    t.cand++;
    const bool in16 = r2h < fr.t_lo;
    const bool band = !in16 && r2h <= fr.t_hi;
    bool nb;
    int oj = -1;
    if (MODE == 2 || band) {
        oj = sorig ? sorig[posl - cb] : a.perm[g.global_of(r, posl)];
        const bool truth = recheck<DIM>(a.pos, pi, oj, fr.R2);
        const bool naive = r2h <= fr.t_mid;
        t.band += band;
        t.fpos += naive && !truth;
        t.fneg += !naive && truth;
        if (MODE == 2) t.odis += !band && (in16 != truth);
        nb = truth;
    } else {
        nb = in16;
    }
    if (nb && oj < 0 && sorig) oj = sorig[posl - cb];
    *oj_out = oj;
    return nb;
}

// ---------------------------------------------------------------------------
// Count pass (FP16 modes).
template <int DIM, int MODE>
__global__ void __launch_bounds__(64)
k_count16(SearchArgs a)
{
    __shared__ uint4 srec[kStage / 2];
    const int b = blockIdx.x;
    if (b >= *a.nblk) return;
    Geom<DIM> g;
    g.init(a, b);
    const Frame& fr = a.fr;
    const int pp = g.active ? g.p : g.p1 - 1;
    const int oi = a.perm[pp];
    double pi[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) pi[k] = a.pos[static_cast<size_t>(oi) * DIM + k];
    Target16<DIM> tg;
    tg.init(a.q4[pp], g.x, g.sx0);
    Tally t;
    for (int cb = 0; cb < g.U; cb += kStage) {
        const int ce = min(g.U, cb + kStage);
        __syncthreads();
        stage<DIM, false>(a, g, cb, ce, srec, nullptr);
        __syncthreads();
        if (!g.active) continue;
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
            const int lo = max(g.la[r], cb), hi = min(g.lb[r], ce);
            if (lo >= hi) continue;
            const int dy = r % 3 - 1, dz = DIM == 3 ? r / 3 - 1 : 0;
            const h2 ay = splat(tg.qiy + static_cast<_Float16>(-2 * dy));
            const h2 az = splat(tg.qiz + static_cast<_Float16>(-2 * dz));
            const int selfp = (r == Geom<DIM>::SELF) ? g.pself : -1;
            for (int m = lo >> 1; m < (hi + 1) >> 1; ++m) {
                const uint4 rec = srec[m - (cb >> 1)];
                const uint32_t rb = r2_pair<DIM>(tg, ay, az, rec);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int posl = 2 * m + h;
                    if (posl < lo || posl >= hi || posl == selfp) continue;
                    int oj;
                    t.cnt += classify<DIM, MODE>(a, g, pi, r, posl, (rb >> (16 * h)) & 0xFFFF, t,
                                                 nullptr, cb, &oj);
                }
            }
        }
    }
    if (g.active) a.counts[oi] = t.cnt;
    unsigned long long v[5] = {t.cand, t.band, t.fpos, t.fneg, t.odis};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const unsigned long long s = wave_sum_u64(v[k]);
        if ((threadIdx.x & 63) == 0 && s) atomicAdd(&a.stats[k], s);
    }
}

// Count pass, plain FP64 baseline: one lane per target, global FP64 loads.
template <int DIM>
__global__ void __launch_bounds__(64)
k_count64(SearchArgs a)
{
    const int b = blockIdx.x;
    if (b >= *a.nblk) return;
    Geom<DIM> g;
    g.init(a, b);
    const Frame& fr = a.fr;
    int cnt = 0;
    unsigned long long cand = 0;
    if (g.active) {
        const double* pi = a.spos + static_cast<size_t>(g.p) * 4;
        const double pix[3] = {pi[0], pi[1], DIM == 3 ? pi[2] : 0.0};
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
            const int ga = g.global_of(r, g.la[r]), gb = g.global_of(r, g.lb[r]);
            for (int j = ga; j < gb; ++j) {
                if (j == g.p) continue;
                const double* pj = a.spos + static_cast<size_t>(j) * 4;
                cnt += r2_fp64<DIM>(pix, pj) <= fr.R2;
                cand++;
            }
        }
        a.counts[a.perm[g.p]] = cnt;
    }
    const unsigned long long s = wave_sum_u64(cand);
    if ((threadIdx.x & 63) == 0) atomicAdd(&a.stats[kStCandidates], s);
}

// ---------------------------------------------------------------------------
// Fill pass helpers: per-lane row buffers in LDS, sorted by insertion, then written
// cooperatively: the wave walks the concatenation of its 64 rows, 64 entries at a time,
// so consecutive lanes store consecutive CSR slots.
template <int CAP>
__device__ __forceinline__ void lane_sort(int* lst, int len)
{
    for (int i = 1; i < len; ++i) {
        const int v = lst[i];
        int k = i - 1;
        while (k >= 0 && lst[k] > v) {
            lst[k + 1] = lst[k];
            --k;
        }
        lst[k + 1] = v;
    }
}

template <int DIM, int MODE, int CAP>
__device__ __forceinline__ void emit_rows(const SearchArgs& a, int* lists, int mylen, bool mine,
                                          int oi, int* soff, long long* srow, int* soi)
{
    const int lane = threadIdx.x & 63;
    int E;
    const int off = wave_excl_scan_i32(mine ? mylen : 0, &E);
    soff[lane] = off;
    if (lane == 63) soff[64] = E;
    srow[lane] = mine ? a.row_ptr[oi] : 0;
    soi[lane] = oi;
    __syncthreads();
    for (int e0 = 0; e0 < E; e0 += 64) {
        const int e = e0 + lane;
        if (e >= E) break;
        int lo = 0, hi = 63;  // largest t with soff[t] <= e
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (soff[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int t = lo;
        const int k = e - soff[t];
        const int oj = lists[t * (CAP + 1) + k];
        const int ot = soi[t];
        float d;
        if (MODE == 1) d = dist_fp64<DIM>(a.pos, ot, oj);
        else d = dist_fixed<DIM>(a.X, a.fr.n, ot, oj, a.fr.dist_scale);
        const long long idx = srow[t] + k;
        if (idx < a.capacity) {
            a.col[idx] = oj;
            a.dist[idx] = d;
        } else {
            atomicOr(a.err, kErrCapacity);
        }
    }
}

template <int DIM, int MODE>
__global__ void __launch_bounds__(64)
k_fill16(SearchArgs a)
{
    constexpr int CAP = DIM == 3 ? kCap3 : kCap2;
    __shared__ uint4 srec[kStage / 2];
    __shared__ int sorig[kStage];
    __shared__ int lists[64 * (CAP + 1)];
    __shared__ int soff[65];
    __shared__ long long srow[64];
    __shared__ int soi[64];
    const int b = blockIdx.x;
    if (b >= *a.nblk) return;
    const int lane = threadIdx.x & 63;
    Geom<DIM> g;
    g.init(a, b);
    const Frame& fr = a.fr;
    const int pp = g.active ? g.p : g.p1 - 1;
    const int oi = a.perm[pp];
    const long long rlen = g.active ? a.row_ptr[oi + 1] - a.row_ptr[oi] : 0;
    const bool heavy = g.active && rlen > CAP;
    const bool work = g.active && !heavy;
    if (heavy) {
        const int h = atomicAdd(a.nheavy, 1);
        a.heavy[h] = g.p;
    }
    double pi[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) pi[k] = a.pos[static_cast<size_t>(oi) * DIM + k];
    Target16<DIM> tg;
    tg.init(a.q4[pp], g.x, g.sx0);
    int* lst = lists + lane * (CAP + 1);
    int len = 0;
    Tally t;
    for (int cb = 0; cb < g.U; cb += kStage) {
        const int ce = min(g.U, cb + kStage);
        __syncthreads();
        stage<DIM, true>(a, g, cb, ce, srec, sorig);
        __syncthreads();
        if (!work) continue;
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
            const int lo = max(g.la[r], cb), hi = min(g.lb[r], ce);
            if (lo >= hi) continue;
            const int dy = r % 3 - 1, dz = DIM == 3 ? r / 3 - 1 : 0;
            const h2 ay = splat(tg.qiy + static_cast<_Float16>(-2 * dy));
            const h2 az = splat(tg.qiz + static_cast<_Float16>(-2 * dz));
            const int selfp = (r == Geom<DIM>::SELF) ? g.pself : -1;
            for (int m = lo >> 1; m < (hi + 1) >> 1; ++m) {
                const uint4 rec = srec[m - (cb >> 1)];
                const uint32_t rb = r2_pair<DIM>(tg, ay, az, rec);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int posl = 2 * m + h;
                    if (posl < lo || posl >= hi || posl == selfp) continue;
                    int oj;
                    if (classify<DIM, MODE>(a, g, pi, r, posl, (rb >> (16 * h)) & 0xFFFF, t, sorig, cb,
                                            &oj)) {
                        if (len < CAP) lst[len] = oj;
                        ++len;
                    }
                }
            }
        }
    }
    if (work && len != rlen) atomicOr(a.err, kErrLongRow);
    if (work) lane_sort<CAP>(lst, len < CAP ? len : CAP);
    emit_rows<DIM, MODE, CAP>(a, lists, len < CAP ? len : CAP, work, oi, soff, srow, soi);
}

template <int DIM>
__global__ void __launch_bounds__(64)
k_fill64(SearchArgs a)
{
    constexpr int CAP = DIM == 3 ? kCap3 : kCap2;
    __shared__ int lists[64 * (CAP + 1)];
    __shared__ int soff[65];
    __shared__ long long srow[64];
    __shared__ int soi[64];
    const int b = blockIdx.x;
    if (b >= *a.nblk) return;
    const int lane = threadIdx.x & 63;
    Geom<DIM> g;
    g.init(a, b);
    const Frame& fr = a.fr;
    const int pp = g.active ? g.p : g.p1 - 1;
    const int oi = a.perm[pp];
    const long long rlen = g.active ? a.row_ptr[oi + 1] - a.row_ptr[oi] : 0;
    const bool heavy = g.active && rlen > CAP;
    const bool work = g.active && !heavy;
    if (heavy) {
        const int h = atomicAdd(a.nheavy, 1);
        a.heavy[h] = g.p;
    }
    int* lst = lists + lane * (CAP + 1);
    int len = 0;
    if (work) {
        const double* pi = a.spos + static_cast<size_t>(g.p) * 4;
        const double pix[3] = {pi[0], pi[1], DIM == 3 ? pi[2] : 0.0};
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
            const int ga = g.global_of(r, g.la[r]), gb = g.global_of(r, g.lb[r]);
            for (int j = ga; j < gb; ++j) {
                if (j == g.p) continue;
                const double* pj = a.spos + static_cast<size_t>(j) * 4;
                if (r2_fp64<DIM>(pix, pj) <= fr.R2) {
                    if (len < CAP) lst[len] = a.perm[j];
                    ++len;
                }
            }
        }
        if (len != rlen) atomicOr(a.err, kErrLongRow);
        lane_sort<CAP>(lst, len < CAP ? len : CAP);
    }
    emit_rows<DIM, 1, CAP>(a, lists, len < CAP ? len : CAP, work, oi, soff, srow, soi);
}

// ---------------------------------------------------------------------------
// Long rows: one workgroup per target, candidates spread over its threads, entries
// appended to the row in any order and then sorted in LDS (bitonic network in which
// every comparator puts the smaller key first, so padding at +inf never moves).
constexpr int kHeavyThreads = 256;

template <int DIM, int MODE>
__global__ void __launch_bounds__(kHeavyThreads)
k_heavy(SearchArgs a)
{
    __shared__ unsigned long long keys[kHeavySortMax];
    __shared__ int fill;
    const Frame& fr = a.fr;
    const uint32_t ncx = static_cast<uint32_t>(fr.nc[0]);
    const int ncy = fr.nc[1], ncz = fr.nc[2];
    const int nh = *a.nheavy;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int p = a.heavy[h];
        const int oi = a.perm[p];
        const uint32_t key = a.skey[p];
        const uint32_t row = key / ncx;
        const int x = static_cast<int>(key - row * ncx);
        const int y0 = static_cast<int>(row % static_cast<uint32_t>(ncy));
        const int z0 = static_cast<int>(row / static_cast<uint32_t>(ncy));
        const long long rs = a.row_ptr[oi];
        const long long rlen = a.row_ptr[oi + 1] - rs;
        double pi[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) pi[k] = a.pos[static_cast<size_t>(oi) * DIM + k];
        const ushort4 qi = a.q4[p];
        if (threadIdx.x == 0) fill = 0;
        __syncthreads();
        constexpr int NSEG = DIM == 3 ? 9 : 3;
        const int lx0 = x > 0 ? x - 1 : 0;
        const int lx1 = x + 1 < static_cast<int>(ncx) ? x + 1 : static_cast<int>(ncx) - 1;
        for (int r = 0; r < NSEG; ++r) {
            const int dy = r % 3 - 1, dz = DIM == 3 ? r / 3 - 1 : 0;
            const int yy = y0 + dy, zz = z0 + dz;
            if (yy < 0 || yy >= ncy || zz < 0 || zz >= ncz) continue;
            const int rb = (zz * ncy + yy) * static_cast<int>(ncx);
            const int ga = a.cell_start[rb + lx0], gb = a.cell_start[rb + lx1 + 1];
            const _Float16 ay = as_f16(qi.y) + static_cast<_Float16>(-2 * dy);
            const _Float16 az = as_f16(qi.z) + static_cast<_Float16>(-2 * dz);
            for (int j = ga + static_cast<int>(threadIdx.x); j < gb; j += kHeavyThreads) {
                if (j == p) continue;
                bool nb;
                const int oj = a.perm[j];
                if (MODE == 1) {
                    const double* pj = a.spos + static_cast<size_t>(j) * 4;
                    const double* pis = a.spos + static_cast<size_t>(p) * 4;
                    nb = r2_fp64<DIM>(pis, pj) <= fr.R2;
                } else {
                    const ushort4 v = a.q4[j];
                    const uint32_t kj = a.skey[j];
                    const int cjx = static_cast<int>(kj - (kj / ncx) * ncx);
                    const _Float16 s = as_f16(qi.x) - as_f16(v.x);
                    const _Float16 tx = s + static_cast<_Float16>(2 * (x - cjx));
                    const _Float16 ty = ay - as_f16(v.y);
                    _Float16 r2;
                    if (DIM == 3) {
                        const _Float16 tz = az - as_f16(v.z);
                        r2 = tz * tz;
                        r2 = __builtin_fmaf16(ty, ty, r2);
                    } else {
                        r2 = ty * ty;
                    }
                    r2 = __builtin_fmaf16(tx, tx, r2);
                    const uint16_t r2h = __builtin_bit_cast(uint16_t, r2);
                    const bool in16 = r2h < fr.t_lo;
                    const bool band = !in16 && r2h <= fr.t_hi;
                    nb = (MODE == 2 || band) ? recheck<DIM>(a.pos, pi, oj, fr.R2) : in16;
                }
                if (nb) {
                    const int slot = atomicAdd(&fill, 1);
                    const float d = MODE == 1 ? dist_fp64<DIM>(a.pos, oi, oj)
                                              : dist_fixed<DIM>(a.X, fr.n, oi, oj, fr.dist_scale);
                    const long long idx = rs + slot;
                    if (slot < rlen && idx < a.capacity) {
                        a.col[idx] = oj;
                        a.dist[idx] = d;
                    } else {
                        atomicOr(a.err, slot < rlen ? kErrCapacity : kErrLongRow);
                    }
                }
            }
        }
        __syncthreads();
        const int L = fill;
        if (L != rlen) {
            if (threadIdx.x == 0) atomicOr(a.err, kErrLongRow);
        } else if (L > kHeavySortMax) {
            if (threadIdx.x == 0) atomicOr(a.err, kErrLongRow);
        } else if (rs + L <= a.capacity) {
            int P = 1;
            while (P < L) P <<= 1;
            for (int i = threadIdx.x; i < P; i += kHeavyThreads) {
                keys[i] = i < L ? (static_cast<unsigned long long>(static_cast<uint32_t>(a.col[rs + i])) << 32) |
                                      __builtin_bit_cast(uint32_t, a.dist[rs + i])
                                : ~0ull;
            }
            __syncthreads();
            for (int k = 2; k <= P; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int t = threadIdx.x; t < P / 2; t += kHeavyThreads) {
                        int i0, i1;
                        if (j == (k >> 1)) {
                            i0 = (t / j) * k + (t % j);
                            i1 = (t / j) * k + (k - 1 - (t % j));
                        } else {
                            i0 = (t / j) * 2 * j + (t % j);
                            i1 = i0 + j;
                        }
                        const unsigned long long u = keys[i0], v = keys[i1];
                        if (u > v) {
                            keys[i0] = v;
                            keys[i1] = u;
                        }
                    }
                    __syncthreads();
                }
            }
            for (int i = threadIdx.x; i < L; i += kHeavyThreads) {
                a.col[rs + i] = static_cast<int32_t>(keys[i] >> 32);
                a.dist[rs + i] = __builtin_bit_cast(float, static_cast<uint32_t>(keys[i]));
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
hipError_t launch_count(const SearchArgs& a, int nblk_max, hipStream_t st)
{
    if (a.fr.n == 0 || nblk_max == 0) return hipSuccess;
    const dim3 g(nblk_max), b(64);
    const int d = a.fr.dim, m = a.fr.mode;
    if (d == 2 && m == 0) hipLaunchKernelGGL((k_count16<2, 0>), g, b, 0, st, a);
    else if (d == 3 && m == 0) hipLaunchKernelGGL((k_count16<3, 0>), g, b, 0, st, a);
    else if (d == 2 && m == 2) hipLaunchKernelGGL((k_count16<2, 2>), g, b, 0, st, a);
    else if (d == 3 && m == 2) hipLaunchKernelGGL((k_count16<3, 2>), g, b, 0, st, a);
    else if (d == 2) hipLaunchKernelGGL(k_count64<2>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_count64<3>, g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_fill(const SearchArgs& a, int nblk_max, hipStream_t st)
{
    if (a.fr.n == 0 || nblk_max == 0) return hipSuccess;
    const dim3 g(nblk_max), b(64);
    const int d = a.fr.dim, m = a.fr.mode;
    if (d == 2 && m == 0) hipLaunchKernelGGL((k_fill16<2, 0>), g, b, 0, st, a);
    else if (d == 3 && m == 0) hipLaunchKernelGGL((k_fill16<3, 0>), g, b, 0, st, a);
    else if (d == 2 && m == 2) hipLaunchKernelGGL((k_fill16<2, 2>), g, b, 0, st, a);
    else if (d == 3 && m == 2) hipLaunchKernelGGL((k_fill16<3, 2>), g, b, 0, st, a);
    else if (d == 2) hipLaunchKernelGGL(k_fill64<2>, g, b, 0, st, a);
    else hipLaunchKernelGGL(k_fill64<3>, g, b, 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 gh(512), bh(kHeavyThreads);
    if (d == 2 && m == 0) hipLaunchKernelGGL((k_heavy<2, 0>), gh, bh, 0, st, a);
    else if (d == 3 && m == 0) hipLaunchKernelGGL((k_heavy<3, 0>), gh, bh, 0, st, a);
    else if (d == 2 && m == 2) hipLaunchKernelGGL((k_heavy<2, 2>), gh, bh, 0, st, a);
    else if (d == 3 && m == 2) hipLaunchKernelGGL((k_heavy<3, 2>), gh, bh, 0, st, a);
    else if (d == 2) hipLaunchKernelGGL((k_heavy<2, 1>), gh, bh, 0, st, a);
    else hipLaunchKernelGGL((k_heavy<3, 1>), gh, bh, 0, st, a);
    return hipGetLastError();
}

}  // namespace nnps
