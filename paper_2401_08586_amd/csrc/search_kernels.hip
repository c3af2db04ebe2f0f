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

// FP32 distance from the fixed-point positions: the displacement of two exact integers
// below 2^52 is exact in binary64 and is rounded once to FP32.
template <int DIM>
__device__ __forceinline__ float dist_fixed(const double* __restrict__ X, int oi, int oj, float scale)
{
    float s2 = 0.0f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const double d = X[static_cast<size_t>(oj) * x_stride(DIM) + k] - X[static_cast<size_t>(oi) * x_stride(DIM) + k];
        const float f = static_cast<float>(d);
        s2 = s2 + f * f;
    }
    return __builtin_amdgcn_sqrtf(s2) * scale;  // <= 1 ulp; s2 >= 1 or 0
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

__device__ __forceinline__ int wave_sum_i32(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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
    const SetDesc* sd;  // the block's set
    Frame fr;

    __device__ __forceinline__ void init(const SearchArgs& a, int b)
    {
        sd = a.L.sets + a.bset[b];
        fr = sd->fr;
        const uint32_t coff = static_cast<uint32_t>(sd->coff);
        const int* cs = a.cell_start + coff;
        const int lane = threadIdx.x & 63;
        p0 = a.bstart[b];
        p1 = a.bstart[b + 1];
        p = p0 + lane;
        active = p < p1;
        const uint32_t ncx = static_cast<uint32_t>(fr.nc[0]);
        const int ncy = fr.nc[1], ncz = fr.nc[2];
        const uint32_t k0 = a.skey[p0] - coff;
        const uint32_t row0 = k0 / ncx;
        const int xa = static_cast<int>(k0 - row0 * ncx);
        const int y0 = static_cast<int>(row0 % static_cast<uint32_t>(ncy));
        const int z0 = static_cast<int>(row0 / static_cast<uint32_t>(ncy));
        const uint32_t kl = a.skey[p1 - 1] - coff;
        const int xb = static_cast<int>(kl - (kl / ncx) * ncx);
        const uint32_t mk = a.skey[active ? p : p1 - 1] - coff;
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
                g0 = cs[rb + sx0];
                g1 = cs[rb + sx1 + 1];
                ga = cs[rb + lx0];
                gb = cs[rb + lx1 + 1];
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
        // static indices only, so the segment tables stay in registers
        int gi = posl - seg_base[0] + seg_g0[0];
#pragma unroll
        for (int k = 1; k < NSEG; ++k)
            if (posl >= seg_base[k]) gi = posl - seg_base[k] + seg_g0[k];
        return gi;
    }
};

// Per-block descriptor the count pass leaves for the fill, so the fill's set-up reads the
// block's geometry with one load instead of re-deriving it through the block table, the
// sorted cell keys and the cell starts: [0] first particle, [1] end, [2] set, [3] union
// size, [4] 1 for a block of the dense-cell path, then the NSEG segment first-particle
// indices and the NSEG segment union offsets.
constexpr int kDescInts = kBlockDescInts;

template <int DIM>
__device__ __forceinline__ void write_desc(const SearchArgs& a, const Geom<DIM>& g, int b)
{
    const int lane = threadIdx.x & 63;
    int v = 0;
    if (lane == 0) v = g.p0;
    if (lane == 1) v = g.p1;
    if (lane == 2) v = a.bset[b];
    if (lane == 3) v = g.U;
#pragma unroll
    for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
        if (lane == 5 + r) v = g.seg_g0[r];
        if (lane == 5 + Geom<DIM>::NSEG + r) v = g.seg_base[r];
    }
    if (lane < kDescInts) a.bdesc[static_cast<size_t>(b) * kDescInts + lane] = v;
}

// A dense-cell block: only its flag is written.
__device__ __forceinline__ void write_desc_dense(const SearchArgs& a, int b)
{
    if ((threadIdx.x & 63) == 4) a.bdesc[static_cast<size_t>(b) * kDescInts + 4] = 1;
}

// The fill's view of a block, from its descriptor (lane = target).
template <int DIM>
struct FillGeom {
    static constexpr int NSEG = Geom<DIM>::NSEG;
    static constexpr int SELF = Geom<DIM>::SELF;
    int p0, p1, p, U, pself;
    bool active;
    int seg_g0[NSEG], seg_base[NSEG];
    const SetDesc* sd;
    __device__ __forceinline__ void init(const SearchArgs& a, const int* __restrict__ d)
    {
        const int lane = threadIdx.x & 63;
        p0 = d[0];
        p1 = d[1];
        sd = a.L.sets + d[2];
        U = d[3];
#pragma unroll
        for (int r = 0; r < NSEG; ++r) {
            seg_g0[r] = d[5 + r];
            seg_base[r] = d[5 + NSEG + r];
        }
        p = p0 + lane;
        active = p < p1;
        pself = seg_base[SELF] + (p - seg_g0[SELF]);
    }
    __device__ __forceinline__ int global_of_any(int posl) const
    {
        int gi = posl - seg_base[0] + seg_g0[0];
#pragma unroll
        for (int k = 1; k < NSEG; ++k)
            if (posl >= seg_base[k]) gi = posl - seg_base[k] + seg_g0[k];
        return gi;
    }
};

// The fields of a set a kernel uses in its loops, read once into registers. Read through
// the set table instead, they would be loaded again after every store (the compiler
// cannot tell the stores from the table), each time waiting on memory. The outputs are
// global-address-space pointers, so their stores are plain global stores.
#define NNPS_GLOBAL __attribute__((address_space(1)))
struct SetView {
    const NNPS_GLOBAL double* pos;
    const NNPS_GLOBAL int64_t* row_ptr;
    NNPS_GLOBAL int32_t* col;
    NNPS_GLOBAL float* dist;
    int64_t capacity;
    int poff;
    __device__ __forceinline__ explicit SetView(const SetDesc& sd)
        : pos((const NNPS_GLOBAL double*)sd.pos),
          row_ptr((const NNPS_GLOBAL int64_t*)sd.row_ptr),
          col((NNPS_GLOBAL int32_t*)sd.col),
          dist((NNPS_GLOBAL float*)sd.dist),
          capacity(sd.capacity),
          poff(sd.poff)
    {
    }
};

template <int DIM>
__device__ __forceinline__ bool recheck_g(const NNPS_GLOBAL double* __restrict__ pos, const double* pi, int oj,
                                          double R2)
{
    double pj[3];
#pragma unroll
    for (int k = 0; k < DIM; ++k) pj[k] = pos[static_cast<size_t>(oj) * DIM + k];
    return r2_fp64<DIM>(pi, pj) <= R2;
}

// The work block a workgroup takes. Workgroups are dealt to the eight XCDs in turn (the
// i-th to XCD i mod 8), each XCD with its own L2, while neighbouring blocks share most of
// their candidate unions. So XCD k is given the k-th contiguous eighth of the blocks,
// walked in order: block = (i mod 8) * ceil(nblk / 8) + i / 8. Returns -1 for workgroups
// with no block (the grid is sized for an upper bound of the count).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int nblk)
{
    const int i = blockIdx.x;
    const int per = (nblk + kXcds - 1) / kXcds;
    const int b = (i % kXcds) * per + i / kXcds;
    return (i / kXcds < per && b < nblk) ? b : -1;
}

// Blocks of the dense-cell path's windows are left to that path.
__device__ __forceinline__ bool dense_block(const SearchArgs& a, int b)
{
    return a.wdense && a.wdense[a.skey[a.bstart[b]]];
}

// Stage logical positions [cb, ce) as pair records; with ORIG also the original indices.
template <int DIM, bool ORIG>
__device__ __forceinline__ void stage(const SearchArgs& a, const Geom<DIM>& g, int cb, int ce,
                                      uint4* srec, int* sorig)
{
    const int lane = threadIdx.x & 63;
    const int m0 = cb >> 1, m1 = (ce + 1) >> 1;
    const uint16_t base16 = static_cast<uint16_t>(g.sx0 & 0xFFFF);
    // a chunk is at most kStage / 128 records per lane: every gather is issued before
    // the first record is built
    constexpr int RPL = kStage / 128;
    ushort4 v[RPL][2];
    int o[RPL][2];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int m = m0 + lane + 64 * i;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int posl = 2 * m + h;
            v[i][h] = make_ushort4(0, 0, 0, 0);
            o[i][h] = 0;
            if (m < m1 && posl < ce) {
                const int gi = g.global_of_any(posl);
                v[i][h] = a.q4[gi];
                if (ORIG) o[i][h] = a.perm[gi];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int m = m0 + lane + 64 * i;
        if (m >= m1) continue;
        uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int posl = 2 * m + h;
            if (posl < ce) {
                const uint16_t rel = static_cast<uint16_t>(v[i][h].w - base16);
                const _Float16 cx2 = static_cast<_Float16>(2 * static_cast<int>(rel));
                const uint32_t sh = 16u * h;
                w0 |= static_cast<uint32_t>(v[i][h].x) << sh;
                w1 |= static_cast<uint32_t>(v[i][h].y) << sh;
                w2 |= static_cast<uint32_t>(v[i][h].z) << sh;
                w3 |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, cx2)) << sh;
                if (ORIG) sorig[posl - cb] = o[i][h];
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

// Classify one candidate (FP16 bits r2h at union position posl);
// returns whether j is a neighbour. MODE 0: three-way test with FP64 recheck in the
// band; MODE 2: FP64 decides every candidate.
template <int DIM, int MODE>
__device__ __forceinline__ bool classify(const SearchArgs& a, const Geom<DIM>& g, const double* pi,
                                         int posl, uint32_t r2h, Tally& t, const int* sorig,
                                         int cb, int* oj_out)
{
    const Frame& fr = g.fr;
    if (MODE == 2) t.cand++;  // MODE 0 counts candidates from the lane's ranges
    const bool in16 = r2h < fr.t_lo;
    const bool band = !in16 && r2h <= fr.t_hi;
    bool nb;
    int oj = -1;
    if (MODE == 2 || band) {
        oj = sorig ? sorig[posl - cb] : a.perm[g.global_of_any(posl)];
        const bool truth = recheck<DIM>(g.sd->pos, pi, oj - g.sd->poff, fr.R2);
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
// Branch-free classification of a pair of FP16 r2 values. Non-negative FP16 bit
// patterns order like unsigned integers, so with d = r2 - T_lo per 16-bit half
// (wrapping): the sign bit of d is set exactly when r2 < T_lo ("in"), and
// sat16(d + 0xFFFE - (T_hi - T_lo)) is 0xFFFF exactly when r2 lies outside
// [T_lo, T_hi] (not in the band). Halves to ignore get r2 bits >= 0x7C00 (+inf),
// which land in neither class.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t u) { return __builtin_bit_cast(u16x2, u); }
__device__ __forceinline__ uint32_t u16x2_bits(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

struct Thresh {
    u16x2 tlo2, bias2, w12;
    __device__ __forceinline__ void init(const Frame& fr)
    {
        tlo2 = u16x2{fr.t_lo, fr.t_lo};
        const uint16_t b = static_cast<uint16_t>(0xFFFE - (fr.t_hi - fr.t_lo));
        bias2 = u16x2{b, b};
        const uint16_t w1 = static_cast<uint16_t>(fr.t_hi - fr.t_lo + 1);
        w12 = u16x2{w1, w1};
    }
};

// Bits j (j < 8) and 16 + j of x moved to bits 2j and 2j + 1.
__device__ __forceinline__ uint32_t interleave8(uint32_t x)
{
    x &= 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return (x & 0xFFFFu) | ((x >> 15) & 0x1FFFEu);
}

// Bits [a, b) of an 8-bit field (a, b clamped to [0, 8]).
__device__ __forceinline__ uint32_t span8(int a, int b)
{
    a = min(max(a, 0), 8);
    b = min(max(b, 0), 8);
    return ((1u << b) - 1u) & ~((1u << a) - 1u);
}

constexpr uint32_t kInvLo = 0x7C00u, kInvHi = 0x7C000000u;
constexpr int kGroup = 8;  // pair records per group in the FP16 count loop

// Per-lane queue of band pairs (logical position and FP16 r2 bits), held in registers
// and rechecked after the loop so the FP64 work runs with the lanes converged. Band
// pairs are rare (about two per target in 3D); a full queue makes the caller recheck
// on the spot.
struct BandQueue {
    static constexpr int kCap = 4;
    int p0 = 0, p1 = 0, p2 = 0, p3 = 0;
    uint32_t r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    int n = 0;
    // a shift register, so no entry is ever addressed by a runtime index
    __device__ __forceinline__ bool push(int posl, uint32_t r2h)
    {
        if (n >= kCap) return false;
        p3 = p2; p2 = p1; p1 = p0; p0 = posl;
        r3 = r2; r2 = r1; r1 = r0; r0 = r2h;
        ++n;
        return true;
    }
    template <typename F>
    __device__ __forceinline__ void drain(F&& f) const
    {
        if (n > 0) f(p0, r0);
        if (n > 1) f(p1, r1);
        if (n > 2) f(p2, r2);
        if (n > 3) f(p3, r3);
    }
};

// Per-lane queue of groups holding band candidates: the group's row segment and first
// pair (r << 27 | pair) and its 16 band bits in position order; a shift register in
// registers, drained once per staged chunk.
struct BandGroups {
    static constexpr int kCap = 4;
    uint32_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    uint32_t b0 = 0, b1 = 0, b2 = 0, b3 = 0;
    int n = 0;
    __device__ __forceinline__ bool push(uint32_t where, uint32_t bits)
    {
        if (n >= kCap) return false;
        a3 = a2; a2 = a1; a1 = a0; a0 = where;
        b3 = b2; b2 = b1; b1 = b0; b0 = bits;
        ++n;
        return true;
    }
    template <typename F>
    __device__ __forceinline__ void drain(F&& f)
    {
        if (n > 0) f(a0, b0);
        if (n > 1) f(a1, b1);
        if (n > 2) f(a2, b2);
        if (n > 3) f(a3, b3);
        n = 0;
    }
};

// Visit the pair records covering logical positions [lo, hi) of one row segment:
// the first and last records may hold a position outside the range, which is masked.
template <typename F>
__device__ __forceinline__ void for_pairs(int lo, int hi, F&& body)
{
    int m = lo >> 1;
    const int mend = (hi + 1) >> 1;
    if (m < mend) {
        const uint32_t inv = ((lo & 1) ? kInvLo : 0u) | ((2 * m + 1 >= hi) ? kInvHi : 0u);
        body(m, inv);
        ++m;
    }
    const int mlast = (hi & 1) ? mend - 1 : mend;
    for (; m < mlast; ++m) body(m, 0u);
    if (m < mend) body(m, kInvHi);
}

// ---------------------------------------------------------------------------
// Per-lane record of accepted candidates, one bit per candidate in the lane's own
// candidate order (row segment by row segment). Kept in LDS during the count pass and
// written out word-major (cbits[w * n + p]) so the fill pass never repeats the test.
template <int DIM>
struct CandBits {
    static constexpr int CW = DIM == 3 ? kCandWords3 : kCandWords2;
    static constexpr int NSEG = Geom<DIM>::NSEG;
    uint32_t* w;
    int total;  // the lane's candidates (its own stencil ranges)
    int nw;     // words of the block's union
    bool keep;
    // Bits are indexed by union position; the block's tables (CW + 1 words per lane, the
    // last one padding) are cleared by the whole wavefront.
    __device__ __forceinline__ void init(const Geom<DIM>& g, uint32_t* lds)
    {
        const int lane = threadIdx.x & 63;
        w = lds + lane * (CW + 1);
        total = 0;
#pragma unroll
        for (int r = 0; r < NSEG; ++r) total += g.lb[r] - g.la[r];
        keep = g.active && g.U <= 32 * CW;
        nw = (g.U + 31) >> 5;
        static_assert((64 * (CW + 1)) % 4 == 0, "the tables clear as 16-byte words");
        uint4* z = reinterpret_cast<uint4*>(lds);
        for (int k = lane; k < 64 * (CW + 1) / 4; k += 64) z[k] = make_uint4(0, 0, 0, 0);
    }
    __device__ __forceinline__ void set(int posl)
    {
        if (keep) atomicOr(&w[posl >> 5], 1u << (posl & 31));
    }
    __device__ __forceinline__ void clear(int posl)
    {
        if (keep) atomicAnd(&w[posl >> 5], ~(1u << (posl & 31)));
    }
    // Bits of up to 4 consecutive positions starting at posl (bit k = position posl + k),
    // with no branch on the bits: two unconditional ORs, the second into the next word
    // (the padding word after the union's last one).
    __device__ __forceinline__ void put(int posl, uint32_t bits)
    {
        if (!keep) return;
        const int wd = posl >> 5, sh = posl & 31;
        atomicOr(&w[wd], bits << sh);
        atomicOr(&w[wd + 1], sh ? bits >> (32 - sh) : 0u);
    }
    // Bits of 16 consecutive positions starting at posl (bit k = position posl + k).
    __device__ __forceinline__ void put16(int posl, uint32_t bits)
    {
        if (!keep) return;
        const int wd = posl >> 5, sh = posl & 31;
        atomicOr(&w[wd], bits << sh);
        atomicOr(&w[wd + 1], sh ? bits >> (32 - sh) : 0u);
    }
    __device__ __forceinline__ void store(const SearchArgs& a, int p) const
    {
        if (!keep) return;
        for (int k = 0; k < nw; ++k) a.cbits[static_cast<size_t>(k) * a.L.ntot + p] = w[k];
    }
};

// Count pass, FP16 relative coordinates (MODE 0; MODE 2 decides every candidate in FP64).
template <int DIM, int MODE, bool HALF>
__global__ void __launch_bounds__(64)
k_count16(SearchArgs a)
{
    using CB = CandBits<DIM>;
    // pair records of the staged chunk, and kGroup more that the last group of a range may
    // read past the chunk (their bits are masked)
    __shared__ uint4 srec[kStage / 2 + kGroup];
    // half lists: the staged candidates' original indices (same padding)
    __shared__ __attribute__((aligned(16))) int corig[HALF ? kStage + 2 * kGroup : 1];
    __shared__ uint32_t lbits[64 * (CB::CW + 1)];
    const int b = xcd_block(*a.nblk);
    if (b < 0) return;
    const int lane = threadIdx.x & 63;
    if (dense_block(a, b)) {
        if (lane < 5) a.blk_stats[static_cast<size_t>(b) * 5 + lane] = 0;
        write_desc_dense(a, b);
        return;
    }
    Geom<DIM> g;
    g.init(a, b);
    write_desc(a, g, b);
    const Frame& fr = g.fr;
    const int pp = g.active ? g.p : g.p1 - 1;
    const int oi = a.perm[pp];
    const double* spos_set = g.sd->pos;
    const int poff = g.sd->poff;
    double pi[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) pi[k] = spos_set[static_cast<size_t>(oi - poff) * DIM + k];
    Target16<DIM> tg;
    tg.init(a.q4[pp], g.x, g.sx0);
    Thresh th;
    th.init(fr);
    CB cb_;
    cb_.init(g, lbits);
    BandQueue bq;
    uint32_t cnt = 0;
    Tally t;
    // band candidates of a queued group (staged in the current chunk): FP16 r2 bits into the
    // position queue, or, when that is full, the FP64 recheck on the spot
    BandGroups bg;
    int cbase = 0;  // first position of the staged chunk
    auto band_group = [&](uint32_t where, uint32_t bits) {
        const int r = static_cast<int>(where >> 27);
        const int mg = static_cast<int>(where & 0x7FFFFFFu);
        const int dy = r % 3 - 1, dz = DIM == 3 ? r / 3 - 1 : 0;
        const h2 ay = splat(tg.qiy + static_cast<_Float16>(-2 * dy));
        const h2 az = splat(tg.qiz + static_cast<_Float16>(-2 * dz));
        uint32_t bb = bits;
        while (bb) {
            const int k = __builtin_ctz(bb);
            bb &= bb - 1u;
            const int posl = 2 * mg + k;
            const uint32_t rb = r2_pair<DIM>(tg, ay, az, srec[(posl >> 1) - (cbase >> 1)]);
            const uint32_t r2h = (rb >> (16 * (posl & 1))) & 0xFFFFu;
            if (!bq.push(posl, r2h) && posl != g.pself) {
                int oj;
                if (classify<DIM, 0>(a, g, pi, posl, r2h, t, nullptr, cbase, &oj) && (!HALF || oj > oi)) {
                    ++cnt;
                    cb_.set(posl);
                }
            }
        }
    };
    for (int cb = 0; cb < g.U; cb += kStage) {
        const int ce = min(g.U, cb + kStage);
        cbase = cb;
        __syncthreads();
        stage<DIM, HALF>(a, g, cb, ce, srec, corig);
        __syncthreads();
        if (!g.active) continue;
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
            const int lo = max(g.la[r], cb), hi = min(g.lb[r], ce);
            if (lo >= hi) continue;
            const int dy = r % 3 - 1, dz = DIM == 3 ? r / 3 - 1 : 0;
            const h2 ay = splat(tg.qiy + static_cast<_Float16>(-2 * dy));
            const h2 az = splat(tg.qiz + static_cast<_Float16>(-2 * dz));
            if constexpr (MODE == 2) {
                const int selfp = (r == Geom<DIM>::SELF) ? g.pself : -1;
                for_pairs(lo, hi, [&](int m, uint32_t inv) {
                    const uint32_t rb = r2_pair<DIM>(tg, ay, az, srec[m - (cb >> 1)]);
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int posl = 2 * m + h;
                        if (((inv >> (16 * h)) & 0xFFFF) || posl == selfp) continue;
                        int oj;
                        if (classify<DIM, MODE>(a, g, pi, posl, (rb >> (16 * h)) & 0xFFFF, t, nullptr, cb,
                                                &oj) &&
                            (!HALF || oj > oi)) {
                            ++cnt;
                            cb_.set(posl);
                        }
                    }
                });
            } else {
                // kGroup pair records (2 kGroup positions) at a time: the bits of the
                // accepted and of the band candidates gather in registers (bit j: position
                // 2(mg + j), bit 16 + j: position 2(mg + j) + 1) and go to the candidate
                // bits once per group; band candidates are queued for the FP64 recheck.
                const uint4* rec = srec - (cb >> 1);
                const int m0 = lo >> 1, mend = (hi + 1) >> 1;
                for (int mg = m0; mg < mend; mg += kGroup) {
                    uint32_t acc = 0, ebits = 0, gt = 0;
#pragma unroll
                    for (int j = 0; j < kGroup; ++j) {
                        const uint32_t rb = r2_pair<DIM>(tg, ay, az, rec[mg + j]);
                        const u16x2 d = as_u16x2(rb) - th.tlo2;
                        const u16x2 e = d - th.w12;
                        acc |= (u16x2_bits(d) >> (15 - j)) & (0x10001u << j);
                        ebits |= (u16x2_bits(e) >> (15 - j)) & (0x10001u << j);
                        if (HALF) {
                            const int2 oo = *reinterpret_cast<const int2*>(&corig[2 * (mg + j) - cb]);
                            gt |= (oo.x > oi ? 1u << j : 0u) | (oo.y > oi ? 1u << (16 + j) : 0u);
                        }
                    }
                    // the group's positions inside [lo, hi)
                    const int a0 = lo - 2 * mg, b0 = hi - 2 * mg;
                    const uint32_t valid = span8((a0 + 1) >> 1, (b0 + 1) >> 1) |
                                           (span8(a0 >> 1, b0 >> 1) << 16);
                    acc &= valid;
                    const uint32_t bnd = ebits & ~acc & valid;
                    if (HALF) acc &= gt;  // half list: only candidates of larger original index
                    cnt += __builtin_popcount(acc);
                    cb_.put16(2 * mg, interleave8(acc));
                    if (bnd) {
                        const uint32_t where = (static_cast<uint32_t>(r) << 27) | static_cast<uint32_t>(mg);
                        const uint32_t bits = interleave8(bnd);
                        if (!bg.push(where, bits)) band_group(where, bits);
                    }
                }
            }
        }
        if constexpr (MODE == 0) bg.drain(band_group);
    }
    if constexpr (MODE == 0) {
        // self (r2 = 0) was counted as "in" when T_lo > 0, or queued as a band pair; half
        // lists never count it (its index is not larger than its own)
        if (!HALF && g.active && fr.t_lo > 0) cnt -= 1;
        bq.drain([&](int posl, uint32_t r2h) {
            if (posl == g.pself) return;
            const int oj = a.perm[g.global_of_any(posl)];
            const bool truth = recheck<DIM>(spos_set, pi, oj - poff, fr.R2);
            const bool naive = r2h <= fr.t_mid;
            t.band++;
            t.fpos += naive && !truth;
            t.fneg += !naive && truth;
            const bool keep = truth && (!HALF || oj > oi);
            cnt += keep;
            if (keep) cb_.set(posl);
        });
        // candidates: the lane's ranges minus itself
        if (g.active) t.cand += cb_.total - 1;
    }
    if (g.active) {
        a.counts[oi] = static_cast<int>(cnt);
        a.counts_s[g.p] = static_cast<int>(cnt);
    }
    cb_.store(a, g.p);
    unsigned long long v[5] = {t.cand, t.band, t.fpos, t.fneg, t.odis};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const unsigned long long sum = wave_sum_u64(v[k]);
        if (lane == 0) a.blk_stats[static_cast<size_t>(b) * 5 + k] = sum;
    }
}

// Count pass, plain FP64 baseline: one lane per target, global FP64 loads.
template <int DIM, bool HALF>
__global__ void __launch_bounds__(64)
k_count64(SearchArgs a)
{
    using CB = CandBits<DIM>;
    __shared__ uint32_t lbits[64 * (CB::CW + 1)];
    const int b = xcd_block(*a.nblk);
    if (b < 0) return;
    if (dense_block(a, b)) {
        if ((threadIdx.x & 63) < 5) a.blk_stats[static_cast<size_t>(b) * 5 + (threadIdx.x & 63)] = 0;
        write_desc_dense(a, b);
        return;
    }
    Geom<DIM> g;
    g.init(a, b);
    write_desc(a, g, b);
    const Frame& fr = g.fr;
    CB cb_;
    cb_.init(g, lbits);
    int cnt = 0;
    unsigned long long cand = 0;
    if (g.active) {
        const int oi = a.perm[g.p];
        const double* pi = a.spos + static_cast<size_t>(g.p) * 4;
        const double pix[3] = {pi[0], pi[1], DIM == 3 ? pi[2] : 0.0};
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
            const int ga = g.global_of(r, g.la[r]), gb = g.global_of(r, g.lb[r]);
            const int pbase = g.la[r] - ga;  // union position = pbase + j
            cand += gb - ga;
            // four candidates per step, their loads issued together (the last index is
            // repeated past the range end and its result dropped)
            for (int j = ga; j < gb; j += 4) {
                double d2[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double* pj = a.spos + static_cast<size_t>(min(j + u, gb - 1)) * 4;
                    d2[u] = r2_fp64<DIM>(pix, pj);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (j + u < gb && d2[u] <= fr.R2 && (!HALF || a.perm[j + u] > oi)) {
                        ++cnt;
                        cb_.set(pbase + j + u);
                    }
                }
            }
        }
        if (!HALF) cnt -= 1;  // itself (r2 = 0)
        cand -= 1;
        a.counts[oi] = cnt;
        a.counts_s[g.p] = cnt;
    }
    cb_.store(a, g.p);
    const unsigned long long s = wave_sum_u64(cand);
    if ((threadIdx.x & 63) < 5)
        a.blk_stats[static_cast<size_t>(b) * 5 + (threadIdx.x & 63)] = (threadIdx.x & 63) == 0 ? s : 0ull;
}

// FP32 r2 of Eq. 7 on twice the displacement in cell widths: per axis
// t = (q_i - q_j) + 2 dc, then the squares summed left to right, every operation rounded
// once to f32 (no contraction). 2 dc_x = w_i - w_j, where w is twice the cell's x offset
// from the block's first stencil cell (small integers: exact); 2 dc_y and 2 dc_z are the
// row segment's constants.
template <int DIM>
__device__ __forceinline__ float r2_fp32(const float4& qi, float wi, float cy, float cz, const float4& s)
{
#pragma clang fp contract(off)
    const float tx = (qi.x - s.x) + (wi - s.w);
    const float ty = (qi.y - s.y) + cy;
    float r2 = tx * tx + ty * ty;
    if (DIM == 3) {
        const float tz = (qi.z - s.z) + cz;
        r2 = r2 + tz * tz;
    }
    return r2;
}

constexpr int kStage32 = 256;  // candidates per staged chunk of the FP32 count (16 B each)

// Count pass, FP32 relative coordinates (the paper's FP32 variant of the relative-
// coordinate list). The block's candidate union is staged in LDS chunk by chunk as
// {q_x, q_y, q_z, 2 x-offset} (f32); each lane tests its own ranges four candidates per
// step and turns the four results into "in" and "band" bits with no branch; the rare band
// pairs are decided by the FP64 predicate on the caller's positions. The lane's own entry
// (r2 = 0) is "in" when T32_lo > 0 and is taken out at the end; otherwise it is a band
// entry and skipped there.
template <int DIM, bool HALF>
__global__ void __launch_bounds__(64)
k_count32(SearchArgs a)
{
    using CB = CandBits<DIM>;
    // the staged chunk, and 4 more entries that the last step of a range may read past it
    // (their results are dropped)
    __shared__ float4 sq[kStage32 + 4];
    // half lists: the staged candidates' original indices (same padding)
    __shared__ int sorig[HALF ? kStage32 + 4 : 1];
    __shared__ uint32_t lbits[64 * (CB::CW + 1)];
    const int b = xcd_block(*a.nblk);
    if (b < 0) return;
    const int lane = threadIdx.x & 63;
    if (dense_block(a, b)) {
        if (lane < 5) a.blk_stats[static_cast<size_t>(b) * 5 + lane] = 0;
        write_desc_dense(a, b);
        return;
    }
    Geom<DIM> g;
    g.init(a, b);
    write_desc(a, g, b);
    const Frame& fr = g.fr;
    const int pp = g.active ? g.p : g.p1 - 1;
    const int oi = a.perm[pp];
    const double* spos_set = g.sd->pos;
    const int poff = g.sd->poff;
    double pi[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) pi[k] = spos_set[static_cast<size_t>(oi - poff) * DIM + k];
    const float4 qi = a.rq[pp];
    const float wi = static_cast<float>(2 * (g.x - g.sx0));
    const float tlo = fr.t32_lo, thi = fr.t32_hi, tmid = fr.t32_mid;
    CB cb_;
    cb_.init(g, lbits);
    int cnt = 0;
    Tally t;
    const uint32_t sx0 = static_cast<uint32_t>(g.sx0);
    for (int cb = 0; cb < g.U; cb += kStage32) {
        const int ce = min(g.U, cb + kStage32);
        __syncthreads();
        for (int u = cb + lane; u < ce; u += 64) {
            const float4 v = a.rq[g.global_of_any(u)];
            // the union spans fewer than 2^10 cells in x, so the offset mod 2^10 is exact
            const uint32_t rel = (__builtin_bit_cast(uint32_t, v.w) - sx0) & 1023u;
            sq[u - cb] = make_float4(v.x, v.y, v.z, static_cast<float>(2 * static_cast<int>(rel)));
            if (HALF) sorig[u - cb] = a.perm[g.global_of_any(u)];
        }
        __syncthreads();
        if (!g.active) continue;
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) {
            const int lo = max(g.la[r], cb), hi = min(g.lb[r], ce);
            if (lo >= hi) continue;
            const float cy = static_cast<float>(2 - 2 * (r % 3));                 // -2 dy
            const float cz = DIM == 3 ? static_cast<float>(2 - 2 * (r / 3)) : 0.0f;  // -2 dz
            for (int j = lo; j < hi; j += 4) {
                uint32_t in4 = 0, band4 = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float v = r2_fp32<DIM>(qi, wi, cy, cz, sq[j - cb + u]);
                    in4 |= static_cast<uint32_t>(v < tlo) << u;
                    band4 |= static_cast<uint32_t>(v <= thi) << u;
                }
                const int left = hi - j;
                const uint32_t valid = left >= 4 ? 0xFu : (1u << left) - 1u;
                in4 &= valid;
                band4 &= valid & ~in4;
                if (band4) {
                    uint32_t bb = band4;
                    while (bb) {
                        const int k = __builtin_ctz(bb);
                        bb &= bb - 1u;
                        const int posl = j + k;
                        if (posl == g.pself) continue;
                        const float v = r2_fp32<DIM>(qi, wi, cy, cz, sq[j - cb + k]);
                        const bool truth = recheck<DIM>(spos_set, pi, a.perm[g.global_of(r, posl)] - poff, fr.R2);
                        const bool naive = v <= tmid;
                        t.band++;
                        t.fpos += naive && !truth;
                        t.fneg += !naive && truth;
                        in4 |= static_cast<uint32_t>(truth) << k;
                    }
                }
                if (HALF) {
                    uint32_t gt = 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) gt |= static_cast<uint32_t>(sorig[j - cb + u] > oi) << u;
                    in4 &= gt;
                }
                cnt += __builtin_popcount(in4);
                cb_.put(j, in4);
            }
        }
    }
    if (g.active) {
        if (!HALF && tlo > 0.0f) {  // itself, taken as "in" (half lists never keep it)
            cnt -= 1;
            cb_.clear(g.pself);
        }
#pragma unroll
        for (int r = 0; r < Geom<DIM>::NSEG; ++r) t.cand += g.lb[r] - g.la[r];
        t.cand -= 1;  // itself
        a.counts[oi] = cnt;
        a.counts_s[g.p] = cnt;
    }
    cb_.store(a, g.p);
    const unsigned long long v[5] = {t.cand, t.band, t.fpos, t.fneg, 0ull};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const unsigned long long sum = wave_sum_u64(v[k]);
        if (lane == 0) a.blk_stats[static_cast<size_t>(b) * 5 + k] = sum;
    }
}

// Sum of the per-block statistics and of the dense path's per-workgroup statistics
// (one workgroup; no contended atomics).
__global__ void __launch_bounds__(1024)
k_reduce_stats(const unsigned long long* __restrict__ blk, const int* __restrict__ nblk,
               const unsigned long long* __restrict__ dst, int ndst, unsigned long long* __restrict__ out)
{
    __shared__ unsigned long long sh[16][kDenseStats];
    const int nb = *nblk;
    unsigned long long acc[kDenseStats] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] += blk[static_cast<size_t>(b) * 5 + k];
    for (int w = threadIdx.x; w < ndst; w += blockDim.x)
#pragma unroll
        for (int k = 0; k < kDenseStats; ++k) acc[k] += dst[static_cast<size_t>(w) * kDenseStats + k];
#pragma unroll
    for (int k = 0; k < kDenseStats; ++k) {
        const unsigned long long s = wave_sum_u64(acc[k]);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kDenseStats) {
        unsigned long long s = 0;
        for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += sh[w][threadIdx.x];
        // slots 0..4 as in StatSlot; the sixth (rows of the dense path) goes to kStDenseRows
        out[threadIdx.x < 5 ? threadIdx.x : kStDenseRows] = s;
    }
}

// ---------------------------------------------------------------------------
// Fill pass. The block's whole candidate union is staged and sorted once by original
// index (a bitonic network over the wavefront's registers); each lane then records its
// accepted neighbours as a bitmask over those ranks, so reading the bits in order gives
// the row in ascending original index with no per-row sort. The rows are compacted into
// one flat list per block and written 64 entries at a time: consecutive lanes store
// consecutive CSR slots.
template <int DIM>
struct FillCfg {
    static constexpr int UCAP = DIM == 3 ? kUnion3 : kUnion2;
    static constexpr int MW = UCAP / 32;    // mask words per lane
    static constexpr int FCAP = DIM == 3 ? kFlat3 : kFlat2;
    static constexpr int SHIFT = DIM == 3 ? 10 : 9;  // log2(UCAP): key = orig << SHIFT | pos
};

// Bitonic sort of 64*EPL keys held blocked across the wavefront (element e = lane*EPL + i).
template <int EPL>
__device__ __forceinline__ void wave_bitonic(uint32_t (&v)[EPL])
{
    const int lane = threadIdx.x & 63;
    constexpr int P = 64 * EPL;
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= EPL) {
                const int lx = j / EPL;
                const bool lower = (lane & lx) == 0;
                const bool asc = ((lane * EPL) & k) == 0;
#pragma unroll
                for (int i = 0; i < EPL; ++i) {
                    const uint32_t w = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v[i]), lx, 64));
                    const uint32_t mn = min(v[i], w), mx = max(v[i], w);
                    v[i] = (lower == asc) ? mn : mx;
                }
            } else {
#pragma unroll
                for (int i = 0; i < EPL; ++i) {
                    if (i & j) continue;
                    const bool asc = ((lane * EPL + i) & k) == 0;
                    const uint32_t x = v[i], y = v[i | j];
                    const uint32_t mn = min(x, y), mx = max(x, y);
                    v[i] = asc ? mn : mx;
                    v[i | j] = asc ? mx : mn;
                }
            }
        }
    }
}

// One wavefront sorts n <= 64 EPL column indices of a row in place (registers, element
// e = lane EPL + i; padding sorts last and is not written back).
template <int EPL>
__device__ __forceinline__ void wave_sort_row(NNPS_GLOBAL int32_t* col, int n)
{
    const int lane = threadIdx.x & 63;
    uint32_t v[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        const int e = lane * EPL + i;
        v[i] = e < n ? static_cast<uint32_t>(col[e]) : 0xFFFFFFFFu;
    }
    wave_bitonic<EPL>(v);
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        const int e = lane * EPL + i;
        if (e < n) col[e] = static_cast<int32_t>(v[i]);
    }
}

// Number of keys below `key` in a sorted run of P keys (P a power of two, the run padded
// with all-ones keys): fixed-step binary lifting, every read inside the run.
template <int P>
__device__ __forceinline__ int count_below(const uint32_t* run, uint32_t key)
{
    int c = 0;
#pragma unroll
    for (int s = P >> 1; s > 0; s >>= 1) c += run[c + s - 1] < key ? s : 0;
    return c + (run[c] < key ? 1 : 0);
}

// Ranks of the U union keys (key_of(e), e < U) across NW wavefronts: wavefront wv sorts
// keys [wv Q, wv Q + Q) in registers and stores them padded to 64 EPL entries; a key's
// rank is the number of keys below it in the NW sorted quarters. Writes rank_of[e] and
// moves the original indices into rank order (sorig[rank]). Keys that carry their
// position (packed) are ranked straight from the registers; otherwise every element
// looks its own key up in all quarters.
template <int UCAP, int SHIFT, int NW, int EPL, typename K>
__device__ __forceinline__ void rank_union(int U, int Q, bool packed, int omin, K&& key_of, uint32_t* skeys,
                                           uint16_t* rank_of, int* sorig)
{
    constexpr int QP = 64 * EPL;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int e0 = wv * Q, n = max(0, min(Q, U - e0));
    uint32_t v[EPL];
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
        const int k = lane * EPL + i;
        v[i] = k < n ? key_of(e0 + k) : 0xFFFFFFFFu;
    }
    wave_bitonic<EPL>(v);
#pragma unroll
    for (int i = 0; i < EPL; ++i) skeys[wv * QP + lane * EPL + i] = v[i];
    __syncthreads();
    if (packed) {
        int rk[EPL];
#pragma unroll
        for (int i = 0; i < EPL; ++i) rk[i] = lane * EPL + i;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (q == wv) continue;
#pragma unroll
            for (int i = 0; i < EPL; ++i) rk[i] += count_below<QP>(skeys + q * QP, v[i]);
        }
#pragma unroll
        for (int i = 0; i < EPL; ++i) {
            if (v[i] == 0xFFFFFFFFu) continue;
            rank_of[v[i] & (UCAP - 1)] = static_cast<uint16_t>(rk[i]);
            sorig[rk[i]] = static_cast<int>(v[i] >> SHIFT) + omin;
        }
    } else {
        constexpr int EPT = UCAP / (64 * NW);
        int rk[EPT], og[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + i * 64 * NW;
            rk[i] = -1;
            og[i] = 0;
            if (e < U) {
                const uint32_t key = static_cast<uint32_t>(sorig[e]);
                int r = 0;
#pragma unroll
                for (int q = 0; q < NW; ++q) r += count_below<QP>(skeys + q * QP, key);
                rk[i] = r;
                og[i] = static_cast<int>(key);
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            if (rk[i] < 0) continue;
            rank_of[tid + i * 64 * NW] = static_cast<uint16_t>(rk[i]);
            sorig[rk[i]] = og[i];
        }
    }
}

// Ranks by bitmap, for unions whose original indices span at most 32 BW values (the
// common case when particles are numbered in space): one bit per index in [omin, omin +
// range), an exclusive scan of the word popcounts, and a key's rank is the number of set
// bits below it. Same outputs as rank_union: rank_of[e], and the original indices moved
// into rank order (sorig[rank]). bw (BW words) and pc (BW 16-bit prefixes) are scratch.
template <int UCAP, int NW, int BW>
__device__ __forceinline__ void rank_bitmap(int U, int omin, int range, uint32_t* bw, uint16_t* pc, int* wsum,
                                            uint16_t* rank_of, int* sorig)
{
    constexpr int NT = 64 * NW;
    constexpr int EPT = UCAP / NT;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int W = (range + 31) >> 5;
    for (int w = tid; w < W; w += NT) bw[w] = 0u;
    __syncthreads();
    int og[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        og[i] = e < U ? sorig[e] : omin;
        if (e < U) {
            const int o = og[i] - omin;
            atomicOr(&bw[o >> 5], 1u << (o & 31));
        }
    }
    __syncthreads();
    // thread t takes words [t per, t per + per): their popcounts, scanned across the block
    const int per = (W + NT - 1) / NT;
    const int w0 = min(W, tid * per), w1 = min(W, w0 + per);
    int cnt = 0;
    for (int w = w0; w < w1; ++w) cnt += __builtin_popcount(bw[w]);
    int wtot;
    const int ex = wave_excl_scan_i32(cnt, &wtot);
    if (lane == 0) wsum[wv] = wtot;
    __syncthreads();
    int run = ex;
    for (int q = 0; q < wv; ++q) run += wsum[q];
    for (int w = w0; w < w1; ++w) {
        pc[w] = static_cast<uint16_t>(run);
        run += __builtin_popcount(bw[w]);
    }
    __syncthreads();
    int rk[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        const int o = og[i] - omin;
        const int w = o >> 5;
        rk[i] = pc[w] + __builtin_popcount(bw[w] & ((1u << (o & 31)) - 1u));
        if (e < U) rank_of[e] = static_cast<uint16_t>(rk[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        if (e < U) sorig[rk[i]] = og[i];
    }
}

// Ranks by a two-level bitmap, for unions whose original indices span fewer than 2^17
// values but too many for one bit per index (3D lattices numbered row by row: a union
// covers a few planes of indices, sparsely). Level 1 marks which 32-index chunks of
// [omin, omin + 2^17) hold a union index (4096 bits); the occupied chunks are numbered in
// order by a scan of the level-1 word popcounts; level 2 keeps one 32-bit word of index
// bits per occupied chunk; a key's rank is the set level-2 bits before it (a block scan of
// the level-2 word popcounts, plus the bits below it in its own word). Same outputs as
// rank_union: rank_of[e], and the original indices moved into rank order (sorig[rank]).
// l1 (128 words), l1pre (128), l2 (UCAP words) and l2pre (UCAP) are scratch.
template <int UCAP, int NW>
__device__ __forceinline__ void rank_bitmap2(int U, int omin, uint32_t* l1, uint16_t* l1pre, uint32_t* l2,
                                             uint16_t* l2pre, int* wsum, uint16_t* rank_of, int* sorig)
{
    constexpr int NT = 64 * NW;
    constexpr int EPT = UCAP / NT;
    static_assert(NT >= 128 && UCAP % NT == 0, "the level-1 words fit one pass of the block");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < 128) l1[tid] = 0u;
#pragma unroll
    for (int i = 0; i < EPT; ++i) l2[tid * EPT + i] = 0u;
    __syncthreads();
    int og[EPT], ch[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        og[i] = e < U ? sorig[e] - omin : 0;
        ch[i] = og[i] >> 5;
        if (e < U) atomicOr(&l1[ch[i] >> 5], 1u << (ch[i] & 31));
    }
    __syncthreads();
    // number the occupied chunks: exclusive scan of the 128 level-1 popcounts (waves 0, 1)
    {
        const int c = tid < 128 ? __builtin_popcount(l1[tid]) : 0;
        int tot;
        const int ex = wave_excl_scan_i32(c, &tot);
        if (lane == 0 && wv < 2) wsum[wv] = tot;
        __syncthreads();
        if (tid < 128) l1pre[tid] = static_cast<uint16_t>(ex + (wv == 1 ? wsum[0] : 0));
    }
    __syncthreads();
    int slot[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        const int w1 = ch[i] >> 5;
        slot[i] = l1pre[w1] + __builtin_popcount(l1[w1] & ((1u << (ch[i] & 31)) - 1u));
        if (e < U) atomicOr(&l2[slot[i]], 1u << (og[i] & 31));
    }
    __syncthreads();
    // exclusive scan of the level-2 popcounts: thread t takes slots [t EPT, t EPT + EPT)
    {
        int c[EPT], sum = 0;
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            c[i] = __builtin_popcount(l2[tid * EPT + i]);
            sum += c[i];
        }
        int tot;
        int run = wave_excl_scan_i32(sum, &tot);
        if (lane == 0) wsum[wv] = tot;
        __syncthreads();
        for (int q = 0; q < wv; ++q) run += wsum[q];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            l2pre[tid * EPT + i] = static_cast<uint16_t>(run);
            run += c[i];
        }
    }
    __syncthreads();
    int rk[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        rk[i] = l2pre[slot[i]] + __builtin_popcount(l2[slot[i]] & ((1u << (og[i] & 31)) - 1u));
        if (e < U) rank_of[e] = static_cast<uint16_t>(rk[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NT;
        if (e < U) sorig[rk[i]] = og[i] + omin;
    }
}

__device__ __forceinline__ int wave_min_i32(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ long long wave_max_i64(long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, static_cast<long long>(__shfl_xor(v, o, 64)));
    return v;
}

__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int kFillThreads = 256;  // four wavefronts share one block's tables

template <int DIM, int MODE>
__global__ void __launch_bounds__(kFillThreads) __attribute__((amdgpu_waves_per_eu(5)))
k_fill(SearchArgs a)
{
    using C = FillCfg<DIM>;
    using CB = CandBits<DIM>;
    constexpr int NW = kFillThreads / 64;
    // LDS: the rank table is dead once the rows are compacted, so the flat entry list
    // reuses its space.
    constexpr int kRankBytes = C::UCAP * 2;
    constexpr int kFlatBytes = C::FCAP * 2;
    constexpr int kShared = kRankBytes > kFlatBytes ? kRankBytes : kFlatBytes;
    __shared__ __attribute__((aligned(16))) unsigned char smem[kShared];
    __shared__ int sorig[C::UCAP];
    __shared__ uint32_t masks[64 * (C::MW + 1)];
    __shared__ long long sbase[64];  // row start in the output minus the row's flat offset
    __shared__ double sxi[64 * DIM];  // targets' positions: fixed point, or FP64 (baseline)
    __shared__ int spart[NW][64];   // per-wave popcounts of each row's mask quarter
    __shared__ int sred[2][NW];
    __shared__ int swsum[NW];
    uint16_t* rank_of = reinterpret_cast<uint16_t*>(smem);
    // flat list entry: target lane << SHIFT | the candidate's rank in the union
    uint16_t* flat = reinterpret_cast<uint16_t*>(smem);
    static_assert(64 << C::SHIFT <= 65536 && (1 << C::SHIFT) == C::UCAP, "flat entries fit 16 bits");

    const int b = xcd_block(*a.nblk);
    if (b < 0) return;
    // the block's geometry from the count pass's descriptor (wave-uniform), and each
    // target's row start and length in sorted order: no chain of dependent loads
    const int* __restrict__ dsc = a.bdesc + static_cast<size_t>(b) * kDescInts;
    if (dsc[4]) return;  // a block of the dense-cell path
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront index, uniform
    FillGeom<DIM> g;
    g.init(a, dsc);
    const SetView sd(*g.sd);
    const float dist_scale = g.sd->fr.dist_scale;  // in a register: stores below cannot change it
    const int pp = g.active ? g.p : g.p1 - 1;
    const long long rs = a.rsort[pp];
    const int rlen = g.active ? a.counts_s[g.p] : 0;
    int E;
    const int off = wave_excl_scan_i32(rlen, &E);
    E = __builtin_amdgcn_readfirstlane(E);  // the block's entry count, wave-uniform
    static_assert(32 * CB::CW == C::UCAP, "the count pass keeps a bit per union position");
    if (g.U > C::UCAP || E > C::FCAP) {
        // too big for this path: every row of the block goes to the long-row path
        if (wv == 0 && g.active) a.heavy[atomicAdd(a.nheavy, 1)] = g.p;
        return;
    }
    // the count pass's accepted-candidate bits (by union position), this wavefront's words
    // w = wv + NW k, are loaded first: their latency is hidden behind staging and ranking
    constexpr int KW = (CB::CW + NW - 1) / NW;
    uint32_t wbits[KW];
    {
        const int nwt = g.active ? (g.U + 31) >> 5 : 0;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int w = wv + NW * k;
            wbits[k] = w < nwt ? a.cbits[static_cast<size_t>(w) * a.L.ntot + g.p] : 0u;
        }
    }
    // 1. stage the union's original indices; clear the masks
    const int U = g.U;
    int omin = 0x7FFFFFFF, omax = 0;
    {
        // a thread's gathers are issued together, then stored
        constexpr int EPT = C::UCAP / kFillThreads;
        int og[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + i * kFillThreads;
            og[i] = e < U ? a.perm[g.global_of_any(e)] : -1;
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = tid + i * kFillThreads;
            if (e < U) {
                sorig[e] = og[i];
                omin = min(omin, og[i]);
                omax = max(omax, og[i]);
            }
        }
    }
    for (int i = tid; i < 64 * (C::MW + 1); i += kFillThreads) masks[i] = 0;
    omin = wave_min_i32(omin);
    omax = wave_max_i32(omax);
    if (lane == 0) {
        sred[0][wv] = omin;
        sred[1][wv] = omax;
    }
    if (wv == 0) {
        sbase[lane] = rs - off;
        const int oi = a.perm[pp];
        const int li = oi - sd.poff;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
            // the target's own coordinates for the distance: fixed point, or FP64 bits (baseline)
            sxi[lane * DIM + k] = MODE == 1 ? sd.pos[static_cast<size_t>(li) * DIM + k]
                                            : a.X[static_cast<size_t>(oi) * x_stride(DIM) + k];
        }
    }
    __syncthreads();
    // 2. rank the union by original index. Keys are (orig - omin) << SHIFT | position when
    // the union's index range allows, else the original index itself: distinct either way,
    // and below the all-ones key that pads the sorted quarters.
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        omin = min(omin, sred[0][w]);
        omax = max(omax, sred[1][w]);
    }
    const bool packed = static_cast<uint32_t>(omax - omin) < (1u << (32 - C::SHIFT)) - 1u;
    static_assert(C::UCAP * 2 + C::UCAP * 4 <= kShared, "sorted quarters fit beside the rank table");
    uint32_t* skeys = reinterpret_cast<uint32_t*>(smem + C::UCAP * 2);
    const int Q = (U + NW - 1) / NW;
    auto key_of = [&](int e) -> uint32_t {
        const int o = sorig[e];
        return packed ? (static_cast<uint32_t>(o - omin) << C::SHIFT) | static_cast<uint32_t>(e)
                      : static_cast<uint32_t>(o);
    };
    // unions spanning few original indices are ranked by bitmap (scratch after the rank table)
    constexpr int BW = (kShared - C::UCAP * 2) / 6;
    // the two-level bitmap's tables after the rank table: level 1 (512 B) and its prefixes
    // (256 B), level 2 (4 UCAP B) and its prefixes (2 UCAP B)
    constexpr bool kTwoLevel = C::UCAP * 2 + 768 + C::UCAP * 6 <= kShared;
    if (static_cast<unsigned>(omax - omin) < 32u * BW)
        rank_bitmap<C::UCAP, NW, BW>(U, omin, omax - omin + 1, reinterpret_cast<uint32_t*>(smem + C::UCAP * 2),
                                     reinterpret_cast<uint16_t*>(smem + C::UCAP * 2 + BW * 4), swsum, rank_of, sorig);
    else if (kTwoLevel && static_cast<unsigned>(omax - omin) < (1u << 17))
        rank_bitmap2<C::UCAP, NW>(U, omin, reinterpret_cast<uint32_t*>(smem + C::UCAP * 2),
                                  reinterpret_cast<uint16_t*>(smem + C::UCAP * 2 + 512),
                                  reinterpret_cast<uint32_t*>(smem + C::UCAP * 2 + 768),
                                  reinterpret_cast<uint16_t*>(smem + C::UCAP * 6 + 768), swsum, rank_of, sorig);
    else if (Q <= 64) rank_union<C::UCAP, C::SHIFT, NW, 1>(U, Q, packed, omin, key_of, skeys, rank_of, sorig);
    else if (Q <= 128) rank_union<C::UCAP, C::SHIFT, NW, 2>(U, Q, packed, omin, key_of, skeys, rank_of, sorig);
    else rank_union<C::UCAP, C::SHIFT, NW, 4>(U, Q, packed, omin, key_of, skeys, rank_of, sorig);
    __syncthreads();
    // 3. accepted candidates from the count pass, re-indexed by rank into each target's
    // mask. Wavefront wv holds the bit words w = wv (mod 4) of every target; it lists its
    // nonzero ones (one ballot per word) in LDS and then takes one listed word per lane,
    // so a round of bit extraction waits for the fullest of 64 nonzero words, not for the
    // fullest lane of every word. The list lives in the ranking scratch, dead by now.
    uint32_t* mk = masks + lane * (C::MW + 1);
    {
        constexpr int kListBytes = kShared - C::UCAP * 2;
        constexpr int LCAP = (kListBytes / NW / 6) & ~63;  // entries per wavefront
        static_assert(LCAP >= 64, "a wavefront lists at least one word per lane");
        uint32_t* lbits = reinterpret_cast<uint32_t*>(smem + C::UCAP * 2) + wv * LCAP;
        uint16_t* ltw = reinterpret_cast<uint16_t*>(smem + C::UCAP * 2 + NW * LCAP * 4) + wv * LCAP;
        auto drain = [&](int n) {
            for (int e = lane; e < n; e += 64) {
                uint32_t bits = lbits[e];
                const int tw = ltw[e];
                uint32_t* mt = masks + (tw & 63) * (C::MW + 1);
                const int w32 = (tw >> 6) * 32;
                // four bits per round: their rank lookups are issued together, and bits past
                // the word's last read entry 0 and OR nothing
                while (bits) {
                    uint32_t rk[4], on[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        on[j] = bits != 0u ? 1u : 0u;
                        const int posl = w32 + __builtin_ctz(bits | (on[j] ? 0u : 1u));
                        bits &= bits - 1u;
                        rk[j] = rank_of[on[j] ? posl : 0];
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j) atomicOr(&mt[rk[j] >> 5], on[j] << (rk[j] & 31));
                }
            }
        };
        int qn = 0;
#pragma unroll
        for (int k = 0; k < KW; ++k) {
            const int w = wv + NW * k;
            const uint32_t word = g.active ? wbits[k] : 0u;
            const uint64_t nz = __builtin_amdgcn_ballot_w64(word != 0u);
            const int add = __builtin_popcountll(nz);
            if (qn + add > LCAP) {  // wave-uniform
                drain(qn);
                qn = 0;
            }
            if (word) {
                const int at = qn + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                        static_cast<uint32_t>(nz >> 32),
                                        __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(nz), 0u)));
                lbits[at] = word;
                ltw[at] = static_cast<uint16_t>(lane | (w << 6));
            }
            qn += add;
        }
        drain(qn);
    }
    // the target's own bit (set by the count pass when it accepted the target itself) is
    // masked out below
    const int rself = g.active ? rank_of[g.pself] : -1;
    __syncthreads();
    // 4. compaction: each target's mask walked in rank order into the block's flat list;
    // wavefront wv takes word quarter wv, after the popcounts of the quarters before it
    const int nw = (U + 31) >> 5;
    const int qw = (nw + NW - 1) / NW;
    const int wa = wv * qw, wb = min(nw, wa + qw);
    const int wself = rself >> 5;
    const uint32_t keep_self = ~(1u << (rself & 31));
    auto word = [&](int w) { return mk[w] & (w == wself ? keep_self : ~0u); };
    int cnt = 0;
    if (g.active)
        for (int w = wa; w < wb; ++w) cnt += __builtin_popcount(word(w));
    spart[wv][lane] = cnt;
    __syncthreads();  // rank table dead from here on: the flat list reuses its space
    if (g.active) {
        int got = 0;
        for (int q = 0; q < wv; ++q) got += spart[q][lane];
        for (int w = wa; w < wb; ++w) {
            uint32_t bits = word(w);
            while (bits) {
                const int bi = __builtin_ctz(bits);
                bits &= bits - 1;
                if (got < rlen) flat[off + got] = static_cast<uint16_t>((lane << C::SHIFT) | (w * 32 + bi));
                ++got;
            }
        }
        if (wv == NW - 1 && got != rlen) atomicOr(a.err, kErrLongRow);
    }
    __syncthreads();
    // 5. emission, 64 entries per round, rounds dealt to the wavefronts in turn. Later
    // rounds' gathers are issued before this round's stores, and every round issues the
    // same memory instructions on every path. Vector-memory counters count loads and
    // stores in issue order, so with a fixed instruction count the wait for the prefetch
    // need not include the previous round's stores.
    struct Ent {
        int t, oj;
        long long idx;
        double xj[DIM];
    };
    auto gather = [&](Ent& s) {
#pragma unroll
        for (int c = 0; c < DIM; ++c)
            s.xj[c] = MODE == 1 ? sd.pos[static_cast<size_t>(s.oj - sd.poff) * DIM + c]
                                : a.X[static_cast<size_t>(s.oj) * x_stride(DIM) + c];
    };
    auto distance = [&](const Ent& s) -> float {
        if constexpr (MODE == 1) {
            double pi2[3], pj2[3];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                pi2[c] = sxi[s.t * DIM + c];
                pj2[c] = s.xj[c];
            }
            return static_cast<float>(__dsqrt_rn(r2_fp64<DIM>(pi2, pj2)));
        } else {
            float s2 = 0.0f;
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const float f = static_cast<float>(s.xj[c] - sxi[s.t * DIM + c]);  // exact difference, one rounding
                s2 = s2 + f * f;
            }
            return __builtin_amdgcn_sqrtf(s2) * dist_scale;  // <= 1 ulp; s2 >= 1 or 0
        }
    };
    constexpr int R = 64 * NW;  // stride between a wavefront's rounds
    const int64_t cap = sd.capacity;
    const long long rend = g.active ? rs + rlen : 0;  // the row's end in the output
    if (wave_max_i64(rend) <= cap) {
        // every row fits the output: lanes past the list repeat the list's last entry (the
        // same values to the same place), so no address is ever switched
        auto fetch = [&](int e, Ent& s) {
            const uint32_t f = flat[min(e, E - 1)];
            s.t = static_cast<int>(f >> C::SHIFT);
            s.oj = sorig[f & (C::UCAP - 1)];
            s.idx = sbase[s.t] + min(e, E - 1);
            gather(s);
        };
        auto emit = [&](const Ent& s) {
            const float d = distance(s);
            sd.col[s.idx] = s.oj - sd.poff;
            sd.dist[s.idx] = d;
        };
        // four entry sets in rotation: the fetch three rounds ahead never waits for a copy
        Ent A, B, Cn, D;
        int e0 = wv * 64;
        if (e0 < E) {
            fetch(e0 + lane, A);
            fetch(e0 + R + lane, B);
            fetch(e0 + 2 * R + lane, Cn);
            for (;;) {
                fetch(e0 + 3 * R + lane, D);
                emit(A);
                if ((e0 += R) >= E) break;
                fetch(e0 + 3 * R + lane, A);
                emit(B);
                if ((e0 += R) >= E) break;
                fetch(e0 + 3 * R + lane, B);
                emit(Cn);
                if ((e0 += R) >= E) break;
                fetch(e0 + 3 * R + lane, Cn);
                emit(D);
                if ((e0 += R) >= E) break;
            }
        }
        return;
    }
    // some row ends past the output capacity: entries there (and lanes past the list)
    // store to a per-lane sink slot, and the capacity error is raised
    NNPS_GLOBAL int32_t* sink_col = (NNPS_GLOBAL int32_t*)a.sink + 2 * lane;
    NNPS_GLOBAL float* sink_dist = (NNPS_GLOBAL float*)(a.sink + 2 * lane + 1);
    auto fetch = [&](int e, Ent& s) {
        // every read stays inside its table whatever e is, so no branch is needed: entries
        // past the list read stale values that the selects below discard
        const bool ok = e < E;
        const uint32_t f = flat[min(e, C::FCAP - 1)];
        const int t = static_cast<int>(f >> C::SHIFT) & 63;
        const int o = sorig[f & (C::UCAP - 1)];
        const long long base = sbase[t];
        s.t = t;
        s.oj = ok ? o : sd.poff;
        s.idx = ok ? base + e : -1;
        gather(s);
    };
    Ent cur, n1;
    fetch(wv * 64 + lane, cur);
    fetch(wv * 64 + R + lane, n1);
    for (int e0 = wv * 64; e0 < E; e0 += R) {
        Ent n2;
        fetch(e0 + 2 * R + lane, n2);
        const float d = distance(cur);
        const bool valid = cur.idx >= 0 && cur.idx < cap;
        if (cur.idx >= cap) atomicOr(a.err, kErrCapacity);
        NNPS_GLOBAL int32_t* pc = valid ? sd.col + cur.idx : sink_col;
        NNPS_GLOBAL float* pd = valid ? sd.dist + cur.idx : sink_dist;
        *pc = cur.oj - sd.poff;
        *pd = d;
        cur = n1;
        n1 = n2;
    }
}

// ---------------------------------------------------------------------------
// Long rows (blocks whose union, entry count or candidate count exceed the fill's
// limits): one workgroup per target. Its candidates are tested across the workgroup and
// the accepted original indices appended to the row in any order; the row is then sorted
// in place (LDS bitonic network for up to lr_keys entries, in which every comparator puts
// the smaller key first so padding at +inf never moves; longer rows are sorted in chunks
// and merged pairwise by rank, using the row's distance slots as scratch), and finally
// the distances are computed from the sorted column indices.
constexpr int kLongThreads = 256;

template <int DIM, int MODE>
__global__ void __launch_bounds__(kLongThreads)
k_long(SearchArgs a)
{
    extern __shared__ uint32_t keys[];  // a.lr_keys entries
    __shared__ int fill;
    const int nh = *a.nheavy;
    const int T = kLongThreads;
    for (int h = blockIdx.x; h < nh; h += gridDim.x) {
        const int p = a.heavy[h];
        const uint32_t gkey = a.skey[p];
        const SetDesc& sdesc = a.L.sets[find_set(a.L.coffs, a.L.nsets, static_cast<int>(gkey))];
        const Frame fr = sdesc.fr;
        const int* cs = a.cell_start + sdesc.coff;
        const uint32_t scoff = static_cast<uint32_t>(sdesc.coff);
        const SetView sd(sdesc);
        const uint32_t ncx = static_cast<uint32_t>(fr.nc[0]);
        const int ncy = fr.nc[1], ncz = fr.nc[2];
        const uint32_t key = gkey - scoff;
        const uint32_t row = key / ncx;
        const int x = static_cast<int>(key - row * ncx);
        const int y0 = static_cast<int>(row % static_cast<uint32_t>(ncy));
        const int z0 = static_cast<int>(row / static_cast<uint32_t>(ncy));
        const int oi = a.perm[p];
        const int li = oi - sd.poff;
        const long long rs = sd.row_ptr[li];
        const int rlen = static_cast<int>(sd.row_ptr[li + 1] - rs);
        double pi[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < DIM; ++k) pi[k] = sd.pos[static_cast<size_t>(li) * DIM + k];
        const ushort4 qi = a.q4[p];
        if (threadIdx.x == 0) fill = 0;
        __syncthreads();
        const bool room = rs + rlen <= sd.capacity;
        NNPS_GLOBAL int32_t* col = sd.col + rs;
        // 1. test every candidate; append accepted set-local indices in any order
        constexpr int NSEG = DIM == 3 ? 9 : 3;
        const int lx0 = x > 0 ? x - 1 : 0;
        const int lx1 = x + 1 < static_cast<int>(ncx) ? x + 1 : static_cast<int>(ncx) - 1;
        for (int r = 0; r < NSEG; ++r) {
            const int dy = r % 3 - 1, dz = DIM == 3 ? r / 3 - 1 : 0;
            const int yy = y0 + dy, zz = z0 + dz;
            if (yy < 0 || yy >= ncy || zz < 0 || zz >= ncz) continue;
            const int rb = (zz * ncy + yy) * static_cast<int>(ncx);
            const int ga = cs[rb + lx0], gb = cs[rb + lx1 + 1];
            const _Float16 ay = as_f16(qi.y) + static_cast<_Float16>(-2 * dy);
            const _Float16 az = as_f16(qi.z) + static_cast<_Float16>(-2 * dz);
            for (int j = ga + static_cast<int>(threadIdx.x); j < gb; j += T) {
                if (j == p) continue;
                bool nb;
                const int oj = a.perm[j];
                if (MODE == 1) {
                    nb = r2_fp64<DIM>(a.spos + static_cast<size_t>(p) * 4, a.spos + static_cast<size_t>(j) * 4) <= fr.R2;
                } else {
                    const ushort4 v = a.q4[j];
                    const uint32_t kj = a.skey[j] - scoff;
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
                    nb = (MODE == 2 || band) ? recheck_g<DIM>(sd.pos, pi, oj - sd.poff, fr.R2) : in16;
                }
                if (nb && (!a.half || oj > oi)) {
                    const int slot = atomicAdd(&fill, 1);
                    if (slot < rlen && room) col[slot] = oj - sd.poff;
                }
            }
        }
        __syncthreads();
        const int L = fill;
        if (L != rlen || !room) {
            if (threadIdx.x == 0) atomicOr(a.err, !room ? kErrCapacity : kErrLongRow);
            __syncthreads();
            continue;
        }
        // 2. sort the row's column indices (distinct keys): rows of up to 512 entries in the
        // registers of the first wavefront (no workgroup barrier inside the network), longer
        // ones in LDS chunks merged pairwise below
        const int K = L <= 512 ? 512 : a.lr_keys;
        if (L <= 512) {
            if (threadIdx.x < 64) {
                if (L <= 64) wave_sort_row<1>(col, L);
                else if (L <= 128) wave_sort_row<2>(col, L);
                else if (L <= 256) wave_sort_row<4>(col, L);
                else wave_sort_row<8>(col, L);
            }
            __syncthreads();
        }
        for (int c0 = 0; L > 512 && c0 < L; c0 += K) {
            const int len = min(K, L - c0);
            int P = 1;
            while (P < len) P <<= 1;
            for (int i = threadIdx.x; i < P; i += T) keys[i] = i < len ? static_cast<uint32_t>(col[c0 + i]) : 0xFFFFFFFFu;
            __syncthreads();
            for (int k = 2; k <= P; k <<= 1) {
                for (int j = k >> 1; j > 0; j >>= 1) {
                    for (int t = threadIdx.x; t < P / 2; t += T) {
                        int i0, i1;
                        if (j == (k >> 1)) {
                            i0 = (t / j) * k + (t % j);
                            i1 = (t / j) * k + (k - 1 - (t % j));
                        } else {
                            i0 = (t / j) * 2 * j + (t % j);
                            i1 = i0 + j;
                        }
                        const uint32_t u = keys[i0], v = keys[i1];
                        if (u > v) {
                            keys[i0] = v;
                            keys[i1] = u;
                        }
                    }
                    __syncthreads();
                }
            }
            for (int i = threadIdx.x; i < len; i += T) col[c0 + i] = static_cast<int32_t>(keys[i]);
            __syncthreads();
        }
        // merge sorted runs of width K, 2K, ... between the column slots and the
        // distance slots (reinterpreted as 32-bit keys)
        NNPS_GLOBAL uint32_t* src = (NNPS_GLOBAL uint32_t*)col;
        NNPS_GLOBAL uint32_t* dst = (NNPS_GLOBAL uint32_t*)(sd.dist + rs);
        for (int width = K; width < L; width <<= 1) {
            for (int e = threadIdx.x; e < L; e += T) {
                const int run = e / width;
                const int base = (run & ~1) * width;           // start of the pair of runs
                const int mid = min(base + width, L), end = min(base + 2 * width, L);
                const uint32_t v = src[e];
                // position among the other run: keys are distinct
                int lo, hi, own;
                if (e < mid) { lo = mid; hi = end; own = e - base; }
                else { lo = base; hi = mid; own = e - mid; }
                int cnt = 0, l = lo, r = hi;
                while (l < r) {
                    const int m = (l + r) >> 1;
                    if (src[m] < v) l = m + 1;
                    else r = m;
                }
                cnt = l - lo;
                dst[base + own + cnt] = v;
            }
            __syncthreads();
            NNPS_GLOBAL uint32_t* tmp = src;
            src = dst;
            dst = tmp;
        }
        if (src != (NNPS_GLOBAL uint32_t*)col) {
            for (int e = threadIdx.x; e < L; e += T) col[e] = static_cast<int32_t>(src[e]);
            __syncthreads();
        }
        // 3. distances of the sorted row
        for (int e = threadIdx.x; e < L; e += T) {
            const int lj = col[e];
            sd.dist[rs + e] = MODE == 1 ? dist_fp64<DIM>(sdesc.pos, li, lj)
                                        : dist_fixed<DIM>(a.X, oi, lj + sd.poff, fr.dist_scale);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Grid of the block kernels: a whole number of rounds over the XCDs, so xcd_block reaches
// every block of any count up to nblk_max.
static dim3 block_grid(int nblk_max) { return dim3((nblk_max + kXcds - 1) / kXcds * kXcds); }

hipError_t launch_count(const SearchArgs& a, int nblk_max, hipStream_t st)
{
    if (a.L.ntot == 0 || nblk_max == 0) return hipSuccess;
    const dim3 g = block_grid(nblk_max), b(64);
    const int d = a.L.dim, m = a.L.mode;
    if (a.half) {
        if (d == 2 && m == 0) hipLaunchKernelGGL((k_count16<2, 0, true>), g, b, 0, st, a);
        else if (d == 3 && m == 0) hipLaunchKernelGGL((k_count16<3, 0, true>), g, b, 0, st, a);
        else if (d == 2 && m == 2) hipLaunchKernelGGL((k_count16<2, 2, true>), g, b, 0, st, a);
        else if (d == 3 && m == 2) hipLaunchKernelGGL((k_count16<3, 2, true>), g, b, 0, st, a);
        else if (d == 2 && m == 3) hipLaunchKernelGGL((k_count32<2, true>), g, b, 0, st, a);
        else if (d == 3 && m == 3) hipLaunchKernelGGL((k_count32<3, true>), g, b, 0, st, a);
        else if (d == 2) hipLaunchKernelGGL((k_count64<2, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_count64<3, true>), g, b, 0, st, a);
        return hipGetLastError();
    }
    if (d == 2 && m == 0) hipLaunchKernelGGL((k_count16<2, 0, false>), g, b, 0, st, a);
    else if (d == 3 && m == 0) hipLaunchKernelGGL((k_count16<3, 0, false>), g, b, 0, st, a);
    else if (d == 2 && m == 2) hipLaunchKernelGGL((k_count16<2, 2, false>), g, b, 0, st, a);
    else if (d == 3 && m == 2) hipLaunchKernelGGL((k_count16<3, 2, false>), g, b, 0, st, a);
    else if (d == 2 && m == 3) hipLaunchKernelGGL((k_count32<2, false>), g, b, 0, st, a);
    else if (d == 3 && m == 3) hipLaunchKernelGGL((k_count32<3, false>), g, b, 0, st, a);
    else if (d == 2) hipLaunchKernelGGL((k_count64<2, false>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_count64<3, false>), g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_stats(const SearchArgs& a, hipStream_t st)
{
    if (a.L.ntot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_stats, dim3(1), dim3(1024), 0, st, a.blk_stats, a.nblk,
                       static_cast<const unsigned long long*>(a.dstats), a.dstats ? a.dgrid : 0, a.stats);
    return hipGetLastError();
}

hipError_t launch_fill(const SearchArgs& a, int nblk_max, hipStream_t st)
{
    if (a.L.ntot == 0 || nblk_max == 0) return hipSuccess;
    const dim3 g = block_grid(nblk_max), b(kFillThreads);
    const int d = a.L.dim, m = a.L.mode == 3 ? 1 : a.L.mode;  // FP32 mode: binary64 distances
    if (d == 2 && m == 0) hipLaunchKernelGGL((k_fill<2, 0>), g, b, 0, st, a);
    else if (d == 3 && m == 0) hipLaunchKernelGGL((k_fill<3, 0>), g, b, 0, st, a);
    else if (d == 2 && m == 2) hipLaunchKernelGGL((k_fill<2, 2>), g, b, 0, st, a);
    else if (d == 3 && m == 2) hipLaunchKernelGGL((k_fill<3, 2>), g, b, 0, st, a);
    else if (d == 2) hipLaunchKernelGGL((k_fill<2, 1>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_fill<3, 1>), g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_long_rows(const SearchArgs& a, int grid, hipStream_t st)
{
    if (a.L.ntot == 0) return hipSuccess;
    const int d = a.L.dim, m = a.L.mode == 3 ? 1 : a.L.mode;  // FP32 mode: long rows in FP64
    const dim3 gh(grid), bh(kLongThreads);
    const size_t lds = static_cast<size_t>(a.lr_keys) * 4;
    if (d == 2 && m == 0) hipLaunchKernelGGL((k_long<2, 0>), gh, bh, lds, st, a);
    else if (d == 3 && m == 0) hipLaunchKernelGGL((k_long<3, 0>), gh, bh, lds, st, a);
    else if (d == 2 && m == 2) hipLaunchKernelGGL((k_long<2, 2>), gh, bh, lds, st, a);
    else if (d == 3 && m == 2) hipLaunchKernelGGL((k_long<3, 2>), gh, bh, lds, st, a);
    else if (d == 2) hipLaunchKernelGGL((k_long<2, 1>), gh, bh, lds, st, a);
    else hipLaunchKernelGGL((k_long<3, 1>), gh, bh, lds, st, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dense-cell path. A work unit is up to kDenseSlice targets of one dense cell, all with
// the same stencil union (the cell's list, ascending original index). A workgroup of four
// wavefronts (eight in the fill that takes the count's kept bits) takes units from a
// counter; for each chunk of candidates (kDenseChunkF16 in the FP16 modes, kDenseChunk in
// FP64) it stages their FP16 pair records and original indices (and, for the fill, FP64
// positions) in LDS, then each wavefront runs its targets one at a time over the chunk.
// Lane L tests a contiguous run of the chunk's candidates, two per packed FP16
// instruction with the same op sequence as the block kernels, and band pairs are settled
// by the FP64 recheck (on the staged positions in the fill). A target's accepted
// candidates thus come out lane by lane in row order: the fill places them with one
// wavefront prefix sum of the lanes' counts, queues them per lane and writes them 64 at a
// time, so consecutive lanes store consecutive CSR entries and the row comes out
// ascending. In the FP16 modes the count keeps each lane's accepted bits of every
// (target, chunk) when the buffer holds them; the fill then reads them back instead of
// testing again and stages only original indices and positions.
// Wavefront w of a unit's W holds targets w, w + W, ...: lane k keeps target w + W k's data
// in registers, read by the whole wavefront with readlane when its turn comes.
__device__ __forceinline__ int rl32(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
// A pointer every lane holds, marked wave-uniform (scalar registers), so that stores through
// it can take a 32-bit per-lane offset.
template <typename T>
__device__ __forceinline__ NNPS_GLOBAL T* uniform_ptr(NNPS_GLOBAL T* p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (NNPS_GLOBAL T*)((static_cast<uint64_t>(hi) << 32) | lo);
}
__device__ __forceinline__ long long rl64(long long v, int k)
{
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(v & 0xFFFFFFFF), k);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), k);
    return (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo);
}
__device__ __forceinline__ double rlf64(double v, int k)
{
    return __builtin_bit_cast(double, rl64(__builtin_bit_cast(long long, v), k));
}

// BITS: the FP16 fill that takes the count's kept bits. It holds no pair records, so
// eight wavefronts share one staged chunk (about 34 KB of LDS) and six wavefronts per SIMD
// fit, where the passes that test run four wavefronts per workgroup and four or five per
// SIMD.
template <int DIM, int MODE, bool FILL, bool BITS = false>
__global__ void __launch_bounds__(BITS ? kDenseBitsThreads : kDenseThreads)
    __attribute__((amdgpu_waves_per_eu(BITS ? 6 : 4))) k_dense(SearchArgs a)
{
    constexpr int NTH = BITS ? kDenseBitsThreads : kDenseThreads;  // threads per workgroup
    constexpr int NWV = NTH / 64;                                  // wavefronts per workgroup
    constexpr bool F16 = MODE != 1;
    static_assert(!BITS || (FILL && F16), "only the FP16 fill takes the count's bits");
    constexpr bool kTest = F16 && !BITS;  // the pass tests candidates in FP16
    constexpr int K = F16 ? kDenseChunkF16 : kDenseChunk;
    constexpr int QCAP = kDenseQueue;
    static_assert(K % 128 == 0 && K <= 2048, "whole 128-candidate groups, chunk positions fit 16 bits");
    static_assert(QCAP >= 64 && K <= 65536, "a queue holds a full store; chunk positions fit 16 bits");
    static_assert(!F16 || K / 128 <= 7, "a lane's accepted bits of a chunk fit 14 bits");
    __shared__ uint4 recA[kTest ? K / 2 : 1];             // qx, qy, qz, 2(c_x - c_jx) pairs
    __shared__ uint2 recB[kTest ? K / 2 : 1];             // 2(c_y - c_jy), 2(c_z - c_jz) pairs
    __shared__ __attribute__((aligned(16))) int sorig[K];
    // candidates' FP64 positions: [K][DIM] (baseline), axis-major [DIM][K] (FP16 fill)
    __shared__ double sdbl[(!F16 || FILL) ? K * DIM : 1];
    double* const spj = sdbl;
    __shared__ unsigned long long s_red[FILL ? 1 : kDenseThreads / 64][kDenseStats];  // count pass only
    // fill: per-wavefront queues of a row's accepted candidates in a chunk (chunk positions,
    // in row order)
    __shared__ uint16_t squeue[FILL ? NWV * QCAP : 1];
    // FP16 count keeping its bits: eight targets' bit words per wavefront, stored together
    __shared__ uint16_t sbits[(!FILL && F16) ? (kDenseThreads / 64) * 8 * 64 : 1];
    // fill: each target's position in the union (found while staging; kNotSeen before)
    __shared__ int sself[FILL ? kDenseSlice : 1];
    constexpr int kNotSeen = 1 << 30;
    // the unit counter's broadcast slot: the first record word, free between the last use of
    // one unit's staged chunk and the staging of the next unit's first chunk
    int* const s_unit = reinterpret_cast<int*>(recA);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int nunits = *a.dn > 0 ? a.unit_off[a.L.ncell_tot] : 0;
    // FP16: the count keeps the accepted bits of every (target, chunk) when they fit, and
    // the fill then takes them instead of testing again. The host launches both FP16 fills;
    // the one that does not apply returns here.
    const bool bits_fit = F16 && a.dbits && nunits > 0 && a.dboff[a.L.ncell_tot] * 64 <= a.dbits_cap;
    if (FILL && F16 && bits_fit != BITS) return;
    const bool bits = FILL ? BITS : bits_fit;
    unsigned long long tc[kDenseStats] = {0, 0, 0, 0, 0, 0};
    for (;;) {
        __syncthreads();  // the previous unit is done with s_unit and the staged chunk
        if (threadIdx.x == 0) *s_unit = atomicAdd(a.ucount, 1);
        __syncthreads();
        const int u = *s_unit;
        if (u >= nunits) break;
        const int g = a.ucell[u];
        const int slice = u - a.unit_off[g];
        const SetDesc& sdesc = a.L.sets[find_set(a.L.coffs, a.L.nsets, g)];
        const SetView sd(sdesc);
        const int poff = sd.poff;
        const double R2 = sdesc.fr.R2;
        const int ncx = sdesc.fr.nc[0], ncy = sdesc.fr.nc[1];
        const uint32_t coff = static_cast<uint32_t>(sdesc.coff);
        const int lk = g - sdesc.coff;
        const int cx = lk % ncx, crow = lk / ncx, cy = crow % ncy, cz = crow / ncy;
        const int t0 = a.cell_start[g] + slice * kDenseSlice;
        const int t1 = min(a.cell_start[g + 1], t0 + kDenseSlice);
        const int U = a.usz[g];
        const int64_t ub = a.uoff[g];
        const int nchunk = (U + K - 1) / K;
        // this wavefront's first (target, chunk) bit row: targets wv + NWV k of the unit
        const int64_t brow = bits ? a.dboff[g] + static_cast<int64_t>(slice * kDenseSlice + wv) * nchunk : 0;
        Thresh th;
        th.init(sdesc.fr);
        const uint16_t tmid = sdesc.fr.t_mid;
        const uint16_t tlo = sdesc.fr.t_lo;
        // this lane's target (held for the wavefront)
        const int pk = t0 + wv + NWV * lane;
        const bool vk = pk < t1;
        const int nt = (t1 - t0 > wv) ? (t1 - t0 - wv + NWV - 1) / NWV : 0;
        int oi_k = 0, q01_k = 0, q2_k = 0, acc_k = 0, rl_k = 0;
        long long rs_k = 0;
        double pi_k[3] = {0, 0, 0};
        if (vk) {
            oi_k = a.perm[pk];
            const int li = oi_k - poff;
#pragma unroll
            for (int k = 0; k < DIM; ++k) pi_k[k] = sd.pos[static_cast<size_t>(li) * DIM + k];
            if (F16) {
                const ushort4 q = a.q4[pk];
                q01_k = static_cast<int>(static_cast<uint32_t>(q.x) | (static_cast<uint32_t>(q.y) << 16));
                q2_k = static_cast<int>(q.z);
            }
            if (FILL) {
                rs_k = sd.row_ptr[li];
                rl_k = static_cast<int>(sd.row_ptr[li + 1] - rs_k);
            } else {
                tc[0] += static_cast<unsigned long long>(U - 1);
                tc[5] += 1;
            }
        }
        if (FILL) {
            for (int t = threadIdx.x; t < kDenseSlice; t += NTH) sself[t] = kNotSeen;
        }
        for (int c0 = 0; c0 < U; c0 += K) {
            const int nc = min(K, U - c0);
            // lane L tests the chunk's candidates 2 L nit ... 2 (L + 1) nit - 1, pair by pair
            // (pair L nit + it at iteration it), so a target's accepted candidates come out
            // in order lane by lane
            const int nit = (nc + 127) >> 7;
            __syncthreads();
            // stage the chunk (padding tests as +inf / far away: never a neighbour)
            if constexpr (BITS) {
                // the fill with the count's bits: original indices and FP64 positions only
                for (int e = threadIdx.x; e < K; e += NTH) {
                    if (e < nc) {
                        const int j = a.ulist[ub + c0 + e];
                        const int oj = a.perm[j];
                        sorig[e] = oj;
#pragma unroll
                        for (int k = 0; k < DIM; ++k)
                            spj[k * K + e] = a.spos ? a.spos[static_cast<size_t>(j) * 4 + k]
                                                    : sd.pos[static_cast<size_t>(oj - poff) * DIM + k];
                        if (j >= t0 && j < t1) sself[j - t0] = c0 + e;  // a target of this unit
                    } else {
                        sorig[e] = -1;
                    }
                }
            } else if constexpr (F16) {
                // pair m goes to record slot (m mod nit) 64 + m / nit: the test reads slot
                // it 64 + lane, consecutive lanes, at iteration it
                for (int m = threadIdx.x; m < 64 * nit; m += NTH) {
                    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, w4 = 0, w5 = 0;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int e = 2 * m + h;
                        const uint32_t sh = 16u * h;
                        if (e < nc) {
                            const int j = a.ulist[ub + c0 + e];
                            const ushort4 v = a.q4[j];
                            const uint32_t kj = a.skey[j] - coff;
                            const int xj = static_cast<int>(kj % static_cast<uint32_t>(ncx));
                            const uint32_t rj = kj / static_cast<uint32_t>(ncx);
                            const int yj = static_cast<int>(rj % static_cast<uint32_t>(ncy));
                            const int zj = static_cast<int>(rj / static_cast<uint32_t>(ncy));
                            const _Float16 c2x = static_cast<_Float16>(2 * (cx - xj));
                            const _Float16 c2y = static_cast<_Float16>(2 * (cy - yj));
                            const _Float16 c2z = static_cast<_Float16>(2 * (cz - zj));
                            w0 |= static_cast<uint32_t>(v.x) << sh;
                            w1 |= static_cast<uint32_t>(v.y) << sh;
                            w2 |= static_cast<uint32_t>(v.z) << sh;
                            w3 |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, c2x)) << sh;
                            w4 |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, c2y)) << sh;
                            w5 |= static_cast<uint32_t>(__builtin_bit_cast(uint16_t, c2z)) << sh;
                            const int oj = a.perm[j];
                            sorig[e] = oj;
                            if (FILL) {
#pragma unroll
                                for (int k = 0; k < DIM; ++k)
                                    spj[k * K + e] = a.spos ? a.spos[static_cast<size_t>(j) * 4 + k]
                                                        : sd.pos[static_cast<size_t>(oj - poff) * DIM + k];
                                if (j >= t0 && j < t1) sself[j - t0] = c0 + e;  // a target of this unit
                            }
                        } else {
                            w0 |= 0x7C00u << sh;  // qx = +inf: r2 = +inf
                            sorig[e] = -1;
                        }
                    }
                    const int slot = (m % nit) * 64 + m / nit;
                    recA[slot] = make_uint4(w0, w1, w2, w3);
                    recB[slot] = make_uint2(w4, w5);
                }
            } else {
                for (int e = threadIdx.x; e < K; e += NTH) {
                    if (e < nc) {
                        const int j = a.ulist[ub + c0 + e];
                        sorig[e] = a.perm[j];
                        if (FILL && j >= t0 && j < t1) sself[j - t0] = c0 + e;  // a target of this unit
#pragma unroll
                        for (int k = 0; k < DIM; ++k) spj[e * DIM + k] = a.spos[static_cast<size_t>(j) * 4 + k];
                    } else {
                        sorig[e] = -1;
#pragma unroll
                        for (int k = 0; k < DIM; ++k) spj[e * DIM + k] = 1e300;  // r2 = +inf
                    }
                }
            }
            __syncthreads();
            // bit row of target k of this wavefront in this chunk
            auto bit_index = [&](int k) {
                return (brow + static_cast<int64_t>(NWV * k) * nchunk + c0 / K) * 64 + lane;
            };
            // the fill's emission of target k's accepted candidates in this chunk: bit j of
            // M is the lane's candidate 2 lane nit + j
            auto fill_row = [&](int k, uint32_t M, const double* pi) {
                // ascending emission: candidate order is original-index order and a lane
                // holds a contiguous run of it, so a lane's accepted candidates go to the row's
                // slots after those of the lanes below it (a wave prefix of the lanes' counts).
                // They pass through the wavefront's queue in LDS, where each lane writes its
                // own in order; then lane i takes entries i, i + 64, ..., computes their
                // distances and writes them, so every store covers 64 consecutive slots with
                // all lanes active
                const long long rs = rl64(rs_k, k);
                const int rl = rl32(rl_k, k);
                const int done = rl32(acc_k, k);
                const bool room = rs + rl <= sd.capacity;
                const double* pis = pi;
                // the row's output, wave-uniform: entries are addressed by a 32-bit slot
                NNPS_GLOBAL int32_t* const rcol = uniform_ptr(sd.col + rs);
                NNPS_GLOBAL float* const rdist = uniform_ptr(sd.dist + rs);
                auto emit = [&](int e, int slot, int oj) {
                    if (slot < rl && room) {
                        float dv;
                        if (F16) {
                            // the FP64 displacement rounded once to FP32 per axis
                            float s2 = 0.0f;
#pragma unroll
                            for (int d = 0; d < DIM; ++d) {
                                const float f = static_cast<float>(spj[d * K + e] - pi[d]);
                                s2 = s2 + f * f;
                            }
                            dv = __builtin_amdgcn_sqrtf(s2);
                        } else {
                            dv = static_cast<float>(__dsqrt_rn(r2_fp64<DIM>(pis, spj + e * DIM)));
                        }
                        if (rl <= (1 << 30)) {  // byte offsets within the row fit 32 bits
                            const uint32_t off = static_cast<uint32_t>(slot) * 4u;
                            *(NNPS_GLOBAL int32_t*)((NNPS_GLOBAL char*)rcol + off) = oj - poff;
                            *(NNPS_GLOBAL float*)((NNPS_GLOBAL char*)rdist + off) = dv;
                        } else {
                            rcol[slot] = oj - poff;
                            rdist[slot] = dv;
                        }
                    }
                };
                // the target itself is never its own neighbour and half lists keep only
                // larger original indices: the union is in original-index order, so both
                // are a condition on the chunk position against the target's own, p
                const int p = sself[wv + NWV * k] - c0;
                const int lb = 2 * lane * nit;  // the lane's first candidate
                const int d = p - lb;
                if (a.half) M &= d < 0 ? 0xFFFFu : (d >= 15 ? 0u : (0xFFFEu << d) & 0xFFFFu);
                else if (p >= 0 && p < nc && d >= 0 && d < 2 * nit) M &= ~(1u << d);
                int tot;
                const int base = wave_excl_scan_i32(__builtin_popcount(M), &tot);
                if (tot <= QCAP) {
                    uint16_t* const q = squeue + wv * QCAP;
                    int pos = base;
                    for (uint32_t mm = M; mm; mm &= mm - 1) q[pos++] = static_cast<uint16_t>(lb + __builtin_ctz(mm));
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    for (int q0 = 0; q0 < tot; q0 += 64) {
                        if (q0 + lane < tot) {
                            const int e = q[q0 + lane];
                            emit(e, done + q0 + lane, sorig[e]);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                } else {
                    // more than the queue holds (a chunk with most candidates accepted): each
                    // lane writes its own entries
                    int pos = done + base;
                    for (uint32_t mm = M; mm; mm &= mm - 1) {
                        const int e = lb + __builtin_ctz(mm);
                        emit(e, pos++, sorig[e]);
                    }
                }
                const int w = done + tot;
                if (!room && lane == 0 && w > done) atomicOr(a.err, kErrCapacity);
                if (lane == k) acc_k = w;
            };
            if constexpr (BITS) {
                // the count's bits, loaded for eight targets at a time and packed two to a
                // register at once (waiting for a load also waits for every store issued
                // before it, so that wait is paid once per eight rows); each row takes the
                // low half and the rest shift down
                uint32_t wp0 = 0, wp1 = 0, wp2 = 0, wp3 = 0;
                for (int k = 0; k < nt; ++k) {
                    if ((k & 7) == 0) {
                        uint32_t wb[8];
#pragma unroll
                        for (int t = 0; t < 8; ++t) wb[t] = a.dbits[bit_index(min(k + t, nt - 1))];
                        wp0 = wb[0] | (wb[1] << 16);
                        wp1 = wb[2] | (wb[3] << 16);
                        wp2 = wb[4] | (wb[5] << 16);
                        wp3 = wb[6] | (wb[7] << 16);
                    }
                    const uint32_t w16 = wp0 & 0xFFFFu;
                    wp0 = (wp0 >> 16) | (wp1 << 16);
                    wp1 = (wp1 >> 16) | (wp2 << 16);
                    wp2 = (wp2 >> 16) | (wp3 << 16);
                    wp3 >>= 16;
                    double pi[3];
#pragma unroll
                    for (int d = 0; d < 3; ++d) pi[d] = rlf64(pi_k[d], k);
                    fill_row(k, w16, pi);
                }
            } else {
                for (int k = 0; k < nt; ++k) {
                    const int oi = rl32(oi_k, k);
                    double pi[3] = {0.0, 0.0, 0.0};
                    // the FP16 count needs the target's FP64 position only for a band recheck
                    if (!F16 || FILL) {
#pragma unroll
                        for (int d = 0; d < 3; ++d) pi[d] = rlf64(pi_k[d], k);
                    }
                    uint32_t inb = 0, bnd = 0, gt = 0;
                    {
                        h2 qix2, qiy2, qiz2;
                        if (F16) {
                            const uint32_t q01 = static_cast<uint32_t>(rl32(q01_k, k));
                            const uint32_t q2 = static_cast<uint32_t>(rl32(q2_k, k));
                            qix2 = splat(as_f16(static_cast<uint16_t>(q01 & 0xFFFF)));
                            qiy2 = splat(as_f16(static_cast<uint16_t>(q01 >> 16)));
                            qiz2 = splat(as_f16(static_cast<uint16_t>(q2 & 0xFFFF)));
                        }
                        // candidate bits: bit it for candidate 2 (lane nit + it), bit 16 + it for the
                        // one after it; "in" and "in or band" from the sign bits of two 16-bit
                        // subtractions
                        uint32_t ebits = 0;
#pragma unroll
                        for (int it = 0; it < K / 128; ++it) {
                            if (it >= nit) break;
                            const int m = it * 64 + lane;  // record slot of pair lane nit + it
                            const int e0 = 2 * (lane * nit + it);
                            if (!FILL && a.half) {  // half lists: candidates of larger original index
                                const int2 oo = *reinterpret_cast<const int2*>(&sorig[e0]);
                                gt |= (oo.x > oi ? 1u << it : 0u) | (oo.y > oi ? 1u << (16 + it) : 0u);
                            }
                            if (F16) {
                                const uint4 A = recA[m];
                                const uint2 B = recB[m];
                                const h2 s = qix2 - as_h2(A.x);
                                const h2 tx = s + as_h2(A.w);
                                const h2 ay = qiy2 + as_h2(B.x);
                                const h2 ty = ay - as_h2(A.y);
                                h2 r2;
                                if (DIM == 3) {
                                    const h2 az = qiz2 + as_h2(B.y);
                                    const h2 tz = az - as_h2(A.z);
                                    r2 = tz * tz;
                                    r2 = __builtin_elementwise_fma(ty, ty, r2);
                                } else {
                                    r2 = ty * ty;
                                }
                                r2 = __builtin_elementwise_fma(tx, tx, r2);
                                const u16x2 dd = as_u16x2(as_u32(r2)) - th.tlo2;
                                const u16x2 ee = dd - th.w12;
                                inb |= (u16x2_bits(dd) >> (15 - it)) & (0x10001u << it);
                                ebits |= (u16x2_bits(ee) >> (15 - it)) & (0x10001u << it);
                            } else {
#pragma unroll
                                for (int h = 0; h < 2; ++h)
                                    if (r2_fp64<DIM>(pi, spj + (e0 + h) * DIM) <= R2) inb |= 1u << (it + 16 * h);
                            }
                        }
                        bnd = ebits & ~inb;
                        // the FP64 recheck of candidate e: from its staged position in the fill
                        auto recheck = [&](int e, int oj) -> bool {
                            if constexpr (FILL && F16) {
                                double pj[3];
#pragma unroll
                                for (int d = 0; d < DIM; ++d) pj[d] = spj[d * K + e];
                                return r2_fp64<DIM>(pi, pj) <= R2;
                            } else if constexpr (F16) {
                                double pt[3];
#pragma unroll
                                for (int d = 0; d < 3; ++d) pt[d] = rlf64(pi_k[d], k);
                                return recheck_g<DIM>(sd.pos, pt, oj - poff, R2);
                            } else {
                                return recheck_g<DIM>(sd.pos, pi, oj - poff, R2);
                            }
                        };
                        if (MODE == 2) {
                            // every candidate decided in FP64; the FP16 classes are only compared
                            uint32_t all = 0;
                            for (int it = 0; it < nit; ++it) {
                                const int e0 = 2 * (lane * nit + it);
                                all |= (e0 < nc ? 1u << it : 0u) | (e0 + 1 < nc ? 1u << (16 + it) : 0u);
                            }
                            uint32_t dec = 0;
                            while (all) {
                                const int bb = __builtin_ctz(all);
                                all &= all - 1;
                                const int e = 2 * (lane * nit + (bb & 15)) + (bb >> 4);
                                const int oj = sorig[e];
                                if (oj == oi) continue;
                                const bool truth = recheck(e, oj);
                                if (truth) dec |= 1u << bb;
                                if (!FILL) {
                                    const bool band = (bnd >> bb) & 1u;
                                    const bool in16 = (inb >> bb) & 1u;
                                    // naive FP16 test: r2 <= RN16(4 rho^2), from the staged record
                                    const uint4 A = recA[(bb & 15) * 64 + lane];
                                    const uint2 B = recB[(bb & 15) * 64 + lane];
                                    const h2 s = qix2 - as_h2(A.x);
                                    const h2 tx = s + as_h2(A.w);
                                    const h2 ty = (qiy2 + as_h2(B.x)) - as_h2(A.y);
                                    h2 r2;
                                    if (DIM == 3) {
                                        const h2 tz = (qiz2 + as_h2(B.y)) - as_h2(A.z);
                                        r2 = tz * tz;
                                        r2 = __builtin_elementwise_fma(ty, ty, r2);
                                    } else {
                                        r2 = ty * ty;
                                    }
                                    r2 = __builtin_elementwise_fma(tx, tx, r2);
                                    const uint16_t r2h = static_cast<uint16_t>((as_u32(r2) >> (16 * (e & 1))) & 0xFFFF);
                                    const bool naive = r2h <= tmid;
                                    tc[1] += band;
                                    tc[2] += naive && !truth;
                                    tc[3] += !naive && truth;
                                    tc[4] += !band && (in16 != truth);
                                }
                            }
                            inb = dec;
                        } else if (MODE == 0) {
                            uint32_t bb_all = bnd;
                            while (bb_all) {
                                const int bb = __builtin_ctz(bb_all);
                                bb_all &= bb_all - 1;
                                const int e = 2 * (lane * nit + (bb & 15)) + (bb >> 4);
                                const int oj = sorig[e];
                                if (oj == oi) continue;  // itself (a band pair only when T_lo = 0)
                                const bool truth = recheck(e, oj);
                                if (truth) inb |= 1u << bb;
                                if (!FILL) {
                                    const uint4 A = recA[(bb & 15) * 64 + lane];
                                    const uint2 B = recB[(bb & 15) * 64 + lane];
                                    const h2 s = qix2 - as_h2(A.x);
                                    const h2 tx = s + as_h2(A.w);
                                    const h2 ty = (qiy2 + as_h2(B.x)) - as_h2(A.y);
                                    h2 r2;
                                    if (DIM == 3) {
                                        const h2 tz = (qiz2 + as_h2(B.y)) - as_h2(A.z);
                                        r2 = tz * tz;
                                        r2 = __builtin_elementwise_fma(ty, ty, r2);
                                    } else {
                                        r2 = ty * ty;
                                    }
                                    r2 = __builtin_elementwise_fma(tx, tx, r2);
                                    const uint16_t r2h = static_cast<uint16_t>((as_u32(r2) >> (16 * (e & 1))) & 0xFFFF);
                                    const bool naive = r2h <= tmid;
                                    tc[1] += 1;
                                    tc[2] += naive && !truth;
                                    tc[3] += !naive && truth;
                                }
                            }
                        }
                        if (!FILL && bits) {
                            // the decided bits, before the half-list mask; stored eight targets at
                            // a time, so the band recheck's loads seldom wait for a store
                            uint16_t* const cb = sbits + wv * 8 * 64;
                            cb[(k & 7) * 64 + lane] = static_cast<uint16_t>(interleave8(inb & 0x007F007Fu));
                            if ((k & 7) == 7 || k == nt - 1) {
                                const int k0 = k & ~7;
                                for (int t = 0; t <= (k & 7); ++t) a.dbits[bit_index(k0 + t)] = cb[t * 64 + lane];
                            }
                        }
                    }
                    if constexpr (!FILL) {
                        if (a.half) inb &= gt;
                        const int tot = wave_sum_i32(__builtin_popcount(inb));
                        if (lane == k) acc_k += tot;
                    } else {
                        fill_row(k, interleave8(inb), pi);
                    }
                }
            }
        }
        if (vk) {
            if (!FILL) {
                // itself: "in" in FP16 when T_lo > 0, always in the FP64 baseline; never
                // counted when every candidate is decided in FP64 (it is skipped there)
                const int self = a.half ? 0 : (MODE == 1 ? 1 : (MODE == 2 ? 0 : (tlo > 0 ? 1 : 0)));
                a.counts[oi_k] = acc_k - self;
            } else if (acc_k != rl_k) {
                atomicOr(a.err, kErrLongRow);
            }
        }
    }
    if (!FILL) {
#pragma unroll
        for (int k = 0; k < kDenseStats; ++k) {
            const unsigned long long sum = wave_sum_u64(tc[k]);
            if (lane == 0) s_red[wv][k] = sum;
        }
        __syncthreads();
        if (threadIdx.x < kDenseStats) {
            unsigned long long sum = 0;
            for (int w = 0; w < kDenseThreads / 64; ++w) sum += s_red[w][threadIdx.x];
            a.dstats[static_cast<size_t>(blockIdx.x) * kDenseStats + threadIdx.x] = sum;
        }
    }
}

template <int D, int M>
void launch_dense_pass(const SearchArgs& a, bool fill, hipStream_t st)
{
    const dim3 g(a.dgrid), b(kDenseThreads);
    if (!fill) {
        hipLaunchKernelGGL((k_dense<D, M, false>), g, b, 0, st, a);
        return;
    }
    // FP16 fills: both kernels run, and the one that does not match whether the count kept
    // its bits returns at once
    if constexpr (M != 1) hipLaunchKernelGGL((k_dense<D, M, true, true>), g, dim3(kDenseBitsThreads), 0, st, a);
    hipLaunchKernelGGL((k_dense<D, M, true, false>), g, b, 0, st, a);
}

hipError_t launch_dense(const SearchArgs& a, bool fill, hipStream_t st)
{
    if (a.L.ntot == 0 || !a.wdense) return hipSuccess;
    hipError_t e = launch_fill_i32(a.ucount, 1, 0, st);
    if (e != hipSuccess) return e;
    const int d = a.L.dim, m = a.L.mode == 3 ? 1 : a.L.mode;  // FP32 mode: dense cells in FP64
    if (d == 2 && m == 0) launch_dense_pass<2, 0>(a, fill, st);
    else if (d == 3 && m == 0) launch_dense_pass<3, 0>(a, fill, st);
    else if (d == 2 && m == 1) launch_dense_pass<2, 1>(a, fill, st);
    else if (d == 3 && m == 1) launch_dense_pass<3, 1>(a, fill, st);
    else if (d == 2) launch_dense_pass<2, 2>(a, fill, st);
    else launch_dense_pass<3, 2>(a, fill, st);
    return hipGetLastError();
}

}  // namespace nnps
