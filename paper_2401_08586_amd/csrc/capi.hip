// C-ABI entry points (include/nnps.h): argument checks, grid set-up, device buffers
// and the stream-ordered sequence of cell-build and search kernels.
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cstring>
#include <utility>
#include <vector>

#include "../../include/nnps.h"
#include "build_kernels.h"
#include "sph_kernels.h"
#include "allpairs_kernels.h"

using namespace nnps;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        const size_t want = std::max<size_t>(bytes, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Modes that keep sorted FP64 positions (the FP64 test, and the FP32 mode's dense cells
// and long rows).
bool uses_spos(int mode) { return mode == NNPS_MODE_FP64_BASELINE || mode == NNPS_MODE_FP32_RCLL; }

// Round a double to binary32 toward -inf (dir -1), nearest-even (0) or +inf (+1).
float f32_dir(double x, int dir)
{
    float f = static_cast<float>(x);
    if (dir < 0 && static_cast<double>(f) > x) f = nextafterf(f, -INFINITY);
    if (dir > 0 && static_cast<double>(f) < x) f = nextafterf(f, INFINITY);
    return f;
}

// Round a non-negative double to an IEEE binary16 bit pattern: dir 0 = nearest-even,
// -1 = toward -inf, +1 = toward +inf. Negative inputs give 0 (never used otherwise).
uint16_t f16_bits(double x, int dir)
{
    if (!(x > 0.0)) return 0;
    int e2;
    frexp(x, &e2);  // x = f 2^e2, f in [0.5, 1)
    int E = e2 - 1;
    if (E < -14) E = -14;  // subnormal range shares the smallest exponent's step
    const double ulp = ldexp(1.0, E - 10);
    const double m = x / ulp;  // exact: division by a power of two
    double r = dir == 0 ? nearbyint(m) : (dir < 0 ? floor(m) : ceil(m));
    int64_t mi = static_cast<int64_t>(r);
    if (mi >= 2048) {
        mi = 1024;
        ++E;
    }
    if (E + 15 >= 31) return 0x7C00;
    if (mi < 1024) return static_cast<uint16_t>(mi);  // subnormal (E == -14)
    return static_cast<uint16_t>(((E + 15) << 10) | (mi - 1024));
}

int bitlen(int64_t v)
{
    int b = 0;
    while (v > 0) {
        ++b;
        v >>= 1;
    }
    return b;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

nnps_status frame_of(const nnps_problem* p, Frame* fr, int block_target)
{
    nnps_status st = nnps_validate(p);
    if (st != NNPS_OK) return st;
    memset(fr, 0, sizeof(*fr));
    fr->dim = p->dim;
    fr->mode = p->mode;
    fr->n = static_cast<int>(p->n);
    const double w = std::max(p->cell_size, p->radius) * (1.0 + ldexp(1.0, -30));
    int64_t ncest = 1;
    for (int k = 0; k < p->dim; ++k)
        ncest = std::max<int64_t>(ncest, static_cast<int64_t>(floor((p->hi[k] - p->lo[k]) / w)) + 1);
    const int F = std::min(40, 51 - bitlen(ncest));
    const double s = ldexp(1.0, F) / w;
    int64_t ncell = 1;
    for (int k = 0; k < 3; ++k) {
        fr->lo[k] = k < p->dim ? p->lo[k] : 0.0;
        fr->hi[k] = k < p->dim ? p->hi[k] : 0.0;
        if (k < p->dim) {
            const int64_t xh = static_cast<int64_t>(rint((p->hi[k] - p->lo[k]) * s));
            fr->nc[k] = static_cast<int>((xh >> F) + 1);
        } else {
            fr->nc[k] = 1;
        }
        ncell *= fr->nc[k];
    }
    if (ncell > (int64_t(1) << 30)) return NNPS_ETOOMANYCELLS;
    fr->ncell = static_cast<int>(ncell);
    fr->F = F;
    fr->w = w;
    fr->s = s;
    fr->R2 = p->radius * p->radius;
    fr->dist_scale = static_cast<float>(ldexp(w, -F));
    const double rho = p->radius / w;
    const double rho2 = rho * rho;
    const double band = ldexp(1.0, -7);
    fr->t_lo = f16_bits(4.0 * (rho2 - band), -1);
    fr->t_hi = f16_bits(4.0 * (rho2 + band), +1);
    fr->t_mid = f16_bits(4.0 * rho2, 0);
    // FP32 thresholds: band 2^-15 squared cell widths, which covers the FP32 pass's error
    // near the cutoff (fixed point, the stored f32 coordinate and the five f32 roundings
    // of r2) for every admissible F >= 20
    const double band32 = ldexp(1.0, -15);
    fr->t32_lo = std::max(0.0f, f32_dir(4.0 * (rho2 - band32), -1));
    fr->t32_hi = f32_dir(4.0 * (rho2 + band32), +1);
    fr->t32_mid = f32_dir(4.0 * rho2, 0);
    // x-window of a work block: about block_target particles on average, so most windows
    // fill one wavefront and the candidate union stays small; and at most what keeps the
    // union of 3^(d-1) rows of xwin + 2 cells at 85 % of the fill's union limit on average
    const double occ = static_cast<double>(p->n) / static_cast<double>(ncell);
    int xwin = occ > 0.0 ? static_cast<int>(block_target / occ) : kMaxXWin;
    if (occ > 0.0) {
        const double rows = p->dim == 3 ? 9.0 : 3.0;
        const double ucap = p->dim == 3 ? kUnion3 : kUnion2;
        xwin = std::min(xwin, static_cast<int>(0.85 * ucap / (rows * occ)) - 2);
    }
    fr->xwin = std::max(1, std::min(kMaxXWin, xwin));
    // targets per block: at most what keeps the block's CSR entries (targets times the
    // expected neighbours, occupancy times the radius ball in cell units) at 85 % of the
    // fill's entry limit
    const double ball = p->dim == 3 ? 4.18879020478639 * rho * rho * rho : 3.14159265358979 * rho * rho;
    const double nb = occ * ball;
    const double fcap = p->dim == 3 ? kFlat3 : kFlat2;
    const int bm = nb > 0.0 ? static_cast<int>(0.85 * fcap / nb) : kWave;
    fr->bmax = std::max(8, std::min(kWave, bm));
    return NNPS_OK;
}

}  // namespace

struct nnps_ctx {
    int device = 0;
    int64_t* h_pinned = nullptr;  // pinned staging for synchronous read-backs
    // device error words: [0] the all-list count's domain flag; [1] errors of the
    // asynchronous calls (all-list fill, SPH gradient), kept until nnps_ctx_check reads them
    int* d_flag = nullptr;
    int* d_apcnt = nullptr;       // all-list per-slice row counts
    size_t apcnt_cap = 0;         // ints in d_apcnt
    struct {                      // the last successful all-list count (what a fill may follow)
        bool valid = false;
        int dim = 0;
        const double* pos = nullptr;
        const int64_t* row_ptr = nullptr;
        double R2 = 0.0;
        int64_t nnz = 0;
        ApPlan plan;
    } ap;
    int max_lds = 65536;          // LDS bytes a workgroup may use on this device
    nnps_tuning tuning{80, 1024, 0, 0, 0, 0, 0};
};

namespace {

// Per-phase HIP-event timing. Every begin/end pair recorded since the last read is
// kept, so a run of many calls can be summed without synchronising in between.
struct PhaseTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int open[NNPS_NPHASES] = {};
    std::vector<std::pair<int, int>> rec[NNPS_NPHASES];
    hipEvent_t* next()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return &pool[used++];
    }
    void reset()
    {
        used = 0;
        for (auto& r : rec) r.clear();
    }
    void release()
    {
        for (auto& e : pool) (void)hipEventDestroy(e);
        pool.clear();
        reset();
        on = false;
    }
    void begin(int ph, hipStream_t s)
    {
        if (!on) return;
        hipEvent_t* e = next();
        if (!e) return;
        open[ph] = static_cast<int>(e - pool.data());
        (void)hipEventRecord(*e, s);
    }
    void end(int ph, hipStream_t s)
    {
        if (!on) return;
        hipEvent_t* e = next();
        if (!e) return;
        (void)hipEventRecord(*e, s);
        rec[ph].push_back({open[ph], static_cast<int>(e - pool.data())});
    }
};

// A captured build + count + fill sequence and the launch signature it was made for.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    std::vector<unsigned char> sig;
    void reset()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        sig.clear();
    }
};

}  // namespace

struct nnps_cells {
    nnps_ctx* ctx = nullptr;
    PhaseTimer timer;
    GraphCache graph;
    bool use_graphs = false;
    bool half = false;                    // rows keep only neighbours of larger original index
    bool built = false, counted = false;
    int nsets = 0, dim = 0, mode = 0, ntot = 0, ncell_tot = 0, nblk_max = 0;
    std::vector<Frame> frames;
    int nrows_tot = 0;                    // row segments of all sets
    std::vector<const double*> pos;
    SetDesc* h_sets = nullptr;            // pinned mirror of the set table
    int* h_offs = nullptr;                // pinned mirror of the offsets
    int h_cap = 0;                        // sets the pinned mirrors can hold
    hipEvent_t upload_done = nullptr;     // last upload from the pinned mirrors
    bool upload_pending = false;
    // what the device tables hold (bytes of the last upload, and the buffers' generation)
    std::vector<unsigned char> up_sets, up_offs;
    uint64_t up_gen = ~0ull;
    int64_t* h_report = nullptr;          // pinned: nnz per set, then error and dense words
    int h_report_cap = 0;
    hipEvent_t report_done = nullptr;     // the last enqueued report's copies
    bool report_pending = false;
    uint64_t buf_gen = 0;                 // bumps whenever a device buffer moves
    uint32_t* skey = nullptr;
    int* perm = nullptr;
    DevBuf counts_s, rsort, bdesc;
    DevBuf d_sets, d_offs, X, k0, k1, v0, v1, cell_count, cell_start, q4, spos, rq, boff, bstart, bset,
        counts, table, partial, stats, blk_stats, cbits, err, heavy, nheavy, rowg, nnz, sink;
    // dense-cell path (see DenseBuild)
    bool dense = false;         // the tuning allows the dense-cell path
    bool dense_active = false;  // the last build uses it
    int dense_seen = -1;        // dense cells at the last synchronising call: -1 unknown, 0, 1
    int dthresh = 0, dgrid = 0;
    int64_t dcap = 0;
    int* ulist = nullptr;
    DevBuf usz, wdense, uoff, nsl, unit_off, ucell, dn, ecnt, epos, uk0, uk1, uv0, uv1, inv, ucount, dstats, dseen;
    // FP16 dense passes: (target, chunk) offsets per cell and the count's accepted bits,
    // sized at a build from what the last synchronising call found the dense cells need
    DevBuf dbn, dboff, dbits;
    size_t dbits_want = 0;  // bytes
    // incremental update (nnps_cells_update): see Update
    DevBuf uleave, ucs_old, uskey2, uperm2;
    GraphCache ugraph;  // a captured update + count + fill sequence
};

#define HIP_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return NNPS_EDEVICE; \
    } while (0)

namespace {

nnps_status err_status(int err)
{
    if (err & kErrDomain) return NNPS_EDOMAIN;
    if (err & kErrCapacity) return NNPS_ECAPACITY;
    if (err & kErrLongRow) return NNPS_EUNSUPPORTED;
    return NNPS_OK;
}

// Make the pinned mirrors writable again: the previous upload must have been consumed.
nnps_status wait_upload(nnps_cells* c)
{
    if (c->upload_pending) {
        HIP_TRY(hipEventSynchronize(c->upload_done));
        c->upload_pending = false;
    }
    return NNPS_OK;
}

// Queue the copies of the set table (and the offsets) to the device, unless the device
// tables already hold exactly these bytes: no kernel writes them, so they hold what was
// last copied into the same buffers. Repeated steps over the same sets and outputs then
// copy nothing.
nnps_status upload(nnps_cells* c, bool with_offsets, hipStream_t s)
{
    const size_t ns = sizeof(SetDesc) * c->nsets, no = sizeof(int) * 3 * (c->nsets + 1);
    const unsigned char* hs = reinterpret_cast<const unsigned char*>(c->h_sets);
    const unsigned char* ho = reinterpret_cast<const unsigned char*>(c->h_offs);
    const bool gen_ok = c->up_gen == c->buf_gen;
    const bool sets_ok = gen_ok && c->up_sets.size() == ns && memcmp(c->up_sets.data(), hs, ns) == 0;
    const bool offs_ok = !with_offsets || (gen_ok && c->up_offs.size() == no && memcmp(c->up_offs.data(), ho, no) == 0);
    if (sets_ok && offs_ok) return NNPS_OK;
    if (!gen_ok) c->up_offs.clear();  // the offsets buffer moved too: not known to hold anything
    HIP_TRY(hipMemcpyAsync(c->d_sets.p, c->h_sets, ns, hipMemcpyHostToDevice, s));
    c->up_sets.assign(hs, hs + ns);
    if (with_offsets) {
        HIP_TRY(hipMemcpyAsync(c->d_offs.p, c->h_offs, no, hipMemcpyHostToDevice, s));
        c->up_offs.assign(ho, ho + no);
    }
    c->up_gen = c->buf_gen;
    HIP_TRY(hipEventRecord(c->upload_done, s));
    c->upload_pending = true;
    return NNPS_OK;
}

// The FP16 dense passes (FP16 RCLL and its recheck-all mode) may keep the count's
// accepted bits for the fill, within a bound on the scratch (tuning; -1 = never).
bool dense_bits_on(const nnps_cells* c)
{
    return c->dense && (c->mode == NNPS_MODE_FP16_RCLL || c->mode == NNPS_MODE_RECHECK_ALL) &&
           c->ctx->tuning.dense_bits_mib >= 0;
}

size_t dense_bits_bound(const nnps_cells* c)
{
    const int mib = c->ctx->tuning.dense_bits_mib > 0 ? c->ctx->tuning.dense_bits_mib : kDenseBitsMiB;
    return static_cast<size_t>(mib) << 20;
}

// Sorted FP64 positions: always in the FP64 and FP32 modes; in the FP16 modes while the
// dense-cell path runs (its fill stages the candidates' positions from them, contiguous in
// sorted order, instead of gathering them by original index). The pack and the search
// passes of one step see the same answer unless a synchronising call in between finds
// that the dense cells are gone; the dense fill then gathers from the caller's positions.
double* spos_of(const nnps_cells* c)
{
    if (uses_spos(c->mode)) return c->spos.as<double>();
    if (c->dense && c->dense_seen != 0 && c->spos.p && c->spos.cap >= static_cast<size_t>(c->ntot) * 4 * sizeof(double))
        return c->spos.as<double>();
    return nullptr;
}

Launch launch_of(const nnps_cells* c)
{
    Launch L{};
    L.dim = c->dim;
    L.mode = c->mode;
    L.nsets = c->nsets;
    L.ntot = c->ntot;
    L.ncell_tot = c->ncell_tot;
    L.sets = c->d_sets.as<SetDesc>();
    L.poffs = c->d_offs.as<int>();
    L.coffs = c->d_offs.as<int>() + c->nsets + 1;
    L.roffs = c->d_offs.as<int>() + 2 * (c->nsets + 1);
    L.nrows_tot = c->nrows_tot;
    return L;
}

SearchArgs args_of(const nnps_cells* c)
{
    SearchArgs a{};
    a.L = launch_of(c);
    a.skey = c->skey;
    a.perm = c->perm;
    a.cell_start = c->cell_start.as<int>();
    a.q4 = c->q4.as<ushort4>();
    a.spos = spos_of(c);
    a.rq = c->mode == NNPS_MODE_FP32_RCLL ? c->rq.as<float4>() : nullptr;
    a.X = c->X.as<double>();
    a.bstart = c->bstart.as<int>();
    a.bset = c->bset.as<int>();
    a.nblk = c->boff.as<int>() + c->nrows_tot;
    a.counts = c->counts.as<int>();
    a.counts_s = c->counts_s.as<int>();
    a.rsort = c->rsort.as<int64_t>();
    a.bdesc = c->bdesc.as<int>();
    a.heavy = c->heavy.as<int>();
    a.nheavy = c->nheavy.as<int>();
    a.stats = c->stats.as<unsigned long long>();
    a.blk_stats = c->blk_stats.as<unsigned long long>();
    a.cbits = c->cbits.as<uint32_t>();
    int keys = 1;
    while (keys * 2 <= std::min(c->ctx->max_lds - 1024, 64 * 1024) / 4) keys *= 2;
    a.lr_keys = c->ctx->tuning.long_rows_keys > 0 ? std::min(c->ctx->tuning.long_rows_keys, keys) : keys;
    a.err = c->err.as<int>();
    a.sink = c->sink.as<int>();
    a.half = c->half ? 1 : 0;
    if (c->dense_active) {
        a.wdense = c->wdense.as<int>();
        a.usz = c->usz.as<int>();
        a.uoff = c->uoff.as<int64_t>();
        a.ulist = c->ulist;
        a.unit_off = c->unit_off.as<int>();
        a.ucell = c->ucell.as<int>();
        a.dn = c->dn.as<int>();
        a.ucount = c->ucount.as<int>();
        a.dstats = c->dstats.as<unsigned long long>();
        a.dgrid = c->dgrid;
        a.dboff = c->dboff.as<int64_t>();
        if (dense_bits_on(c) && c->dbits.p) {
            a.dbits = c->dbits.as<uint16_t>();
            a.dbits_cap = static_cast<int64_t>(c->dbits.cap / sizeof(uint16_t));
        }
    }
    return a;
}

DenseBuild dense_of(nnps_cells* c)
{
    DenseBuild d{};
    d.thresh = c->dthresh;
    d.cap = c->dcap;
    d.usz = c->usz.as<int>();
    d.wdense = c->wdense.as<int>();
    d.uoff = c->uoff.as<int64_t>();
    d.nsl = c->nsl.as<int>();
    d.unit_off = c->unit_off.as<int>();
    d.ucell = c->ucell.as<int>();
    d.dn = c->dn.as<int>();
    d.ecnt = c->ecnt.as<int>();
    d.epos = c->epos.as<int>();
    d.uk0 = c->uk0.as<uint32_t>();
    d.uk1 = c->uk1.as<uint32_t>();
    d.uv0 = c->uv0.as<int>();
    d.uv1 = c->uv1.as<int>();
    d.table = c->table.as<uint32_t>();
    d.partial = c->partial.as<int64_t>();
    d.seen = c->dseen.as<int>();
    d.dbn = c->dbn.as<int>();
    d.dboff = c->dboff.as<int64_t>();
    return d;
}

// Validate a batch, lay out its grids and index spaces, size the device buffers and fill
// the pinned set table (output pointers cleared). No device work is queued.
nnps_status prepare(nnps_ctx* ctx, nnps_cells* c, int nsets, const nnps_problem* probs, const double* const* d_pos)
{
    if (nsets < 1 || !probs || !d_pos) return NNPS_EINVAL;
    std::vector<Frame> frames(nsets);
    int64_t ntot = 0, ncell = 0;
    for (int s = 0; s < nsets; ++s) {
        nnps_status st = frame_of(&probs[s], &frames[s], ctx->tuning.block_target);
        if (st != NNPS_OK) return st;
        if (probs[s].dim != probs[0].dim || probs[s].mode != probs[0].mode) return NNPS_EINVAL;
        if (probs[s].n > 0 && !d_pos[s]) return NNPS_EINVAL;
        ntot += probs[s].n;
        ncell += frames[s].ncell;
    }
    if (ntot >= (int64_t(1) << 31)) return NNPS_EINVAL;
    if (ncell >= (int64_t(1) << 31)) return NNPS_ETOOMANYCELLS;
    nnps_status st = wait_upload(c);
    if (st != NNPS_OK) return st;
    if (nsets > c->h_cap) {
        if (c->h_sets) (void)hipHostFree(c->h_sets);
        if (c->h_offs) (void)hipHostFree(c->h_offs);
        c->h_sets = nullptr;
        c->h_offs = nullptr;
        c->h_cap = 0;
        if (hipHostMalloc(reinterpret_cast<void**>(&c->h_sets), sizeof(SetDesc) * nsets, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&c->h_offs), sizeof(int) * 3 * (nsets + 1),
                          hipHostMallocDefault) != hipSuccess)
            return NNPS_ENOMEM;
        c->h_cap = nsets;
    }
    if (!c->upload_done && hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess)
        return NNPS_EDEVICE;
    c->nsets = nsets;
    c->dim = probs[0].dim;
    c->mode = probs[0].mode;
    c->ntot = static_cast<int>(ntot);
    c->ncell_tot = static_cast<int>(ncell);
    c->frames = frames;
    c->pos.assign(d_pos, d_pos + nsets);
    const nnps_tuning& tu = ctx->tuning;
    c->dense = tu.dense_min_union >= 0;
    c->dthresh = tu.dense_min_union > 0 ? tu.dense_min_union : (c->dim == 3 ? kDenseUnion3 : kDenseUnion2);
    const int64_t stencil = c->dim == 3 ? 27 : 9;
    int poff = 0, coff = 0, roff = 0;
    int64_t nblk_bound = 0;
    for (int s = 0; s < nsets; ++s) {
        SetDesc& sd = c->h_sets[s];
        memset(&sd, 0, sizeof(sd));
        sd.fr = frames[s];
        sd.poff = poff;
        sd.coff = coff;
        sd.pos = d_pos[s];
        c->h_offs[s] = poff;
        c->h_offs[nsets + 1 + s] = coff;
        c->h_offs[2 * (nsets + 1) + s] = roff;
        const Frame& fr = frames[s];
        const int64_t nrows = static_cast<int64_t>(fr.nc[1]) * fr.nc[2];
        const int64_t nseg = nrows * row_segments(fr.nc[0]);
        // blocks: full ones, at most one per span of xwin cells and one per row segment
        // ending early, and around each run of dense cells one marker plus one cut short
        int64_t b = fr.n / fr.bmax + nrows * ((fr.nc[0] + fr.xwin - 1) / fr.xwin) + nseg;
        if (c->dense && c->dense_seen != 0)  // the build will use the dense-cell path
            b += 2 * std::min<int64_t>(fr.ncell, stencil * fr.n / (static_cast<int64_t>(c->dthresh) + 1));
        nblk_bound += std::min<int64_t>(fr.n, b);
        poff += fr.n;
        coff += fr.ncell;
        roff += static_cast<int>(nseg);
    }
    c->h_offs[nsets] = poff;
    c->h_offs[2 * nsets + 1] = coff;
    c->h_offs[3 * nsets + 2] = roff;
    c->nrows_tot = roff;
    c->nblk_max = static_cast<int>(std::min<int64_t>(nblk_bound, ntot));

    const size_t n = static_cast<size_t>(ntot);
    const size_t nn = std::max<size_t>(n, 1);
    const size_t nc = static_cast<size_t>(ncell);
    // dense-cell path: list capacity min(3^d n, bound)
    c->dgrid = tu.dense_grid > 0 ? tu.dense_grid : kDenseGrid;
    const int64_t dmax = tu.dense_max_entries > 0 ? tu.dense_max_entries : kDenseMaxEntries;
    c->dcap = c->dense ? std::max<int64_t>(1, std::min<int64_t>((c->dim == 3 ? 27 : 9) * static_cast<int64_t>(nn), dmax))
                       : 0;
    const size_t dcap = static_cast<size_t>(c->dcap);
    const size_t table_n = (c->dense ? radix_table_entries(static_cast<int>(dcap)) : size_t(0)) + 1;
    const int64_t scan_m = std::max<int64_t>({static_cast<int64_t>(nn) + 1, static_cast<int64_t>(nc) + 1,
                                              static_cast<int64_t>(table_n),
                                              static_cast<int64_t>(c->nrows_tot) + 1});
    const bool base = uses_spos(c->mode);
    const int cw = c->dim == 3 ? kCandWords3 : kCandWords2;
    struct Need {
        DevBuf* b;
        size_t bytes;
    } need[] = {
        {&c->d_sets, sizeof(SetDesc) * nsets},
        {&c->d_offs, sizeof(int) * 3 * (nsets + 1)},
        {&c->X, nn * x_stride(c->dim) * sizeof(int64_t)},
        {&c->k0, nn * 4}, {&c->k1, nn * 4}, {&c->v0, nn * 4}, {&c->v1, nn * 4},
        {&c->cell_count, (nc + 1) * 4}, {&c->cell_start, (nc + 1) * 4},
        {&c->q4, nn * sizeof(ushort4)},
        {&c->spos, (base || (c->dense && c->dense_seen != 0)) ? nn * 4 * sizeof(double) : 0},
        {&c->rq, c->mode == NNPS_MODE_FP32_RCLL ? nn * sizeof(float4) : 0},
        {&c->boff, (static_cast<size_t>(c->nrows_tot) + 1) * 4}, {&c->bstart, (nn + 2) * 4}, {&c->bset, (nn + 1) * 4},
        {&c->counts, nn * 4}, {&c->counts_s, nn * 4}, {&c->rsort, nn * 8},
        {&c->bdesc, static_cast<size_t>(std::max(c->nblk_max, 1) + kXcdPad) * kBlockDescInts * 4},
        {&c->table, table_n * 4},
        {&c->partial, static_cast<size_t>(scan_partials_needed(scan_m) + 1) * 8},
        {&c->stats, kStCount * 8},
        {&c->blk_stats, static_cast<size_t>(std::max(c->nblk_max, 1)) * 5 * 8},
        {&c->cbits, nn * cw * 4},
        {&c->err, 4}, {&c->heavy, nn * 4}, {&c->nheavy, 4}, {&c->sink, 2 * 64 * 4},
        {&c->rowg, (nn + 1) * 8},
        {&c->nnz, sizeof(int64_t) * nsets},
        {&c->usz, c->dense ? (nc + 1) * 4 : 0}, {&c->wdense, c->dense ? (nc + 1) * 4 : 0},
        {&c->uoff, c->dense ? (nc + 1) * 8 : 0}, {&c->nsl, c->dense ? (nc + 1) * 4 : 0},
        {&c->unit_off, c->dense ? (nc + 1) * 4 : 0}, {&c->ucell, c->dense ? (nn + 1) * 4 : 0},
        {&c->dn, c->dense ? size_t(4) : size_t(0)}, {&c->ecnt, c->dense ? nn * 4 : 0}, {&c->epos, c->dense ? (nn + 1) * 4 : 0},
        {&c->uk0, dcap * 4}, {&c->uk1, dcap * 4}, {&c->uv0, dcap * 4}, {&c->uv1, dcap * 4},
        {&c->inv, nn * 4}, {&c->ucount, c->dense ? size_t(4) : size_t(0)},
        {&c->dstats, c->dense ? static_cast<size_t>(c->dgrid) * kDenseStats * 8 : 0},
        {&c->dseen, c->dense ? size_t(4) : size_t(0)},
        {&c->dbn, c->dense ? (nc + 1) * 4 : 0}, {&c->dboff, c->dense ? (nc + 1) * 8 : 0},
        {&c->dbits, dense_bits_on(c) ? c->dbits_want : 0},
        // leave, arrive (ncell + 1 each) and the migrant bits (ceil(n / 32) words), one block
        {&c->uleave, (2 * (nc + 1) + (nn + 31) / 32) * 4},
        {&c->ucs_old, (nc + 1) * 4}, {&c->uskey2, nn * 4}, {&c->uperm2, nn * 4},
    };
    for (auto& q : need) {
        if (q.bytes == 0) continue;
        void* before = q.b->p;
        hipError_t e = q.b->ensure(q.bytes);
        if (e != hipSuccess) return e == hipErrorOutOfMemory ? NNPS_ENOMEM : NNPS_EDEVICE;
        if (q.b->p != before) ++c->buf_gen;
    }
    c->built = false;
    c->counted = false;
    return NNPS_OK;
}

nnps_status enqueue_build_tail(nnps_cells* c, hipStream_t s);

Update update_of(nnps_cells* c)
{
    Update u{};
    u.knew = c->k0.as<uint32_t>();  // the build's unsorted keys and slots are free after it
    u.aslot = c->v1.as<int>();
    u.leave = c->uleave.as<int>();
    u.arrive = u.leave + c->ncell_tot + 1;
    u.mig = reinterpret_cast<uint32_t*>(u.arrive + c->ncell_tot + 1);
    u.cs_old = c->ucs_old.as<int>();
    u.skey2 = c->uskey2.as<uint32_t>();
    u.perm2 = c->uperm2.as<int>();
    return u;
}

// The stream-ordered incremental update: move and re-bin (the assignment phase), new
// cell starts (cell scan), new sorted positions (sort), pack (and copy the new order
// back), then the same dense tables and blocks as a build.
nnps_status enqueue_update(nnps_cells* c, hipStream_t s)
{
    const Launch L = launch_of(c);
    PhaseTimer& tm = c->timer;
    const Update u = update_of(c);
    const int64_t zero = 2 * (static_cast<int64_t>(c->ncell_tot) + 1) + (c->ntot + 31) / 32;
    HIP_TRY(launch_fill2_i32(u.leave, zero, c->err.as<int>(), 1, 0, s));
    tm.begin(NNPS_PHASE_ASSIGN, s);
    HIP_TRY(launch_update_move(L, c->skey, c->inv.as<int>(), c->X.as<double>(), u, c->err.as<int>(), s));
    tm.end(NNPS_PHASE_ASSIGN, s);
    tm.begin(NNPS_PHASE_CELLSCAN, s);
    HIP_TRY(launch_update_cells(L, c->cell_start.as<int>(), c->cell_count.as<int>(), u, c->partial.as<int64_t>(), s));
    tm.end(NNPS_PHASE_CELLSCAN, s);
    tm.begin(NNPS_PHASE_SORT, s);
    HIP_TRY(launch_update_place(L, c->skey, c->perm, c->cell_start.as<int>(), u, s));
    tm.end(NNPS_PHASE_SORT, s);
    tm.begin(NNPS_PHASE_PACK, s);
    HIP_TRY(launch_pack(L, u.skey2, u.perm2, c->X.as<double>(), c->q4.as<ushort4>(),
                        spos_of(c),
                        c->mode == NNPS_MODE_FP32_RCLL ? c->rq.as<float4>() : nullptr,
                        c->inv.as<int>(), s, c->skey, c->perm));
    tm.end(NNPS_PHASE_PACK, s);
    return enqueue_build_tail(c, s);
}

// The stream-ordered build: assign, cell starts, sort, pack, blocks.
nnps_status enqueue_build(nnps_cells* c, hipStream_t s)
{
    const Launch L = launch_of(c);
    PhaseTimer& tm = c->timer;
    HIP_TRY(launch_fill2_i32(c->cell_count.as<int>(), static_cast<int64_t>(c->ncell_tot) + 1, c->err.as<int>(), 1, 0, s));
    tm.begin(NNPS_PHASE_ASSIGN, s);
    HIP_TRY(launch_assign(L, c->X.as<double>(), c->k0.as<uint32_t>(), c->v1.as<int>(), c->cell_count.as<int>(),
                          c->err.as<int>(), s));
    tm.end(NNPS_PHASE_ASSIGN, s);
    tm.begin(NNPS_PHASE_CELLSCAN, s);
    HIP_TRY(launch_scan_i32_i32(c->cell_count.as<int>(), c->ncell_tot, c->cell_start.as<int>(),
                                c->partial.as<int64_t>(), s));
    tm.end(NNPS_PHASE_CELLSCAN, s);
    tm.begin(NNPS_PHASE_SORT, s);
    HIP_TRY(launch_place(c->ntot, c->k0.as<uint32_t>(), c->v1.as<int>(), c->cell_start.as<int>(),
                         c->k1.as<uint32_t>(), c->v0.as<int>(), s));
    tm.end(NNPS_PHASE_SORT, s);
    uint32_t* kf = c->k1.as<uint32_t>();
    int* vf = c->v0.as<int>();
    c->skey = kf;
    c->perm = vf;
    tm.begin(NNPS_PHASE_PACK, s);
    HIP_TRY(launch_pack(L, c->skey, c->perm, c->X.as<double>(), c->q4.as<ushort4>(),
                        spos_of(c),
                        c->mode == NNPS_MODE_FP32_RCLL ? c->rq.as<float4>() : nullptr,
                        c->inv.as<int>(), s));
    tm.end(NNPS_PHASE_PACK, s);
    return enqueue_build_tail(c, s);
}

// After the cells and the sorted arrays are in place (build or update): the dense-cell
// tables and the work blocks.
nnps_status enqueue_build_tail(nnps_cells* c, hipStream_t s)
{
    const Launch L = launch_of(c);
    PhaseTimer& tm = c->timer;
    // The dense-cell path runs unless the last synchronising call saw no dense cell; the
    // stencil sizes are computed either way, so a change is seen at the next such call.
    c->dense_active = c->dense && c->dense_seen != 0;
    if (c->dense) {
        tm.begin(NNPS_PHASE_UNIONS, s);
        const DenseBuild d = dense_of(c);
        if (c->dense_active) {
            HIP_TRY(launch_dense_cells(L, c->cell_start.as<int>(), d, s));
            HIP_TRY(launch_dense_unions(L, c->skey, c->inv.as<int>(), d, s, &c->ulist));
        } else {
            HIP_TRY(launch_dense_detect(L, c->cell_start.as<int>(), d, s));
        }
        tm.end(NNPS_PHASE_UNIONS, s);
    }
    tm.begin(NNPS_PHASE_BLOCKS, s);
    HIP_TRY(launch_blocks(L, c->cell_start.as<int>(), c->dense_active ? c->wdense.as<int>() : nullptr,
                          c->boff.as<int>(), c->bstart.as<int>(), c->bset.as<int>(), c->partial.as<int64_t>(), s));
    tm.end(NNPS_PHASE_BLOCKS, s);
    c->built = true;
    c->counted = false;
    return NNPS_OK;
}

// Count pass and row pointers (written into the row_ptr arrays of the set table).
nnps_status enqueue_count(nnps_cells* c, hipStream_t s)
{
    SearchArgs a = args_of(c);
    c->timer.begin(NNPS_PHASE_COUNT, s);
    HIP_TRY(launch_count(a, c->nblk_max, s));
    c->timer.end(NNPS_PHASE_COUNT, s);
    if (c->dense_active) {
        c->timer.begin(NNPS_PHASE_DCOUNT, s);
        HIP_TRY(launch_dense(a, false, s));
        c->timer.end(NNPS_PHASE_DCOUNT, s);
    }
    // the per-block statistics stay in place until the next count; nnps_stats_get sums
    // them when asked, so a step does not pay for the reduction
    c->timer.begin(NNPS_PHASE_ROWSCAN, s);
    HIP_TRY(launch_rowptr(a.L, c->counts.as<int>(), c->rowg.as<int64_t>(), c->partial.as<int64_t>(),
                          c->nnz.as<int64_t>(), c->inv.as<int>(), c->rsort.as<int64_t>(), s));
    c->timer.end(NNPS_PHASE_ROWSCAN, s);
    c->counted = true;
    return NNPS_OK;
}

nnps_status enqueue_fill(nnps_cells* c, hipStream_t s)
{
    SearchArgs a = args_of(c);
    HIP_TRY(launch_fill_i32(c->nheavy.as<int>(), 1, 0, s));
    c->timer.begin(NNPS_PHASE_FILL, s);
    HIP_TRY(launch_fill(a, c->nblk_max, s));
    c->timer.end(NNPS_PHASE_FILL, s);
    c->timer.begin(NNPS_PHASE_LONGROWS, s);
    HIP_TRY(launch_long_rows(a, c->ctx->tuning.long_rows_grid, s));
    c->timer.end(NNPS_PHASE_LONGROWS, s);
    if (c->dense_active) {
        c->timer.begin(NNPS_PHASE_DFILL, s);
        HIP_TRY(launch_dense(a, true, s));
        c->timer.end(NNPS_PHASE_DFILL, s);
    }
    return NNPS_OK;
}

void set_outputs(nnps_cells* c, int64_t* const* row_ptr, int32_t* const* col, float* const* dist,
                 const int64_t* capacity)
{
    for (int s = 0; s < c->nsets; ++s) {
        SetDesc& sd = c->h_sets[s];
        if (row_ptr) sd.row_ptr = row_ptr[s];
        if (col) sd.col = col[s];
        if (dist) sd.dist = dist[s];
        if (capacity) sd.capacity = capacity[s];
    }
}

nnps_status read_nnz(nnps_cells* c, int64_t* h_nnz, hipStream_t s)
{
    int64_t* hp = c->ctx->h_pinned;
    nnps_status st = NNPS_OK;
    // the pinned staging holds 64 values: up to 62 counts per piece, the dense cells'
    // (target, chunk) pairs, the error word and the dense flag
    const bool bits = c->dense_active && dense_bits_on(c);
    for (int s0 = 0; s0 < c->nsets; s0 += 62) {
        const int k = std::min(62, c->nsets - s0);
        HIP_TRY(hipMemcpyAsync(hp, c->nnz.as<int64_t>() + s0, 8 * k, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hp + 63, c->err.p, 4, hipMemcpyDeviceToHost, s));
        if (c->dense) HIP_TRY(hipMemcpyAsync(reinterpret_cast<int*>(hp + 63) + 1, c->dseen.p, 4, hipMemcpyDeviceToHost, s));
        if (bits && s0 == 0)
            HIP_TRY(hipMemcpyAsync(hp + 62, c->dboff.as<int64_t>() + launch_of(c).ncell_tot, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < k; ++i) h_nnz[s0 + i] = hp[i];
        st = err_status(static_cast<int>(hp[63] & 0xFFFFFFFF));
        if (c->dense) c->dense_seen = reinterpret_cast<int*>(hp + 63)[1] != 0 ? 1 : 0;
        if (bits && s0 == 0) {
            // the next build keeps room for the count's bits if they fit the bound
            const size_t want = static_cast<size_t>(hp[62]) * 64 * sizeof(uint16_t);
            if (want <= dense_bits_bound(c)) c->dbits_want = std::max(c->dbits_want, want);
        }
    }
    return st;
}

}  // namespace

extern "C" {

const char* nnps_status_str(nnps_status s)
{
    switch (s) {
    case NNPS_OK: return "NNPS_OK";
    case NNPS_EINVAL: return "NNPS_EINVAL: invalid argument";
    case NNPS_EDOMAIN: return "NNPS_EDOMAIN: a position is not finite or lies outside the box";
    case NNPS_ENOMEM: return "NNPS_ENOMEM: allocation failed";
    case NNPS_ECAPACITY: return "NNPS_ECAPACITY: output capacity below the neighbour count";
    case NNPS_EDEVICE: return "NNPS_EDEVICE: HIP runtime error";
    case NNPS_ETOOMANYCELLS: return "NNPS_ETOOMANYCELLS: too many cells";
    case NNPS_EORDER: return "NNPS_EORDER: call out of order";
    case NNPS_EUNSUPPORTED: return "NNPS_EUNSUPPORTED: internal limit exceeded";
    }
    return "NNPS_UNKNOWN";
}

nnps_status nnps_validate(const nnps_problem* p)
{
    if (!p) return NNPS_EINVAL;
    if (p->dim != 2 && p->dim != 3) return NNPS_EINVAL;
    if (p->mode < NNPS_MODE_FP16_RCLL || p->mode > NNPS_MODE_FP32_RCLL) return NNPS_EINVAL;
    if (p->n < 0 || p->n >= (int64_t(1) << 31)) return NNPS_EINVAL;
    if (!(p->radius > 0.0) || !isfinite(p->radius)) return NNPS_EINVAL;
    if (!(p->cell_size >= p->radius) || !isfinite(p->cell_size)) return NNPS_EINVAL;
    for (int k = 0; k < p->dim; ++k)
        if (!isfinite(p->lo[k]) || !isfinite(p->hi[k]) || !(p->hi[k] > p->lo[k])) return NNPS_EINVAL;
    // cell count guard before any integer conversion
    const double w = std::max(p->cell_size, p->radius);
    double cells = 1.0;
    for (int k = 0; k < p->dim; ++k) cells *= floor((p->hi[k] - p->lo[k]) / w) + 1.0;
    if (cells > ldexp(1.0, 30)) return NNPS_ETOOMANYCELLS;
    return NNPS_OK;
}

nnps_status nnps_grid(const nnps_problem* prob, int32_t ncell[3], int32_t* frac_bits, double* cell_width)
{
    Frame fr;
    nnps_status st = frame_of(prob, &fr, 80);
    if (st != NNPS_OK) return st;
    if (ncell)
        for (int k = 0; k < 3; ++k) ncell[k] = fr.nc[k];
    if (frac_bits) *frac_bits = fr.F;
    if (cell_width) *cell_width = fr.w;
    return NNPS_OK;
}

nnps_status nnps_ctx_create(int device, nnps_ctx** out)
{
    if (!out) return NNPS_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return NNPS_EDEVICE;
    DeviceGuard g(device);
    if (!g.ok) return NNPS_EDEVICE;
    nnps_ctx* c = new (std::nothrow) nnps_ctx;
    if (!c) return NNPS_ENOMEM;
    c->device = device;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_lds = lds;
    // the allocation-free all-list search finds this device's static scratch here, once
    // per device (with the device current); a failed lookup makes that call return
    // NNPS_EDEVICE and leaves every other call unaffected
    (void)allpairs_static_scratch_init(device);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_pinned), 64 * sizeof(int64_t), hipHostMallocDefault) !=
        hipSuccess) {
        delete c;
        return NNPS_ENOMEM;
    }
    if (hipMalloc(reinterpret_cast<void**>(&c->d_flag), 64) != hipSuccess ||
        hipMemset(c->d_flag, 0, 64) != hipSuccess) {
        if (c->d_flag) (void)hipFree(c->d_flag);
        (void)hipHostFree(c->h_pinned);
        delete c;
        return NNPS_ENOMEM;
    }
    *out = c;
    return NNPS_OK;
}

nnps_status nnps_ctx_check(nnps_ctx* ctx, void* stream)
{
    if (!ctx) return NNPS_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int* hp = reinterpret_cast<int*>(ctx->h_pinned);
    hp[0] = 0;
    HIP_TRY(hipMemcpyAsync(hp, ctx->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int e = hp[0];
    if (e == 0) return NNPS_OK;
    HIP_TRY(launch_fill_i32(ctx->d_flag + 1, 1, 0, s));
    return (e & kApErrFill) ? NNPS_EORDER : NNPS_EINVAL;
}

void nnps_ctx_destroy(nnps_ctx* c)
{
    if (!c) return;
    DeviceGuard g(c->device);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    if (c->d_flag) (void)hipFree(c->d_flag);
    if (c->d_apcnt) (void)hipFree(c->d_apcnt);
    delete c;
}

nnps_status nnps_ctx_set_tuning(nnps_ctx* ctx, const nnps_tuning* t)
{
    if (!ctx || !t) return NNPS_EINVAL;
    if (t->block_target < 8 || t->block_target > 4096 || t->long_rows_grid < 1 || t->long_rows_grid > (1 << 20))
        return NNPS_EINVAL;
    const int k = t->long_rows_keys;
    if (k != 0 && (k < 64 || k > 16384 || (k & (k - 1)) != 0)) return NNPS_EINVAL;
    if (t->dense_min_union < -1 || t->dense_min_union > (1 << 30)) return NNPS_EINVAL;
    if (t->dense_grid < 0 || t->dense_grid > (1 << 20)) return NNPS_EINVAL;
    if (t->dense_max_entries < 0 || t->dense_max_entries > INT32_MAX) return NNPS_EINVAL;
    if (t->dense_bits_mib < -1 || t->dense_bits_mib > (1 << 20)) return NNPS_EINVAL;
    ctx->tuning = *t;
    return NNPS_OK;
}

nnps_status nnps_ctx_get_tuning(const nnps_ctx* ctx, nnps_tuning* t)
{
    if (!ctx || !t) return NNPS_EINVAL;
    *t = ctx->tuning;
    return NNPS_OK;
}

nnps_status nnps_cells_create(nnps_ctx* ctx, nnps_cells** out)
{
    if (!ctx || !out) return NNPS_EINVAL;
    nnps_cells* c = new (std::nothrow) nnps_cells;
    if (!c) return NNPS_ENOMEM;
    c->ctx = ctx;
    *out = c;
    return NNPS_OK;
}

void nnps_cells_destroy(nnps_cells* c)
{
    if (!c) return;
    DeviceGuard g(c->ctx->device);
    if (c->upload_pending) (void)hipEventSynchronize(c->upload_done);
    DevBuf* all[] = {&c->d_sets, &c->d_offs, &c->X, &c->k0, &c->k1, &c->v0, &c->v1, &c->cell_count,
                     &c->cell_start, &c->q4, &c->spos, &c->rq, &c->boff, &c->bstart, &c->bset, &c->counts,
                     &c->table, &c->partial, &c->stats, &c->blk_stats, &c->cbits, &c->err, &c->heavy,
                     &c->nheavy, &c->rowg, &c->nnz, &c->sink, &c->usz, &c->wdense, &c->uoff, &c->nsl, &c->unit_off,
                     &c->ucell, &c->dn, &c->ecnt, &c->epos, &c->uk0, &c->uk1, &c->uv0, &c->uv1, &c->inv,
                     &c->ucount, &c->dstats, &c->dseen, &c->uleave, &c->ucs_old,
                     &c->uskey2, &c->uperm2, &c->counts_s, &c->rsort, &c->bdesc};
    for (DevBuf* b : all) b->release();
    c->timer.release();
    c->graph.reset();
    c->ugraph.reset();
    if (c->upload_done) (void)hipEventDestroy(c->upload_done);
    if (c->h_sets) (void)hipHostFree(c->h_sets);
    if (c->h_offs) (void)hipHostFree(c->h_offs);
    if (c->report_done) (void)hipEventDestroy(c->report_done);
    if (c->h_report) (void)hipHostFree(c->h_report);
    delete c;
}

nnps_status nnps_batch_build(nnps_ctx* ctx, nnps_cells* c, int32_t nsets, const nnps_problem* probs,
                             const double* const* d_pos, void* stream)
{
    if (!ctx || !c || c->ctx != ctx) return NNPS_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nnps_status st = prepare(ctx, c, nsets, probs, d_pos);
    if (st != NNPS_OK) return st;
    st = upload(c, true, s);
    if (st != NNPS_OK) return st;
    return enqueue_build(c, s);
}

nnps_status nnps_cells_build(nnps_ctx* ctx, nnps_cells* c, const nnps_problem* prob, const double* d_pos,
                             void* stream)
{
    if (!prob) return NNPS_EINVAL;
    const double* pp[1] = {d_pos};
    return nnps_batch_build(ctx, c, 1, prob, pp, stream);
}

nnps_status nnps_batch_count(nnps_ctx* ctx, nnps_cells* c, int64_t* const* d_row_ptr, int64_t* h_nnz,
                             void* stream)
{
    if (!ctx || !c || c->ctx != ctx || !d_row_ptr) return NNPS_EINVAL;
    for (int s = 0; s < c->nsets; ++s)
        if (!d_row_ptr[s]) return NNPS_EINVAL;
    if (!c->built) return NNPS_EORDER;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nnps_status st = wait_upload(c);
    if (st != NNPS_OK) return st;
    set_outputs(c, d_row_ptr, nullptr, nullptr, nullptr);
    st = upload(c, false, s);
    if (st != NNPS_OK) return st;
    st = enqueue_count(c, s);
    if (st != NNPS_OK) return st;
    return h_nnz ? read_nnz(c, h_nnz, s) : NNPS_OK;
}

nnps_status nnps_count(nnps_ctx* ctx, nnps_cells* c, int64_t* d_row_ptr, int64_t* h_nnz, void* stream)
{
    if (!c || c->nsets != 1) return c ? NNPS_EORDER : NNPS_EINVAL;
    int64_t* rp[1] = {d_row_ptr};
    return nnps_batch_count(ctx, c, rp, h_nnz, stream);
}

nnps_status nnps_allpairs_count(nnps_ctx* ctx, const nnps_problem* prob, const double* d_pos, int64_t* d_row_ptr,
                                int64_t* nnz_out, void* stream)
{
    if (!ctx || !prob || !d_row_ptr || !nnz_out) return NNPS_EINVAL;
    const nnps_status v = nnps_validate(prob);
    if (v != NNPS_OK) return v;
    if (prob->n > kAllPairsMaxN || (prob->n > 0 && !d_pos)) return NNPS_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = static_cast<int>(prob->n);
    ctx->ap.valid = false;
    *nnz_out = 0;
    const double R2 = prob->radius * prob->radius;
    const ApPlan plan = allpairs_plan(n);
    if (n == 0) {
        HIP_TRY(launch_fill_i32(reinterpret_cast<int*>(d_row_ptr), 2, 0, s));  // row_ptr[0] = 0
    } else {
        const size_t need = static_cast<size_t>(plan.nslice) * static_cast<size_t>(n);
        if (need > ctx->apcnt_cap) {
            if (ctx->d_apcnt) {
                HIP_TRY(hipStreamSynchronize(s));  // a queued fill of this context may still read it
                (void)hipFree(ctx->d_apcnt);
                ctx->d_apcnt = nullptr;
                ctx->apcnt_cap = 0;
            }
            if (hipMalloc(reinterpret_cast<void**>(&ctx->d_apcnt), need * sizeof(int)) != hipSuccess) return NNPS_ENOMEM;
            ctx->apcnt_cap = need;
        }
        ApBox box{};
        for (int k = 0; k < prob->dim; ++k) {
            box.lo[k] = prob->lo[k];
            box.hi[k] = prob->hi[k];
        }
        HIP_TRY(launch_fill_i32(ctx->d_flag, 1, 0, s));
        HIP_TRY(launch_allpairs_count(prob->dim, plan, d_pos, R2, box, ctx->d_apcnt, d_row_ptr, ctx->d_flag, s));
        int64_t* hp = ctx->h_pinned;
        hp[0] = 0;
        hp[1] = 0;
        HIP_TRY(hipMemcpyAsync(hp, d_row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hp + 1, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (static_cast<int>(hp[1] & 0xFFFFFFFF) != 0) return NNPS_EDOMAIN;
        *nnz_out = hp[0];
    }
    ctx->ap.valid = true;
    ctx->ap.dim = prob->dim;
    ctx->ap.pos = d_pos;
    ctx->ap.row_ptr = d_row_ptr;
    ctx->ap.R2 = R2;
    ctx->ap.nnz = *nnz_out;
    ctx->ap.plan = plan;
    return NNPS_OK;
}

nnps_status nnps_allpairs_fill(nnps_ctx* ctx, const nnps_problem* prob, const double* d_pos,
                               const int64_t* d_row_ptr, int32_t* d_col, float* d_dist, int64_t capacity,
                               void* stream)
{
    if (!ctx || !prob || !d_row_ptr || capacity < 0) return NNPS_EINVAL;
    if (capacity > 0 && (!d_col || !d_dist)) return NNPS_EINVAL;
    const nnps_status v = nnps_validate(prob);
    if (v != NNPS_OK) return v;
    const auto& ap = ctx->ap;
    if (!ap.valid || ap.plan.n != prob->n || ap.dim != prob->dim || ap.pos != d_pos || ap.row_ptr != d_row_ptr ||
        ap.R2 != prob->radius * prob->radius)
        return NNPS_EORDER;
    if (ap.nnz > capacity) return NNPS_ECAPACITY;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    HIP_TRY(launch_allpairs_fill(ap.dim, ap.plan, d_pos, ap.R2, ctx->d_apcnt, d_row_ptr, d_col, d_dist, capacity,
                                 ctx->d_flag + 1, static_cast<hipStream_t>(stream)));
    return NNPS_OK;
}

nnps_status nnps_allpairs_search(nnps_ctx* ctx, const nnps_problem* prob, const double* d_pos, int64_t* d_row_ptr,
                                 int32_t* d_col, float* d_dist, int64_t capacity, int64_t* nnz_out, void* stream)
{
    if (!ctx || !prob || !d_row_ptr || !nnz_out || capacity < 0) return NNPS_EINVAL;
    if (capacity > 0 && (!d_col || !d_dist)) return NNPS_EINVAL;
    nnps_status st = nnps_allpairs_count(ctx, prob, d_pos, d_row_ptr, nnz_out, stream);
    if (st != NNPS_OK) return st;
    if (*nnz_out > capacity) return NNPS_ECAPACITY;
    return nnps_allpairs_fill(ctx, prob, d_pos, d_row_ptr, d_col, d_dist, capacity, stream);
}

nnps_status nnps_allpairs_search_noalloc(nnps_ctx* ctx, const nnps_problem* prob, const double* d_pos,
                                         int64_t* d_row_ptr, int32_t* d_col, float* d_dist, int64_t capacity,
                                         int64_t* nnz_out, void* stream)
{
    if (!ctx || !prob || !d_row_ptr || !nnz_out || capacity < 0) return NNPS_EINVAL;
    if (capacity > 0 && (!d_col || !d_dist)) return NNPS_EINVAL;
    const nnps_status v = nnps_validate(prob);
    if (v != NNPS_OK) return v;
    if (prob->n > kAllPairsMaxN || (prob->n > 0 && !d_pos)) return NNPS_EINVAL;
    const int n = static_cast<int>(prob->n);
    const ApPlan plan = allpairs_plan(n);
    if (static_cast<int64_t>(plan.nslice) * n > kApStaticCounts) return NNPS_EUNSUPPORTED;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    int* scr = allpairs_static_scratch(ctx->device);
    if (!scr) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    *nnz_out = 0;
    if (n == 0) {
        HIP_TRY(launch_fill_i32(reinterpret_cast<int*>(d_row_ptr), 2, 0, s));  // row_ptr[0] = 0
        return NNPS_OK;
    }
    int* cnt = scr;
    int* flag = scr + kApStaticCounts;
    const double R2 = prob->radius * prob->radius;
    ApBox box{};
    for (int k = 0; k < prob->dim; ++k) {
        box.lo[k] = prob->lo[k];
        box.hi[k] = prob->hi[k];
    }
    HIP_TRY(launch_fill_i32(flag, 1, 0, s));
    HIP_TRY(launch_allpairs_count(prob->dim, plan, d_pos, R2, box, cnt, d_row_ptr, flag, s));
    int64_t* hp = ctx->h_pinned;
    hp[0] = 0;
    hp[1] = 0;
    HIP_TRY(hipMemcpyAsync(hp, d_row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hp + 1, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (static_cast<int>(hp[1] & 0xFFFFFFFF) != 0) return NNPS_EDOMAIN;
    *nnz_out = hp[0];
    if (hp[0] > capacity) return NNPS_ECAPACITY;
    HIP_TRY(launch_allpairs_fill(prob->dim, plan, d_pos, R2, cnt, d_row_ptr, d_col, d_dist, capacity,
                                 ctx->d_flag + 1, s));
    return NNPS_OK;
}

nnps_status nnps_cells_set_half(nnps_cells* c, int on)
{
    if (!c) return NNPS_EINVAL;
    c->half = on != 0;
    c->counted = false;  // row pointers of the other kind must be recounted
    return NNPS_OK;
}

nnps_status nnps_sph_gradient(nnps_ctx* ctx, int32_t dim, int64_t n, double h, const double* d_pos, const double* d_f,
                              const double* d_vol, const int64_t* d_row_ptr, const int32_t* d_col, int64_t ncol,
                              double* d_grad, double* d_grad_norm, void* stream)
{
    if (!ctx || (dim != 2 && dim != 3) || n < 0 || n > INT32_MAX || !(h > 0.0) || !isfinite(h) || ncol < 0)
        return NNPS_EINVAL;
    if (n > 0 && (!d_pos || !d_f || !d_row_ptr)) return NNPS_EINVAL;
    if (ncol > 0 && !d_col) return NNPS_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    HIP_TRY(launch_sph_gradient(dim, n, h, d_pos, d_f, d_vol, d_row_ptr, d_col, ncol, d_grad, d_grad_norm,
                                ctx->d_flag + 1, static_cast<hipStream_t>(stream)));
    return NNPS_OK;
}

nnps_status nnps_batch_fill(nnps_ctx* ctx, nnps_cells* c, int64_t* const* d_row_ptr, int32_t* const* d_col,
                            float* const* d_dist, const int64_t* capacity, void* stream)
{
    if (!ctx || !c || c->ctx != ctx || !d_row_ptr || !d_col || !d_dist || !capacity) return NNPS_EINVAL;
    for (int s = 0; s < c->nsets; ++s) {
        if (!d_row_ptr[s] || capacity[s] < 0) return NNPS_EINVAL;
        if (capacity[s] > 0 && (!d_col[s] || !d_dist[s])) return NNPS_EINVAL;
    }
    if (!c->counted) return NNPS_EORDER;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nnps_status st = wait_upload(c);
    if (st != NNPS_OK) return st;
    set_outputs(c, d_row_ptr, d_col, d_dist, capacity);
    st = upload(c, false, s);
    if (st != NNPS_OK) return st;
    return enqueue_fill(c, s);
}

nnps_status nnps_fill(nnps_ctx* ctx, nnps_cells* c, const int64_t* d_row_ptr, int32_t* d_col, float* d_dist,
                      int64_t capacity, void* stream)
{
    if (!c || c->nsets != 1) return c ? NNPS_EORDER : NNPS_EINVAL;
    if (capacity < 0) return NNPS_EINVAL;
    int64_t* rp[1] = {const_cast<int64_t*>(d_row_ptr)};
    int32_t* cp[1] = {d_col};
    float* dp[1] = {d_dist};
    return nnps_batch_fill(ctx, c, rp, cp, dp, &capacity, stream);
}

nnps_status nnps_batch_search(nnps_ctx* ctx, nnps_cells* c, int32_t nsets, const nnps_problem* probs,
                              const double* const* d_pos, int64_t* const* d_row_ptr, int32_t* const* d_col,
                              float* const* d_dist, const int64_t* capacity, int64_t* nnz_out, void* stream)
{
    if (!nnz_out || !capacity) return NNPS_EINVAL;
    nnps_status st = nnps_batch_build(ctx, c, nsets, probs, d_pos, stream);
    if (st != NNPS_OK) return st;
    st = nnps_batch_count(ctx, c, d_row_ptr, nnz_out, stream);
    if (st != NNPS_OK) return st;
    for (int s = 0; s < nsets; ++s)
        if (nnz_out[s] > capacity[s]) return NNPS_ECAPACITY;
    return nnps_batch_fill(ctx, c, d_row_ptr, d_col, d_dist, capacity, stream);
}

nnps_status nnps_search(nnps_ctx* ctx, nnps_cells* c, const nnps_problem* prob, const double* d_pos,
                        int64_t* d_row_ptr, int32_t* d_col, float* d_dist, int64_t capacity, int64_t* nnz_out,
                        void* stream)
{
    if (!prob || !nnz_out) return NNPS_EINVAL;
    const double* pp[1] = {d_pos};
    int64_t* rp[1] = {d_row_ptr};
    int32_t* cp[1] = {d_col};
    float* dp[1] = {d_dist};
    return nnps_batch_search(ctx, c, 1, prob, pp, rp, cp, dp, &capacity, nnz_out, stream);
}

nnps_status nnps_cells_set_graphs(nnps_cells* c, int on)
{
    if (!c) return NNPS_EINVAL;
    c->use_graphs = on != 0;
    if (!c->use_graphs) c->graph.reset();
    return NNPS_OK;
}

nnps_status nnps_batch_step(nnps_ctx* ctx, nnps_cells* c, int32_t nsets, const nnps_problem* probs,
                            const double* const* d_pos, int64_t* const* d_row_ptr, int32_t* const* d_col,
                            float* const* d_dist, const int64_t* capacity, void* stream)
{
    if (!ctx || !c || c->ctx != ctx || !d_row_ptr || !d_col || !d_dist || !capacity) return NNPS_EINVAL;
    for (int s = 0; s < nsets; ++s) {
        if (!d_row_ptr[s] || capacity[s] < 0) return NNPS_EINVAL;
        if (capacity[s] > 0 && (!d_col[s] || !d_dist[s])) return NNPS_EINVAL;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t gen0 = c->buf_gen;
    nnps_status st = prepare(ctx, c, nsets, probs, d_pos);
    if (st != NNPS_OK) return st;
    set_outputs(c, d_row_ptr, d_col, d_dist, capacity);
    st = upload(c, true, s);
    if (st != NNPS_OK) return st;
    const bool graphs = c->use_graphs && s != nullptr && !c->timer.on;
    if (!graphs) {
        if ((st = enqueue_build(c, s)) != NNPS_OK) return st;
        if ((st = enqueue_count(c, s)) != NNPS_OK) return st;
        return enqueue_fill(c, s);
    }
    // the graph depends on the sizes (grids), the device buffers and the tuning; the
    // per-set pointers travel in the uploaded set table
    std::vector<unsigned char> sig(sizeof(nnps_problem) * nsets + sizeof(uint64_t) + sizeof(nnps_tuning) + 8);
    unsigned char* q = sig.data();
    memcpy(q, probs, sizeof(nnps_problem) * nsets);
    q += sizeof(nnps_problem) * nsets;
    memcpy(q, &c->buf_gen, sizeof(uint64_t));
    q += sizeof(uint64_t);
    memcpy(q, &ctx->tuning, sizeof(nnps_tuning));
    q += sizeof(nnps_tuning);
    memcpy(q, &nsets, 4);
    q += 4;
    const int plan = (c->dense && c->dense_seen != 0 ? 1 : 0) | (c->half ? 2 : 0);
    memcpy(q, &plan, 4);
    (void)gen0;
    if (!c->graph.exec || c->graph.sig != sig) {
        c->graph.reset();
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        nnps_status cst = enqueue_build(c, s);
        if (cst == NNPS_OK) cst = enqueue_count(c, s);
        if (cst == NNPS_OK) cst = enqueue_fill(c, s);
        const hipError_t ee = hipStreamEndCapture(s, &graph);
        if (cst != NNPS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return cst;
        }
        if (ee != hipSuccess) return NNPS_EDEVICE;
        const hipError_t ie = hipGraphInstantiate(&c->graph.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            c->graph.exec = nullptr;
            return NNPS_EDEVICE;
        }
        c->graph.sig = sig;
    }
    HIP_TRY(hipGraphLaunch(c->graph.exec, s));
    c->built = true;
    c->counted = true;
    return NNPS_OK;
}

namespace {

// Point the set table at this update's displacements (or none) and queue its upload.
nnps_status stage_update(nnps_cells* c, const double* const* d_disp, int64_t* const* row_ptr, int32_t* const* col,
                         float* const* dist, const int64_t* capacity, hipStream_t s)
{
    nnps_status st = wait_upload(c);
    if (st != NNPS_OK) return st;
    for (int k = 0; k < c->nsets; ++k) c->h_sets[k].disp = d_disp ? d_disp[k] : nullptr;
    set_outputs(c, row_ptr, col, dist, capacity);
    return upload(c, false, s);
}

}  // namespace

nnps_status nnps_cells_update(nnps_ctx* ctx, nnps_cells* c, const double* const* d_disp, void* stream)
{
    if (!ctx || !c || c->ctx != ctx) return NNPS_EINVAL;
    if (!c->built) return NNPS_EORDER;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nnps_status st = stage_update(c, d_disp, nullptr, nullptr, nullptr, nullptr, s);
    if (st != NNPS_OK) return st;
    return enqueue_update(c, s);
}

nnps_status nnps_batch_update_step(nnps_ctx* ctx, nnps_cells* c, const double* const* d_disp,
                                   int64_t* const* d_row_ptr, int32_t* const* d_col, float* const* d_dist,
                                   const int64_t* capacity, void* stream)
{
    if (!ctx || !c || c->ctx != ctx || !d_row_ptr || !d_col || !d_dist || !capacity) return NNPS_EINVAL;
    if (!c->built) return NNPS_EORDER;
    for (int k = 0; k < c->nsets; ++k) {
        if (!d_row_ptr[k] || capacity[k] < 0) return NNPS_EINVAL;
        if (capacity[k] > 0 && (!d_col[k] || !d_dist[k])) return NNPS_EINVAL;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nnps_status st = stage_update(c, d_disp, d_row_ptr, d_col, d_dist, capacity, s);
    if (st != NNPS_OK) return st;
    const bool graphs = c->use_graphs && s != nullptr && !c->timer.on;
    if (!graphs) {
        if ((st = enqueue_update(c, s)) != NNPS_OK) return st;
        if ((st = enqueue_count(c, s)) != NNPS_OK) return st;
        return enqueue_fill(c, s);
    }
    // the graph depends on the grids, the device buffers, the tuning and the dense plan;
    // positions, displacements and outputs travel in the uploaded set table
    std::vector<unsigned char> sig(sizeof(Frame) * c->nsets + sizeof(uint64_t) + sizeof(nnps_tuning) + 8);
    unsigned char* q = sig.data();
    memcpy(q, c->frames.data(), sizeof(Frame) * c->nsets);
    q += sizeof(Frame) * c->nsets;
    memcpy(q, &c->buf_gen, sizeof(uint64_t));
    q += sizeof(uint64_t);
    memcpy(q, &ctx->tuning, sizeof(nnps_tuning));
    q += sizeof(nnps_tuning);
    memcpy(q, &c->nsets, 4);
    q += 4;
    const int plan = (c->dense && c->dense_seen != 0 ? 1 : 0) | (c->half ? 2 : 0);
    memcpy(q, &plan, 4);
    if (!c->ugraph.exec || c->ugraph.sig != sig) {
        c->ugraph.reset();
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        nnps_status cst = enqueue_update(c, s);
        if (cst == NNPS_OK) cst = enqueue_count(c, s);
        if (cst == NNPS_OK) cst = enqueue_fill(c, s);
        const hipError_t ee = hipStreamEndCapture(s, &graph);
        if (cst != NNPS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return cst;
        }
        if (ee != hipSuccess) return NNPS_EDEVICE;
        const hipError_t ie = hipGraphInstantiate(&c->ugraph.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            c->ugraph.exec = nullptr;
            return NNPS_EDEVICE;
        }
        c->ugraph.sig = sig;
    }
    HIP_TRY(hipGraphLaunch(c->ugraph.exec, s));
    c->built = true;
    c->counted = true;
    return NNPS_OK;
}

nnps_status nnps_batch_nnz(nnps_cells* c, int64_t* h_nnz, void* stream)
{
    if (!c || !h_nnz) return NNPS_EINVAL;
    if (!c->counted) return NNPS_EORDER;
    DeviceGuard g(c->ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    return read_nnz(c, h_nnz, static_cast<hipStream_t>(stream));
}

nnps_status nnps_batch_nnz_enqueue(nnps_cells* c, void* stream)
{
    if (!c) return NNPS_EINVAL;
    if (!c->counted) return NNPS_EORDER;
    DeviceGuard g(c->ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (c->report_pending) HIP_TRY(hipEventSynchronize(c->report_done));  // the buffer is reused
    c->report_pending = false;
    if (c->h_report_cap < c->nsets + 2) {
        if (c->h_report) (void)hipHostFree(c->h_report);
        c->h_report = nullptr;
        c->h_report_cap = 0;
        if (hipHostMalloc(reinterpret_cast<void**>(&c->h_report), sizeof(int64_t) * (c->nsets + 2),
                          hipHostMallocDefault) != hipSuccess)
            return NNPS_ENOMEM;
        c->h_report_cap = c->nsets + 2;
    }
    if (!c->report_done && hipEventCreateWithFlags(&c->report_done, hipEventDisableTiming) != hipSuccess)
        return NNPS_EDEVICE;
    int64_t* hp = c->h_report;
    hp[c->nsets] = 0;
    hp[c->nsets + 1] = 0;
    HIP_TRY(hipMemcpyAsync(hp, c->nnz.p, 8 * c->nsets, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hp + c->nsets, c->err.p, 4, hipMemcpyDeviceToHost, s));
    if (c->dense) HIP_TRY(hipMemcpyAsync(hp + c->nsets + 1, c->dseen.p, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(c->report_done, s));
    c->report_pending = true;
    return NNPS_OK;
}

nnps_status nnps_batch_nnz_fetch(nnps_cells* c, int64_t* h_nnz)
{
    if (!c || !h_nnz) return NNPS_EINVAL;
    if (!c->report_pending) return NNPS_EORDER;
    DeviceGuard g(c->ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    HIP_TRY(hipEventSynchronize(c->report_done));
    const int64_t* hp = c->h_report;
    for (int i = 0; i < c->nsets; ++i) h_nnz[i] = hp[i];
    if (c->dense) c->dense_seen = static_cast<int>(hp[c->nsets + 1] & 0xFFFFFFFF) != 0 ? 1 : 0;
    return err_status(static_cast<int>(hp[c->nsets] & 0xFFFFFFFF));
}

nnps_status nnps_stats_get(nnps_cells* c, nnps_stats* out, void* stream)
{
    if (!c || !out) return NNPS_EINVAL;
    memset(out, 0, sizeof(*out));
    if (!c->built) return NNPS_EORDER;
    DeviceGuard g(c->ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long st[kStCount];
    int err = 0, nh = 0;
    // the sums of the last count pass's per-block (and dense-path) statistics; none
    // before a count
    HIP_TRY(launch_fill_i32(c->stats.as<int>(), 2 * kStCount, 0, s));
    if (c->counted) HIP_TRY(launch_stats(args_of(c), s));
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(st, c->stats.p, sizeof(st), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&err, c->err.p, 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&nh, c->nheavy.p, 4, hipMemcpyDeviceToHost));
    out->n = c->ntot;
    if (c->counted) {
        std::vector<int64_t> nz(c->nsets);
        HIP_TRY(hipMemcpy(nz.data(), c->nnz.p, 8 * c->nsets, hipMemcpyDeviceToHost));
        for (int64_t v : nz) out->nnz += v;
    }
    out->candidates = static_cast<int64_t>(st[kStCandidates]);
    out->band_pairs = static_cast<int64_t>(st[kStBand]);
    out->fp16_false_pos = static_cast<int64_t>(st[kStFalsePos]);
    out->fp16_false_neg = static_cast<int64_t>(st[kStFalseNeg]);
    out->outside_band_disagree = static_cast<int64_t>(st[kStOutsideDisagree]);
    out->heavy_rows = nh;
    out->dense_rows = static_cast<int64_t>(st[kStDenseRows]);
    if (c->dense) {
        int dn = 0, seen = 0;
        HIP_TRY(hipMemcpy(&seen, c->dseen.p, 4, hipMemcpyDeviceToHost));
        c->dense_seen = seen != 0 ? 1 : 0;
        if (c->dense_active) HIP_TRY(hipMemcpy(&dn, c->dn.p, 4, hipMemcpyDeviceToHost));
        out->dense_entries = dn;
    }
    out->dim = c->dim;
    out->mode = c->mode;
    if (!c->frames.empty()) {
        out->frac_bits = c->frames[0].F;
        for (int k = 0; k < 3; ++k) out->ncell[k] = c->frames[0].nc[k];
        out->cell_width = c->frames[0].w;
    }
    out->band = ldexp(1.0, -7);
    return err_status(err);
}

nnps_status nnps_cells_set_profiling(nnps_cells* c, int on)
{
    if (!c) return NNPS_EINVAL;
    DeviceGuard g(c->ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    c->timer.reset();
    c->timer.on = on != 0;
    return NNPS_OK;
}

nnps_status nnps_phase_times(nnps_cells* c, double* ms, int32_t* runs, void* stream)
{
    if (!c || !ms || !runs) return NNPS_EINVAL;
    for (int k = 0; k < NNPS_NPHASES; ++k) {
        ms[k] = 0.0;
        runs[k] = 0;
    }
    if (!c->timer.on) return NNPS_EORDER;
    DeviceGuard g(c->ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    for (int k = 0; k < NNPS_NPHASES; ++k) {
        for (const auto& pr : c->timer.rec[k]) {
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, c->timer.pool[pr.first], c->timer.pool[pr.second]));
            ms[k] += t;
            runs[k] += 1;
        }
    }
    c->timer.reset();
    return NNPS_OK;
}

}  // extern "C"
