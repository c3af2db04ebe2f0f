// C-ABI entry points (include/nnps.h): argument checks, grid set-up, device buffers
// and the stream-ordered sequence of cell-build and search kernels.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "../../include/nnps.h"
#include "build_kernels.h"

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

nnps_status frame_of(const nnps_problem* p, Frame* fr)
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
    // x-window of a work block: about 56 particles on average, so most windows fill one
    // wavefront and the candidate union stays small
    const double occ = static_cast<double>(p->n) / static_cast<double>(ncell);
    int xwin = occ > 0.0 ? static_cast<int>(56.0 / occ) : kMaxXWin;
    fr->xwin = std::max(1, std::min(kMaxXWin, xwin));
    return NNPS_OK;
}

}  // namespace

struct nnps_ctx {
    int device = 0;
    int64_t* h_pinned = nullptr;  // small pinned staging for synchronous readbacks
};

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

struct nnps_cells {
    nnps_ctx* ctx = nullptr;
    PhaseTimer timer;
    Frame fr{};
    bool built = false, counted = false;
    const double* pos = nullptr;
    int nblk_max = 0;
    uint32_t* skey = nullptr;
    int* perm = nullptr;
    DevBuf X, k0, k1, v0, v1, cell_count, cell_start, q4, spos, flags, bidx, bstart, counts, table,
        partial, stats, blk_stats, cbits, err, heavy, nheavy, nnz;
};

#define HIP_TRY(x)                                \
    do {                                          \
        if ((x) != hipSuccess) return NNPS_EDEVICE; \
    } while (0)

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
    case NNPS_ETOOMANYCELLS: return "NNPS_ETOOMANYCELLS: more than 2^30 cells";
    case NNPS_EORDER: return "NNPS_EORDER: call out of order";
    case NNPS_EUNSUPPORTED: return "NNPS_EUNSUPPORTED: a neighbour row is longer than supported";
    }
    return "NNPS_UNKNOWN";
}

nnps_status nnps_validate(const nnps_problem* p)
{
    if (!p) return NNPS_EINVAL;
    if (p->dim != 2 && p->dim != 3) return NNPS_EINVAL;
    if (p->mode < NNPS_MODE_FP16_RCLL || p->mode > NNPS_MODE_RECHECK_ALL) return NNPS_EINVAL;
    if (p->n < 0 || p->n >= (int64_t(1) << 31)) return NNPS_EINVAL;
    if (!(p->radius > 0.0) || !isfinite(p->radius)) return NNPS_EINVAL;
    if (!(p->cell_size >= p->radius) || !isfinite(p->cell_size)) return NNPS_EINVAL;
    double wmax = 0.0;
    for (int k = 0; k < p->dim; ++k) {
        if (!isfinite(p->lo[k]) || !isfinite(p->hi[k]) || !(p->hi[k] > p->lo[k])) return NNPS_EINVAL;
        wmax = std::max(wmax, p->hi[k] - p->lo[k]);
    }
    // cell count guard before any integer conversion
    const double w = std::max(p->cell_size, p->radius);
    double cells = 1.0;
    for (int k = 0; k < p->dim; ++k) cells *= floor((p->hi[k] - p->lo[k]) / w) + 1.0;
    if (cells > ldexp(1.0, 30)) return NNPS_ETOOMANYCELLS;
    (void)wmax;
    return NNPS_OK;
}

nnps_status nnps_grid(const nnps_problem* prob, int32_t ncell[3], int32_t* frac_bits, double* cell_width)
{
    Frame fr;
    nnps_status st = frame_of(prob, &fr);
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
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_pinned), 8 * sizeof(int64_t), hipHostMallocDefault) !=
        hipSuccess) {
        delete c;
        return NNPS_ENOMEM;
    }
    *out = c;
    return NNPS_OK;
}

void nnps_ctx_destroy(nnps_ctx* c)
{
    if (!c) return;
    DeviceGuard g(c->device);
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    delete c;
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
    DevBuf* all[] = {&c->X, &c->k0, &c->k1, &c->v0, &c->v1, &c->cell_count, &c->cell_start, &c->q4,
                     &c->spos, &c->flags, &c->bidx, &c->bstart, &c->counts, &c->table, &c->partial,
                     &c->stats, &c->blk_stats, &c->cbits, &c->err, &c->heavy, &c->nheavy, &c->nnz};
    for (DevBuf* b : all) b->release();
    c->timer.release();
    delete c;
}

nnps_status nnps_cells_build(nnps_ctx* ctx, nnps_cells* c, const nnps_problem* prob, const double* d_pos,
                             void* stream)
{
    if (!ctx || !c || !prob || c->ctx != ctx) return NNPS_EINVAL;
    Frame fr;
    nnps_status st = frame_of(prob, &fr);
    if (st != NNPS_OK) return st;
    if (fr.n > 0 && !d_pos) return NNPS_EINVAL;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = static_cast<size_t>(fr.n);
    const size_t nn = std::max<size_t>(n, 1);
    const size_t ncell = static_cast<size_t>(fr.ncell);
    const int64_t nrows = static_cast<int64_t>(fr.nc[1]) * fr.nc[2];
    const int64_t nwin = nrows * ((fr.nc[0] + fr.xwin - 1) / fr.xwin);
    const int64_t nblk_bound = static_cast<int64_t>(n / kWave) + nwin + 1;
    c->nblk_max = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(n), nblk_bound));
    const size_t table_n = radix_table_entries(static_cast<int>(nn)) + 1;
    const int64_t scan_m = std::max<int64_t>({static_cast<int64_t>(nn) + 1, static_cast<int64_t>(ncell) + 1,
                                              static_cast<int64_t>(table_n)});

    const bool base = fr.mode == NNPS_MODE_FP64_BASELINE;
    hipError_t e = hipSuccess;
    if ((e = c->X.ensure(nn * x_stride(fr.dim) * sizeof(int64_t))) != hipSuccess ||
        (e = c->k0.ensure(nn * 4)) != hipSuccess || (e = c->k1.ensure(nn * 4)) != hipSuccess ||
        (e = c->v0.ensure(nn * 4)) != hipSuccess || (e = c->v1.ensure(nn * 4)) != hipSuccess ||
        (e = c->cell_count.ensure((ncell + 1) * 4)) != hipSuccess ||
        (e = c->cell_start.ensure((ncell + 1) * 4)) != hipSuccess ||
        (e = c->q4.ensure(nn * sizeof(ushort4))) != hipSuccess ||
        (base && (e = c->spos.ensure(nn * 4 * sizeof(double))) != hipSuccess) ||
        (e = c->flags.ensure(nn * 4)) != hipSuccess || (e = c->bidx.ensure((nn + 1) * 4)) != hipSuccess ||
        (e = c->bstart.ensure((nn + 2) * 4)) != hipSuccess || (e = c->counts.ensure(nn * 4)) != hipSuccess ||
        (e = c->table.ensure(table_n * 4)) != hipSuccess ||
        (e = c->partial.ensure(static_cast<size_t>(scan_partials_needed(scan_m) + 1) * 8)) != hipSuccess ||
        (e = c->stats.ensure(kStCount * 8)) != hipSuccess || (e = c->err.ensure(4)) != hipSuccess ||
        (e = c->heavy.ensure(nn * 4)) != hipSuccess || (e = c->nheavy.ensure(4)) != hipSuccess ||
        (e = c->nnz.ensure(8)) != hipSuccess ||
        (e = c->blk_stats.ensure(static_cast<size_t>(std::max(c->nblk_max, 1)) * 5 * 8)) != hipSuccess ||
        (e = c->cbits.ensure(nn * (fr.dim == 3 ? kCandWords3 : kCandWords2) * 4)) != hipSuccess)
        return e == hipErrorOutOfMemory ? NNPS_ENOMEM : NNPS_EDEVICE;

    c->fr = fr;
    c->pos = d_pos;
    c->built = false;
    c->counted = false;
    HIP_TRY(hipMemsetAsync(c->cell_count.p, 0, (ncell + 1) * 4, s));
    HIP_TRY(hipMemsetAsync(c->err.p, 0, 4, s));
    HIP_TRY(hipMemsetAsync(c->stats.p, 0, kStCount * 8, s));
    PhaseTimer& tm = c->timer;
    tm.begin(NNPS_PHASE_ASSIGN, s);
    HIP_TRY(launch_assign(d_pos, fr, c->X.as<int64_t>(), c->k0.as<uint32_t>(), c->cell_count.as<int>(),
                          c->err.as<int>(), s));
    tm.end(NNPS_PHASE_ASSIGN, s);
    tm.begin(NNPS_PHASE_CELLSCAN, s);
    HIP_TRY(launch_scan_i32_i32(c->cell_count.as<int>(), static_cast<int64_t>(ncell), c->cell_start.as<int>(),
                                c->partial.as<int64_t>(), s));
    tm.end(NNPS_PHASE_CELLSCAN, s);
    uint32_t* kf = c->k0.as<uint32_t>();
    int* vf = c->v0.as<int>();
    tm.begin(NNPS_PHASE_SORT, s);
    if (fr.n > 0) {
        const int keybits = bitlen(static_cast<int64_t>(ncell) - 1);
        HIP_TRY(launch_radix_sort(fr.n, keybits, c->k0.as<uint32_t>(), c->v0.as<int>(), c->k1.as<uint32_t>(),
                                  c->v1.as<int>(), c->table.as<uint32_t>(), c->partial.as<int64_t>(), s, &kf,
                                  &vf));
    }
    tm.end(NNPS_PHASE_SORT, s);
    c->skey = kf;
    c->perm = vf;
    tm.begin(NNPS_PHASE_PACK, s);
    HIP_TRY(launch_pack(fr, c->perm, c->X.as<int64_t>(), c->q4.as<ushort4>(), d_pos,
                        base ? c->spos.as<double>() : nullptr, s));
    tm.end(NNPS_PHASE_PACK, s);
    tm.begin(NNPS_PHASE_BLOCKS, s);
    HIP_TRY(launch_blocks(fr, c->skey, c->cell_start.as<int>(), c->flags.as<int>(), c->bidx.as<int>(),
                          c->bstart.as<int>(), c->partial.as<int64_t>(), s));
    tm.end(NNPS_PHASE_BLOCKS, s);
    c->built = true;
    return NNPS_OK;
}

static SearchArgs args_of(nnps_cells* c)
{
    SearchArgs a{};
    a.fr = c->fr;
    a.pos = c->pos;
    a.skey = c->skey;
    a.perm = c->perm;
    a.cell_start = c->cell_start.as<int>();
    a.q4 = c->q4.as<ushort4>();
    a.spos = c->fr.mode == NNPS_MODE_FP64_BASELINE ? c->spos.as<double>() : nullptr;
    a.X = c->X.as<int64_t>();
    a.bstart = c->bstart.as<int>();
    a.nblk = c->bidx.as<int>() + c->fr.n;
    a.counts = c->counts.as<int>();
    a.heavy = c->heavy.as<int>();
    a.nheavy = c->nheavy.as<int>();
    a.stats = c->stats.as<unsigned long long>();
    a.blk_stats = c->blk_stats.as<unsigned long long>();
    a.cbits = c->cbits.as<uint32_t>();
    a.err = c->err.as<int>();
    return a;
}

static nnps_status err_status(int err)
{
    if (err & kErrDomain) return NNPS_EDOMAIN;
    if (err & kErrCapacity) return NNPS_ECAPACITY;
    if (err & kErrLongRow) return NNPS_EUNSUPPORTED;
    return NNPS_OK;
}

nnps_status nnps_count(nnps_ctx* ctx, nnps_cells* c, int64_t* d_row_ptr, int64_t* h_nnz, void* stream)
{
    if (!ctx || !c || c->ctx != ctx || !d_row_ptr) return NNPS_EINVAL;
    if (!c->built) return NNPS_EORDER;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SearchArgs a = args_of(c);
    HIP_TRY(hipMemsetAsync(c->stats.p, 0, kStCount * 8, s));
    c->timer.begin(NNPS_PHASE_COUNT, s);
    HIP_TRY(launch_count(a, c->nblk_max, s));
    c->timer.end(NNPS_PHASE_COUNT, s);
    c->timer.begin(NNPS_PHASE_ROWSCAN, s);
    HIP_TRY(launch_scan_i32_i64(c->counts.as<int>(), c->fr.n, d_row_ptr, c->partial.as<int64_t>(), s));
    c->timer.end(NNPS_PHASE_ROWSCAN, s);
    HIP_TRY(hipMemcpyAsync(c->nnz.p, d_row_ptr + c->fr.n, 8, hipMemcpyDeviceToDevice, s));
    c->counted = true;
    if (h_nnz) {
        int64_t* hp = ctx->h_pinned;
        HIP_TRY(hipMemcpyAsync(hp, d_row_ptr + c->fr.n, 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hp + 1, c->err.p, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        *h_nnz = hp[0];
        const int err = static_cast<int>(hp[1] & 0xFFFFFFFF);
        return err_status(err);
    }
    return NNPS_OK;
}

nnps_status nnps_fill(nnps_ctx* ctx, nnps_cells* c, const int64_t* d_row_ptr, int32_t* d_col, float* d_dist,
                      int64_t capacity, void* stream)
{
    if (!ctx || !c || c->ctx != ctx || !d_row_ptr || capacity < 0) return NNPS_EINVAL;
    if (capacity > 0 && (!d_col || !d_dist)) return NNPS_EINVAL;
    if (!c->counted) return NNPS_EORDER;
    DeviceGuard g(ctx->device);
    if (!g.ok) return NNPS_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    SearchArgs a = args_of(c);
    a.row_ptr = d_row_ptr;
    a.col = d_col;
    a.dist = d_dist;
    a.capacity = capacity;
    HIP_TRY(hipMemsetAsync(c->nheavy.p, 0, 4, s));
    c->timer.begin(NNPS_PHASE_FILL, s);
    HIP_TRY(launch_fill(a, c->nblk_max, s));
    c->timer.end(NNPS_PHASE_FILL, s);
    c->timer.begin(NNPS_PHASE_LONGROWS, s);
    HIP_TRY(launch_long_rows(a, s));
    c->timer.end(NNPS_PHASE_LONGROWS, s);
    return NNPS_OK;
}

nnps_status nnps_search(nnps_ctx* ctx, nnps_cells* c, const nnps_problem* prob, const double* d_pos,
                        int64_t* d_row_ptr, int32_t* d_col, float* d_dist, int64_t capacity, int64_t* nnz_out,
                        void* stream)
{
    nnps_status st = nnps_cells_build(ctx, c, prob, d_pos, stream);
    if (st != NNPS_OK) return st;
    int64_t nnz = 0;
    st = nnps_count(ctx, c, d_row_ptr, &nnz, stream);
    if (nnz_out) *nnz_out = nnz;
    if (st != NNPS_OK) return st;
    if (nnz > capacity) return NNPS_ECAPACITY;
    return nnps_fill(ctx, c, d_row_ptr, d_col, d_dist, capacity, stream);
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
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipMemcpy(st, c->stats.p, sizeof(st), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&err, c->err.p, 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&nh, c->nheavy.p, 4, hipMemcpyDeviceToHost));
    out->n = c->fr.n;
    if (c->counted) HIP_TRY(hipMemcpy(&out->nnz, c->nnz.p, 8, hipMemcpyDeviceToHost));
    out->candidates = static_cast<int64_t>(st[kStCandidates]);
    out->band_pairs = static_cast<int64_t>(st[kStBand]);
    out->fp16_false_pos = static_cast<int64_t>(st[kStFalsePos]);
    out->fp16_false_neg = static_cast<int64_t>(st[kStFalseNeg]);
    out->outside_band_disagree = static_cast<int64_t>(st[kStOutsideDisagree]);
    out->heavy_rows = nh;
    out->dim = c->fr.dim;
    out->mode = c->fr.mode;
    out->frac_bits = c->fr.F;
    for (int k = 0; k < 3; ++k) out->ncell[k] = c->fr.nc[k];
    out->cell_width = c->fr.w;
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
