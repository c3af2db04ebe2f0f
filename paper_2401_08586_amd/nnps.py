"""Python binding for libnnps.so (include/nnps.h): argument marshalling only.

Every step of the search runs in the HIP library. PyTorch supplies device memory and
streams: positions and outputs are torch CUDA tensors passed as raw pointers, and the
stream is torch's current stream unless one is given. If the library is missing this
module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnps.so")

NNPS_OK = 0
NNPS_EINVAL = -1
NNPS_EDOMAIN = -2
NNPS_ENOMEM = -3
NNPS_ECAPACITY = -4
NNPS_EDEVICE = -5
NNPS_ETOOMANYCELLS = -6
NNPS_EORDER = -7
NNPS_EUNSUPPORTED = -8

MODE_FP16_RCLL = 0
MODE_FP64_BASELINE = 1
MODE_RECHECK_ALL = 2
MODE_FP32_RCLL = 3


class NnpsError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {status_str(code)}" if what else status_str(code))


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("mode", ctypes.c_int32), ("n", ctypes.c_int64),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("cell_size", ctypes.c_double), ("radius", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("band_pairs", ctypes.c_int64), ("fp16_false_pos", ctypes.c_int64),
                ("fp16_false_neg", ctypes.c_int64), ("outside_band_disagree", ctypes.c_int64),
                ("heavy_rows", ctypes.c_int64), ("dense_rows", ctypes.c_int64),
                ("dense_entries", ctypes.c_int64), ("dim", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("frac_bits", ctypes.c_int32), ("ncell", ctypes.c_int32 * 3),
                ("cell_width", ctypes.c_double), ("band", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["ncell"] = list(self.ncell)
        return d


class Tuning(ctypes.Structure):
    _fields_ = [("block_target", ctypes.c_int32), ("long_rows_grid", ctypes.c_int32),
                ("long_rows_keys", ctypes.c_int32), ("dense_min_union", ctypes.c_int32),
                ("dense_grid", ctypes.c_int32), ("dense_bits_mib", ctypes.c_int32),
                ("dense_max_entries", ctypes.c_int64)]

    NAMES = ("block_target", "long_rows_grid", "long_rows_keys", "dense_min_union", "dense_grid",
             "dense_bits_mib", "dense_max_entries")


EXPORTS = ["nnps_status_str", "nnps_validate", "nnps_grid", "nnps_ctx_create", "nnps_ctx_destroy",
           "nnps_ctx_set_tuning", "nnps_ctx_get_tuning",
           "nnps_cells_create", "nnps_cells_destroy", "nnps_cells_build", "nnps_count", "nnps_fill",
           "nnps_search", "nnps_stats_get", "nnps_cells_set_profiling", "nnps_phase_times",
           "nnps_batch_build", "nnps_batch_count", "nnps_batch_fill", "nnps_batch_search",
           "nnps_batch_step", "nnps_cells_set_graphs", "nnps_batch_nnz", "nnps_batch_nnz_enqueue",
           "nnps_batch_nnz_fetch", "nnps_sph_gradient", "nnps_cells_set_half", "nnps_allpairs_search",
           "nnps_allpairs_count", "nnps_allpairs_fill", "nnps_ctx_check",
           "nnps_allpairs_search_noalloc", "nnps_cells_update", "nnps_batch_update_step",
           "nnps_probe_valu_rate"]

PHASES = ["assign", "cellscan", "sort", "pack", "blocks", "unions", "count", "dcount", "rowscan", "fill",
          "longrows", "dfill"]

_lib = None


def load():
    """Load libnnps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2401_08586_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    PP = ctypes.POINTER(ctypes.c_void_p)
    I64 = ctypes.c_int64
    lib.nnps_status_str.argtypes = [ctypes.c_int]
    lib.nnps_status_str.restype = ctypes.c_char_p
    lib.nnps_validate.argtypes = [ctypes.POINTER(Problem)]
    lib.nnps_grid.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.nnps_ctx_create.argtypes = [ctypes.c_int, PP]
    lib.nnps_ctx_destroy.argtypes = [P]
    lib.nnps_ctx_destroy.restype = None
    lib.nnps_cells_create.argtypes = [P, PP]
    lib.nnps_cells_destroy.argtypes = [P]
    lib.nnps_cells_destroy.restype = None
    lib.nnps_cells_build.argtypes = [P, P, ctypes.POINTER(Problem), P, P]
    lib.nnps_count.argtypes = [P, P, P, ctypes.POINTER(I64), P]
    lib.nnps_fill.argtypes = [P, P, P, P, P, I64, P]
    lib.nnps_search.argtypes = [P, P, ctypes.POINTER(Problem), P, P, P, P, I64, ctypes.POINTER(I64), P]
    lib.nnps_stats_get.argtypes = [P, ctypes.POINTER(Stats), P]
    lib.nnps_cells_set_profiling.argtypes = [P, ctypes.c_int]
    lib.nnps_ctx_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.nnps_ctx_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
    lib.nnps_batch_build.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(Problem), P, P]
    lib.nnps_batch_count.argtypes = [P, P, P, P, P]
    lib.nnps_batch_fill.argtypes = [P, P, P, P, P, P, P]
    lib.nnps_batch_search.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(Problem), P, P, P, P, P, P, P]
    lib.nnps_batch_step.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(Problem), P, P, P, P, P, P]
    lib.nnps_cells_set_graphs.argtypes = [P, ctypes.c_int]
    lib.nnps_cells_set_half.argtypes = [P, ctypes.c_int]
    lib.nnps_allpairs_search.argtypes = [P, ctypes.POINTER(Problem), P, P, P, P, I64, ctypes.POINTER(I64), P]
    lib.nnps_allpairs_count.argtypes = [P, ctypes.POINTER(Problem), P, P, ctypes.POINTER(I64), P]
    lib.nnps_allpairs_fill.argtypes = [P, ctypes.POINTER(Problem), P, P, P, P, I64, P]
    lib.nnps_batch_nnz.argtypes = [P, P, P]
    lib.nnps_phase_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), P]
    lib.nnps_sph_gradient.argtypes = [P, ctypes.c_int32, I64, ctypes.c_double, P, P, P, P, P, I64, P, P, P]
    lib.nnps_ctx_check.argtypes = [P, P]
    lib.nnps_allpairs_search_noalloc.argtypes = [P, ctypes.POINTER(Problem), P, P, P, P, I64,
                                                 ctypes.POINTER(I64), P]
    lib.nnps_cells_update.argtypes = [P, P, P, P]
    lib.nnps_batch_update_step.argtypes = [P, P, P, P, P, P, P, P]
    lib.nnps_probe_valu_rate.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(I64)]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("nnps_status_str", "nnps_ctx_destroy", "nnps_cells_destroy"):
            fn.restype = ctypes.c_int
    _lib = lib
    return lib


def status_str(code: int) -> str:
    try:
        return load().nnps_status_str(code).decode()
    except ImportError:
        return f"status {code}"


def _check(code: int, what: str):
    if code != NNPS_OK:
        raise NnpsError(code, what)


def make_problem(dim, n, lo, hi, cell_size, radius, mode=MODE_FP16_RCLL) -> Problem:
    p = Problem()
    p.dim = int(dim)
    p.mode = int(mode)
    p.n = int(n)
    for k in range(3):
        p.lo[k] = float(lo[k]) if k < dim else 0.0
        p.hi[k] = float(hi[k]) if k < dim else 0.0
    p.cell_size = float(cell_size)
    p.radius = float(radius)
    return p


def validate(prob: Problem) -> int:
    return load().nnps_validate(ctypes.byref(prob))


def grid(prob: Problem):
    nc = (ctypes.c_int32 * 3)()
    fb = ctypes.c_int32()
    w = ctypes.c_double()
    _check(load().nnps_grid(ctypes.byref(prob), nc, ctypes.byref(fb), ctypes.byref(w)), "nnps_grid")
    return list(nc), fb.value, w.value


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


class Context:
    """A library context on one device, plus a reusable cell structure."""

    def __init__(self, device: int = 0):
        lib = load()
        self._lib = lib
        self.device = device
        h = ctypes.c_void_p()
        _check(lib.nnps_ctx_create(device, ctypes.byref(h)), "nnps_ctx_create")
        self._ctx = h
        self._cells = []

    def close(self):
        for c in self._cells:
            c.close()
        self._cells = []
        if self._ctx:
            self._lib.nnps_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, block_target: int = 80, long_rows_grid: int = 1024, long_rows_keys: int = 0,
                   dense_min_union: int = 0, dense_grid: int = 0, dense_max_entries: int = 0,
                   dense_bits_mib: int = 0):
        t = Tuning(int(block_target), int(long_rows_grid), int(long_rows_keys), int(dense_min_union),
                   int(dense_grid), int(dense_bits_mib), int(dense_max_entries))
        _check(self._lib.nnps_ctx_set_tuning(self._ctx, ctypes.byref(t)), "nnps_ctx_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(self._lib.nnps_ctx_get_tuning(self._ctx, ctypes.byref(t)), "nnps_ctx_get_tuning")
        return {k: getattr(t, k) for k in Tuning.NAMES}

    def cells(self) -> "Cells":
        c = Cells(self)
        self._cells.append(c)
        return c

    def check(self, stream=None) -> int:
        """nnps_ctx_check: waits for the stream and returns (and clears) the status of the
        errors the device recorded for this context's asynchronous calls."""
        return self._lib.nnps_ctx_check(self._ctx, _stream_ptr(stream))


class Cells:
    """A device-resident cell structure (nnps_cells)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self._lib = ctx._lib
        h = ctypes.c_void_p()
        _check(self._lib.nnps_cells_create(ctx._ctx, ctypes.byref(h)), "nnps_cells_create")
        self._h = h
        self.n = 0
        self.nsets = 0
        self._pos = None

    def close(self):
        if self._h:
            self._lib.nnps_cells_destroy(self._h)
            self._h = None

    def build(self, pos, lo, hi, cell_size, radius, mode=MODE_FP16_RCLL, stream=None):
        """pos: torch float64 CUDA tensor [n, dim], contiguous."""
        import torch
        assert pos.is_cuda and pos.dtype == torch.float64 and pos.is_contiguous() and pos.dim() == 2
        n, dim = pos.shape
        prob = make_problem(dim, n, lo, hi, cell_size, radius, mode)
        _check(self._lib.nnps_cells_build(self.ctx._ctx, self._h, ctypes.byref(prob), _ptr(pos),
                                          _stream_ptr(stream)), "nnps_cells_build")
        self.n = n
        self.nsets = 1
        self._pos = pos  # keep alive: the recheck reads it
        return self

    def count(self, row_ptr, sync=True, stream=None):
        """row_ptr: torch int64 CUDA tensor [n+1]. Returns nnz when sync, else None."""
        nnz = ctypes.c_int64(-1)
        _check(self._lib.nnps_count(self.ctx._ctx, self._h, _ptr(row_ptr),
                                    ctypes.byref(nnz) if sync else None, _stream_ptr(stream)),
               "nnps_count")
        return nnz.value if sync else None

    def fill(self, row_ptr, col, dist, stream=None):
        cap = col.numel()
        assert dist.numel() == cap
        _check(self._lib.nnps_fill(self.ctx._ctx, self._h, _ptr(row_ptr), _ptr(col), _ptr(dist), cap,
                                   _stream_ptr(stream)), "nnps_fill")

    # ---- batches ------------------------------------------------------------------
    def batch_build(self, sets, mode=MODE_FP16_RCLL, stream=None):
        """sets: list of (pos tensor [n, dim] float64 CUDA, lo, hi, cell_size, radius)."""
        probs, ptrs = _batch_args(sets, mode)
        _check(self._lib.nnps_batch_build(self.ctx._ctx, self._h, len(sets), probs, ptrs,
                                          _stream_ptr(stream)), "nnps_batch_build")
        self.nsets = len(sets)
        self._pos = [t[0] for t in sets]
        return self

    def batch_count(self, row_ptrs, sync=True, stream=None):
        rp = _ptr_array(row_ptrs)
        nnz = (ctypes.c_int64 * len(row_ptrs))()
        _check(self._lib.nnps_batch_count(self.ctx._ctx, self._h, rp, nnz if sync else None,
                                          _stream_ptr(stream)), "nnps_batch_count")
        return list(nnz) if sync else None

    def batch_fill(self, row_ptrs, cols, dists, stream=None):
        cap = (ctypes.c_int64 * len(cols))(*[c.numel() for c in cols])
        _check(self._lib.nnps_batch_fill(self.ctx._ctx, self._h, _ptr_array(row_ptrs), _ptr_array(cols),
                                         _ptr_array(dists), cap, _stream_ptr(stream)), "nnps_batch_fill")

    def batch_step(self, sets, row_ptrs, cols, dists, mode=MODE_FP16_RCLL, stream=None):
        """Build + count + fill without waiting; outputs must already be large enough."""
        probs, ptrs = _batch_args(sets, mode)
        cap = (ctypes.c_int64 * len(cols))(*[c.numel() for c in cols])
        _check(self._lib.nnps_batch_step(self.ctx._ctx, self._h, len(sets), probs, ptrs,
                                         _ptr_array(row_ptrs), _ptr_array(cols), _ptr_array(dists), cap,
                                         _stream_ptr(stream)), "nnps_batch_step")
        self.nsets = len(sets)
        self._pos = [t[0] for t in sets]

    def update(self, disp=None, stream=None):
        """Incremental update after the particles moved (nnps_cells_update). disp: None (the
        positions of the last build were moved in place by the caller), a float64 CUDA
        tensor [n, dim] for a single-set structure, or a list with one tensor or None per
        set; given displacements are added to the positions in place."""
        _check(self._lib.nnps_cells_update(self.ctx._ctx, self._h, self._disp_array(disp), _stream_ptr(stream)),
               "nnps_cells_update")
        return self

    def batch_update_step(self, row_ptrs, cols, dists, disp=None, stream=None):
        """Update + count + fill without waiting (nnps_batch_update_step); outputs must
        already be large enough."""
        cap = (ctypes.c_int64 * len(cols))(*[c.numel() for c in cols])
        _check(self._lib.nnps_batch_update_step(self.ctx._ctx, self._h, self._disp_array(disp), _ptr_array(row_ptrs),
                                                _ptr_array(cols), _ptr_array(dists), cap, _stream_ptr(stream)),
               "nnps_batch_update_step")

    def _disp_array(self, disp):
        import torch
        if disp is None:
            return None
        if isinstance(disp, torch.Tensor):
            disp = [disp]
        for d in disp:
            assert d is None or (d.is_cuda and d.dtype == torch.float64 and d.is_contiguous())
        self._disp = disp  # keep alive until the caller synchronises
        return _ptr_array([d if d is not None else None for d in disp])

    def batch_nnz(self, stream=None, check: bool = True):
        """Each set's nnz of the last count (waits for the stream). With check=False returns
        (nnz list, status) instead of raising on a device-reported error."""
        nnz = (ctypes.c_int64 * self.nsets)()
        code = self._lib.nnps_batch_nnz(self._h, nnz, _stream_ptr(stream))
        if not check:
            return list(nnz), code
        _check(code, "nnps_batch_nnz")
        return list(nnz)

    def set_half(self, on: bool = True):
        """Half lists: rows keep only neighbours of larger original index (nnps_cells_set_half)."""
        _check(self._lib.nnps_cells_set_half(self._h, 1 if on else 0), "nnps_cells_set_half")

    def batch_nnz_enqueue(self, stream=None):
        """Queue the copies of each set's nnz and the error flags to pinned host memory."""
        _check(self._lib.nnps_batch_nnz_enqueue(self._h, _stream_ptr(stream)), "nnps_batch_nnz_enqueue")

    def batch_nnz_fetch(self, check: bool = True):
        """Each set's nnz from the last enqueue (waits only for those copies)."""
        nnz = (ctypes.c_int64 * self.nsets)()
        code = self._lib.nnps_batch_nnz_fetch(self._h, nnz)
        if not check:
            return list(nnz), code
        _check(code, "nnps_batch_nnz_fetch")
        return list(nnz)

    def set_graphs(self, on: bool = True):
        _check(self._lib.nnps_cells_set_graphs(self._h, 1 if on else 0), "nnps_cells_set_graphs")

    def set_profiling(self, on: bool = True):
        _check(self._lib.nnps_cells_set_profiling(self._h, 1 if on else 0), "nnps_cells_set_profiling")

    def phase_times(self, stream=None) -> dict:
        """{phase: (summed device ms, launches)} since profiling was turned on or last read."""
        ms = (ctypes.c_double * len(PHASES))()
        runs = (ctypes.c_int32 * len(PHASES))()
        _check(self._lib.nnps_phase_times(self._h, ms, runs, _stream_ptr(stream)), "nnps_phase_times")
        return {k: (ms[i], runs[i]) for i, k in enumerate(PHASES)}

    def stats(self, stream=None) -> dict:
        st = Stats()
        code = self._lib.nnps_stats_get(self._h, ctypes.byref(st), _stream_ptr(stream))
        _check(code, "nnps_stats_get")
        return st.as_dict()


PROBE_KINDS = {"pk_fma_f16": 0, "fma_f32": 1, "int32": 2}


def probe_valu_rate(kind: str, device: int = 0):
    """nnps_probe_valu_rate: (wave64 VALU instructions per second, instructions per wave)
    on long runs of independent instructions of `kind` (a key of PROBE_KINDS)."""
    rate = ctypes.c_double(0.0)
    per = ctypes.c_int64(0)
    _check(load().nnps_probe_valu_rate(int(device), PROBE_KINDS[kind], ctypes.byref(rate), ctypes.byref(per)),
           "nnps_probe_valu_rate")
    return rate.value, per.value


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr() if t is not None and t.numel() > 0 else None
    return arr


def _batch_args(sets, mode):
    probs = (Problem * len(sets))()
    ptrs = (ctypes.c_void_p * len(sets))()
    for i, (pos, lo, hi, cell_size, radius) in enumerate(sets):
        n, dim = pos.shape
        probs[i] = make_problem(dim, n, lo, hi, cell_size, radius, mode)
        ptrs[i] = pos.data_ptr() if n > 0 else None
    return probs, ptrs


def search_batch(sets, mode=MODE_FP16_RCLL, ctx: Context | None = None, cells: Cells | None = None,
                 stream=None):
    """Search every set of `sets` (list of (pos, lo, hi, cell_size, radius)) in one batch.
    Returns a list of (row_ptr, col, dist) CUDA tensors, one per set, and the cells."""
    import torch
    if ctx is None:
        ctx = Context(sets[0][0].device.index or 0)
    if cells is None:
        cells = ctx.cells()
    cells.batch_build(sets, mode, stream)
    dev = sets[0][0].device
    rps = [torch.empty(t[0].shape[0] + 1, dtype=torch.int64, device=dev) for t in sets]
    nnz = cells.batch_count(rps, sync=True, stream=stream)
    cols = [torch.empty(max(k, 0), dtype=torch.int32, device=dev) for k in nnz]
    dists = [torch.empty(max(k, 0), dtype=torch.float32, device=dev) for k in nnz]
    cells.batch_fill(rps, cols, dists, stream)
    return list(zip(rps, cols, dists)), cells


def allpairs_search(pos, lo, hi, radius, ctx: Context | None = None, stream=None):
    """All-list search of a small set (nnps_allpairs_count, then nnps_allpairs_fill into
    outputs of exactly nnz entries): returns (row_ptr, col, dist) as CUDA tensors; binary64,
    the same result as the FP64 cell list."""
    import torch
    n, dim = pos.shape
    assert pos.is_cuda and pos.dtype == torch.float64 and pos.is_contiguous()
    own = ctx is None
    ctx = ctx or Context(pos.device.index or 0)
    try:
        prob = make_problem(dim, n, lo, hi, radius, radius, MODE_FP64_BASELINE)
        rp = torch.empty(n + 1, dtype=torch.int64, device=pos.device)
        nnz = ctypes.c_int64(0)
        _check(ctx._lib.nnps_allpairs_count(ctx._ctx, ctypes.byref(prob), _ptr(pos), _ptr(rp), ctypes.byref(nnz),
                                            _stream_ptr(stream)), "nnps_allpairs_count")
        col = torch.empty(nnz.value, dtype=torch.int32, device=pos.device)
        dist = torch.empty(nnz.value, dtype=torch.float32, device=pos.device)
        _check(ctx._lib.nnps_allpairs_fill(ctx._ctx, ctypes.byref(prob), _ptr(pos), _ptr(rp), _ptr(col), _ptr(dist),
                                           nnz.value, _stream_ptr(stream)), "nnps_allpairs_fill")
    finally:
        if own:
            torch.cuda.synchronize()
            ctx.close()
    return rp, col, dist


def allpairs_search_noalloc(pos, lo, hi, radius, row_ptr, col, dist, ctx: Context, stream=None):
    """nnps_allpairs_search_noalloc into caller-sized outputs (row_ptr [n+1] int64, col
    int32 and dist float32 of equal length, the capacity): returns (status, nnz). The
    library allocates nothing for it; its scratch is a static device array."""
    import torch
    n, dim = pos.shape
    assert pos.is_cuda and pos.dtype == torch.float64 and pos.is_contiguous()
    assert row_ptr.dtype == torch.int64 and row_ptr.numel() == n + 1
    assert col.dtype == torch.int32 and dist.dtype == torch.float32 and col.numel() == dist.numel()
    prob = make_problem(dim, n, lo, hi, radius, radius, MODE_FP64_BASELINE)
    nnz = ctypes.c_int64(0)
    st = ctx._lib.nnps_allpairs_search_noalloc(ctx._ctx, ctypes.byref(prob), _ptr(pos), _ptr(row_ptr), _ptr(col),
                                               _ptr(dist), int(col.numel()), ctypes.byref(nnz),
                                               _stream_ptr(stream))
    return st, int(nnz.value)


def sph_gradient(pos, f, h, row_ptr, col, vol=None, ctx: Context | None = None, want=("grad", "grad_norm"),
                 stream=None):
    """SPH gradient of the scalar field f over a CSR neighbour list (nnps_sph_gradient):
    returns (grad, grad_norm), float64 CUDA tensors [n, dim] (None where not in `want`)."""
    import torch
    n, dim = pos.shape
    for t, dt in ((pos, torch.float64), (f, torch.float64), (row_ptr, torch.int64), (col, torch.int32)):
        assert t.is_cuda and t.dtype == dt and t.is_contiguous()
    assert f.numel() == n and row_ptr.numel() == n + 1
    if vol is not None:
        assert vol.is_cuda and vol.dtype == torch.float64 and vol.numel() == n and vol.is_contiguous()
    own = ctx is None
    ctx = ctx or Context(pos.device.index or 0)
    try:
        grad = torch.empty((n, dim), dtype=torch.float64, device=pos.device) if "grad" in want else None
        gnorm = torch.empty((n, dim), dtype=torch.float64, device=pos.device) if "grad_norm" in want else None
        # the kernel reads col only within its length (rows are clamped to it)
        _check(ctx._lib.nnps_sph_gradient(ctx._ctx, int(dim), int(n), float(h), _ptr(pos), _ptr(f),
                                          _ptr(vol) if vol is not None else None, _ptr(row_ptr), _ptr(col),
                                          int(col.numel()), _ptr(grad) if grad is not None else None,
                                          _ptr(gnorm) if gnorm is not None else None, _stream_ptr(stream)),
               "nnps_sph_gradient")
    finally:
        if own:
            torch.cuda.synchronize()
            ctx.close()
    return grad, gnorm


def search(pos, lo, hi, cell_size, radius, mode=MODE_FP16_RCLL, ctx: Context | None = None,
           cells: Cells | None = None, stream=None):
    """Build + count + fill. Returns (row_ptr int64 [n+1], col int32 [nnz], dist float32 [nnz])
    as CUDA tensors, plus the cell structure used."""
    import torch
    own = ctx is None
    if ctx is None:
        ctx = Context(pos.device.index or 0)
    if cells is None:
        cells = ctx.cells()
    cells.build(pos, lo, hi, cell_size, radius, mode, stream)
    row_ptr = torch.empty(pos.shape[0] + 1, dtype=torch.int64, device=pos.device)
    nnz = cells.count(row_ptr, sync=True, stream=stream)
    col = torch.empty(max(nnz, 0), dtype=torch.int32, device=pos.device)
    dist = torch.empty(max(nnz, 0), dtype=torch.float32, device=pos.device)
    cells.fill(row_ptr, col, dist, stream)
    if own:
        cells.stats(stream)  # surfaces device-side errors before the context goes away
    return row_ptr, col, dist, cells
