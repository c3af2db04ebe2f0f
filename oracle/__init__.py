"""CPU oracle for the fixed-radius neighbour search (test infrastructure only).

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py` may
import this package. The product path (the HIP library and its binding) never
touches it, and it shares no code with that path.

* `search` / `search_rows`: the serial FP64 cell link-list search in plain C
  (nnps_oracle.c), with the all-list brute force for small inputs.
* `count_rows` / `search_par`: the same cell-list search with rows computed in parallel
  (OpenMP over rows; each row exactly as in the serial search), for the full-size
  clustered batch and the all-core CPU baseline.
* `rcll_fp16`: a numpy model of the FP16 relative-coordinate test, used to check
  the GPU's FP16 statistics bit for bit.
* `rcll_fp32`: the same for the FP32 relative-coordinate test.
* `sph_gradient`: the SPH gradient sums (Eq. 2 with the kernel of Eq. 3, and Eq. A5).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nnps_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_OK, ORC_EINVAL, ORC_EDOMAIN, ORC_ENOMEM = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile nnps_oracle.c with plain IEEE binary64 semantics (no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_search.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, ctypes.POINTER(P)]
        lib.orc_search.restype = ctypes.c_int
        lib.orc_search_rows.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_double,
                                        ctypes.c_double, P, ctypes.c_int64, ctypes.POINTER(P)]
        lib.orc_search_rows.restype = ctypes.c_int
        lib.orc_count_rows.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_double,
                                       P, ctypes.c_int64, ctypes.c_int, P]
        lib.orc_count_rows.restype = ctypes.c_int
        lib.orc_search_par.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_double,
                                       P, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(P)]
        lib.orc_search_par.restype = ctypes.c_int
        lib.orc_nnz.argtypes = [P]
        lib.orc_nnz.restype = ctypes.c_int64
        lib.orc_copy.argtypes = [P, P, P, P]
        lib.orc_copy.restype = None
        lib.orc_free.argtypes = [P]
        lib.orc_free.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _collect(lib, h, nrows):
    nnz = lib.orc_nnz(h)
    row_ptr = np.empty(nrows + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.int32)
    dist = np.empty(nnz, dtype=np.float32)
    lib.orc_copy(h, _ptr(row_ptr), _ptr(col), _ptr(dist))
    lib.orc_free(h)
    return row_ptr, col, dist


def _box(lo, hi, dim):
    lo3 = np.zeros(3)
    hi3 = np.zeros(3)
    lo3[:dim] = lo[:dim]
    hi3[:dim] = hi[:dim]
    return lo3, hi3


def search(pos, lo, hi, cell_size, radius, brute=False):
    """CSR (row_ptr int64 [n+1], col int32 [nnz] ascending per row, dist float32 [nnz])."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    lo3, hi3 = _box(lo, hi, dim)
    h = ctypes.c_void_p()
    st = lib.orc_search(dim, n, _ptr(pos), _ptr(lo3), _ptr(hi3), float(cell_size), float(radius),
                        1 if brute else 0, ctypes.byref(h))
    if st != ORC_OK:
        raise OracleError(st)
    return _collect(lib, h, n)


def search_rows(pos, lo, hi, cell_size, radius, rows):
    """The rows of the listed targets only (CSR with len(rows) rows, in the given order)."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    lo3, hi3 = _box(lo, hi, dim)
    h = ctypes.c_void_p()
    st = lib.orc_search_rows(dim, n, _ptr(pos), _ptr(lo3), _ptr(hi3), float(cell_size),
                             float(radius), _ptr(rows), rows.size, ctypes.byref(h))
    if st != ORC_OK:
        raise OracleError(st)
    return _collect(lib, h, rows.size)


def count_rows(pos, lo, hi, cell_size, radius, rows=None, threads=0):
    """Neighbour count of every row (or of the listed rows), int64; rows in parallel."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    lo3, hi3 = _box(lo, hi, dim)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if r is None else r.size
    out = np.empty(m, dtype=np.int64)
    st = lib.orc_count_rows(dim, n, _ptr(pos), _ptr(lo3), _ptr(hi3), float(cell_size), float(radius),
                            _ptr(r), m, int(threads), _ptr(out))
    if st != ORC_OK:
        raise OracleError(st)
    return out


def search_par(pos, lo, hi, cell_size, radius, rows=None, threads=0):
    """`search` (or `search_rows` when rows are given) with rows computed in parallel."""
    lib = _load()
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    lo3, hi3 = _box(lo, hi, dim)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if r is None else r.size
    h = ctypes.c_void_p()
    st = lib.orc_search_par(dim, n, _ptr(pos), _ptr(lo3), _ptr(hi3), float(cell_size), float(radius),
                            _ptr(r), m, int(threads), ctypes.byref(h))
    if st != ORC_OK:
        raise OracleError(st)
    return _collect(lib, h, m)


def search_ps(ps, brute=False):
    """`search` on a workloads.ParticleSet."""
    return search(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, brute=brute)
