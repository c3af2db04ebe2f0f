"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every function
include/nnps.h declares, validates arguments as documented, and lays out the same grid
as the FP16 model in the oracle package."""
import ctypes
import math
import os
import re

import pytest

from oracle import rcll_fp16 as M
from paper_2401_08586_amd import nnps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "nnps.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nnps_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = nnps.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(nnps.EXPORTS) == set(names)


def test_status_strings():
    for code in range(-8, 1):
        s = nnps.status_str(code)
        assert s.startswith("NNPS_")
    assert "UNKNOWN" in nnps.status_str(-99)


def P(**kw):
    base = dict(dim=3, n=10, lo=(0, 0, 0), hi=(1, 1, 1), cell_size=0.1, radius=0.1, mode=0)
    base.update(kw)
    return nnps.make_problem(base["dim"], base["n"], base["lo"], base["hi"], base["cell_size"],
                             base["radius"], base["mode"])


@pytest.mark.parametrize("kw,want", [
    ({}, nnps.NNPS_OK),
    (dict(dim=2, lo=(0, 0), hi=(1, 1)), nnps.NNPS_OK),
    (dict(n=0), nnps.NNPS_OK),
    (dict(dim=1), nnps.NNPS_EINVAL),
    (dict(dim=4), nnps.NNPS_EINVAL),
    (dict(n=-1), nnps.NNPS_EINVAL),
    (dict(n=1 << 31), nnps.NNPS_EINVAL),
    (dict(radius=0.2), nnps.NNPS_EINVAL),           # radius above the cell size
    (dict(radius=0.0), nnps.NNPS_EINVAL),
    (dict(radius=float("nan")), nnps.NNPS_EINVAL),
    (dict(cell_size=float("inf")), nnps.NNPS_EINVAL),
    (dict(hi=(1, 0, 1)), nnps.NNPS_EINVAL),          # empty box
    (dict(lo=(0, float("nan"), 0)), nnps.NNPS_EINVAL),
    (dict(mode=3), nnps.NNPS_OK),
    (dict(mode=4), nnps.NNPS_EINVAL),
    (dict(hi=(1e4, 1e4, 1e4), cell_size=1.0, radius=1.0), nnps.NNPS_ETOOMANYCELLS),
])
def test_validate(kw, want):
    assert nnps.validate(P(**kw)) == want


@pytest.mark.parametrize("dim,lo,hi,cell,r", [
    (3, (0, 0, 0), (1, 1, 1), 0.024, 0.024),
    (2, (0, 0), (1, 1), 0.0024, 0.0024),
    (2, (-1.25, -1.25), (1.75, 1.75), 0.05, 0.03),
    (3, (0, 0, 0), (2, 2, 2), 2.0, 1.4142135623730951),
    (2, (0, 0), (40, 0.2), 0.03, 0.03),
    (3, (0, 0, 0), (0.5, 3.0, 1.0), 0.125, 0.125),   # L / w an exact integer
])
def test_grid_matches_model(dim, lo, hi, cell, r):
    nc, F, w = nnps.grid(nnps.make_problem(dim, 100, lo, hi, cell, r))
    fr = M.frame(dim, lo, hi, cell, r)
    assert w == fr["w"]
    assert F == fr["F"]
    assert nc[:dim] == fr["nc"]
    assert all(v == 1 for v in nc[dim:])
    # every pair within the radius is at most one cell apart: w >= R (1 + 2^-31)
    assert w >= r * (1 + 2.0 ** -31)
    assert 2 ** F * max(nc) < 2 ** 52


def test_context_without_device_fails_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = nnps.load()
    h = ctypes.c_void_p()
    assert lib.nnps_ctx_create(0, ctypes.byref(h)) == nnps.NNPS_EDEVICE
    assert not h.value


def test_null_arguments_rejected():
    lib = nnps.load()
    assert lib.nnps_validate(None) == nnps.NNPS_EINVAL
    assert lib.nnps_ctx_create(0, None) == nnps.NNPS_EINVAL
    assert lib.nnps_count(None, None, None, None, None) == nnps.NNPS_EINVAL
    assert lib.nnps_fill(None, None, None, None, None, 0, None) == nnps.NNPS_EINVAL
    assert lib.nnps_stats_get(None, None, None) == nnps.NNPS_EINVAL
    assert lib.nnps_cells_set_profiling(None, 1) == nnps.NNPS_EINVAL
    lib.nnps_ctx_destroy(None)
    lib.nnps_cells_destroy(None)
    assert math.isfinite(1.0)
