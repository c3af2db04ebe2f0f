"""The allocation-free all-list entry point (nnps_allpairs_search_noalloc), called through
the C ABI, against the allocating one (nnps_allpairs_search) on the same inputs: row_ptr,
col and dist bit-identical, on two calls in a row (the second with a smaller set, so the
static scratch holds the first call's larger contents), then the error paths."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2401_08586_amd import nnps
from paper_2401_08586_amd import workloads as W

pytestmark = pytest.mark.gpu

GUARD = 32


def reference(ctx, ps, pos):
    """The existing entry point, outputs sized by a first call that reports the need."""
    lib = ctx._lib
    prob = nnps.make_problem(ps.dim, ps.n, ps.lo, ps.hi, ps.radius, ps.radius, nnps.MODE_FP64_BASELINE)
    rp = torch.empty(ps.n + 1, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64(0)
    st = lib.nnps_allpairs_search(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), None, None, 0,
                                  ctypes.byref(nnz), None)
    assert st in (nnps.NNPS_OK, nnps.NNPS_ECAPACITY)
    col = torch.empty(nnz.value, dtype=torch.int32, device="cuda")
    dist = torch.empty(nnz.value, dtype=torch.float32, device="cuda")
    st = lib.nnps_allpairs_search(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), nnps._ptr(col),
                                  nnps._ptr(dist), nnz.value, ctypes.byref(nnz), None)
    assert st == nnps.NNPS_OK
    torch.cuda.synchronize()
    return rp.cpu().numpy(), col.cpu().numpy(), dist.cpu().numpy()


def test_noalloc_equals_allocating_entry_point_twice():
    ctx = nnps.Context(0)
    try:
        for ps in (W.uniform(3, 5000, seed=21), W.clustered(1200, 22, dim=3)):
            print(f"[gpu] noalloc n={ps.n} dim={ps.dim}", flush=True)
            pos = torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda()
            want_rp, want_col, want_dist = reference(ctx, ps, pos)
            nz = int(want_rp[-1])
            rp = torch.full((ps.n + 1,), -5, dtype=torch.int64, device="cuda")
            col = torch.full((nz + GUARD,), -7, dtype=torch.int32, device="cuda")
            dist = torch.full((nz + GUARD,), -1.0, dtype=torch.float32, device="cuda")
            st, nnz = nnps.allpairs_search_noalloc(pos, ps.lo, ps.hi, ps.radius, rp, col, dist, ctx=ctx)
            torch.cuda.synchronize()
            assert st == nnps.NNPS_OK and nnz == nz
            c = col.cpu().numpy()
            d = dist.cpu().numpy()
            assert np.array_equal(rp.cpu().numpy(), want_rp)
            assert np.array_equal(c[:nz], want_col)
            assert np.array_equal(d[:nz].view(np.uint32), want_dist.view(np.uint32))
            assert np.all(c[nz:] == -7) and np.all(d[nz:] == -1.0)
        assert ctx.check() == nnps.NNPS_OK
    finally:
        ctx.close()


def test_noalloc_errors():
    ctx = nnps.Context(0)
    try:
        ps = W.uniform(2, 800, seed=23)
        pos = torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda()
        want_rp, _, _ = reference(ctx, ps, pos)
        nz = int(want_rp[-1])
        rp = torch.empty(ps.n + 1, dtype=torch.int64, device="cuda")
        small = nz - 1
        col = torch.full((small,), -7, dtype=torch.int32, device="cuda")
        dist = torch.full((small,), -1.0, dtype=torch.float32, device="cuda")
        st, nnz = nnps.allpairs_search_noalloc(pos, ps.lo, ps.hi, ps.radius, rp, col, dist, ctx=ctx)
        torch.cuda.synchronize()
        assert st == nnps.NNPS_ECAPACITY and nnz == nz
        assert np.array_equal(rp.cpu().numpy(), want_rp)
        assert np.all(col.cpu().numpy() == -7)
        # a position outside the box
        bad = pos.clone()
        bad[17, 1] = 2.0
        st, _ = nnps.allpairs_search_noalloc(bad, ps.lo, ps.hi, ps.radius, rp, col, dist, ctx=ctx)
        assert st == nnps.NNPS_EDOMAIN
        # above the size the static scratch is made for: refused before any device work
        lib = ctx._lib
        prob = nnps.make_problem(2, 65537, ps.lo, ps.hi, ps.radius, ps.radius, nnps.MODE_FP64_BASELINE)
        n_out = ctypes.c_int64(0)
        assert lib.nnps_allpairs_search_noalloc(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp),
                                                None, None, 0, ctypes.byref(n_out), None) == nnps.NNPS_EINVAL
        # empty set
        empty = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
        rp0 = torch.full((1,), 9, dtype=torch.int64, device="cuda")
        e_col = torch.zeros(0, dtype=torch.int32, device="cuda")
        e_dist = torch.zeros(0, dtype=torch.float32, device="cuda")
        st, nnz = nnps.allpairs_search_noalloc(empty, ps.lo, ps.hi, ps.radius, rp0, e_col, e_dist, ctx=ctx)
        torch.cuda.synchronize()
        assert st == nnps.NNPS_OK and nnz == 0 and int(rp0.item()) == 0
    finally:
        ctx.close()
