"""The all-list path (nnps_allpairs_search, Fig. 3a) against the oracle's brute force:
row_ptr and col equal, distances bit-identical (both binary64, then rounded to FP32); the
error paths (capacity, domain, size limit)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2401_08586_amd import nnps
from paper_2401_08586_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = nnps.Context(0)
    yield c
    c.close()


def run(ctx, ps):
    pos = torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda()
    rp, col, dist = nnps.allpairs_search(pos, ps.lo, ps.hi, ps.radius, ctx=ctx)
    torch.cuda.synchronize()
    return rp.cpu().numpy(), col.cpu().numpy(), dist.cpu().numpy()


CASES = [
    lambda: W.uniform(2, 3000, seed=1),
    lambda: W.uniform(3, 16001, seed=5),  # 32 slices of 512 candidates, ragged last slice and row group
    lambda: W.uniform(3, 5000, seed=2),
    lambda: W.lattice(2, 50, 0.02, 0.0, name="lat2d_perfect"),
    lambda: W.lattice(3, 12, 1 / 12, 0.1, seed=3),
    lambda: W.clustered(4000, 7, dim=3),
    lambda: W.ring_pairs(500, 0.05, seed=8, dim=2),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_allpairs_matches_brute_force(ctx, case):
    ps = CASES[case]()
    print(f"[gpu] allpairs {ps.name} n={ps.n}", flush=True)
    want = oracle.search_ps(ps, brute=True)
    got = run(ctx, ps)
    np.testing.assert_array_equal(got[0], want[0])
    np.testing.assert_array_equal(got[1], want[1])
    np.testing.assert_array_equal(got[2].view(np.uint32), want[2].view(np.uint32))


@pytest.mark.parametrize("n", [20000, 65536])
def test_allpairs_equals_the_fp64_cell_list(ctx, n):
    """Up to the largest set the path takes; sampled rows also against the oracle."""
    ps = W.uniform(3, n, seed=4)
    pos = torch.from_numpy(ps.pos).cuda()
    a = nnps.allpairs_search(pos, ps.lo, ps.hi, ps.radius, ctx=ctx)
    b = nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, mode=nnps.MODE_FP64_BASELINE, ctx=ctx)[:3]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    rows = np.random.default_rng(n).choice(n, 200, replace=False)
    wrp, wcol, wdist = oracle.search_rows(ps.pos, ps.lo, ps.hi, ps.cell_size, ps.radius, rows)
    rp, col, dist = (t.cpu().numpy() for t in a)
    for k, i in enumerate(rows):
        got = slice(rp[i], rp[i + 1])
        want = slice(wrp[k], wrp[k + 1])
        np.testing.assert_array_equal(col[got], wcol[want])
        np.testing.assert_array_equal(dist[got].view(np.uint32), wdist[want].view(np.uint32))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 257])
def test_allpairs_tiny_sets_and_duplicates(ctx, n):
    rng = np.random.default_rng(n)
    pos = rng.uniform(0, 1, (n, 3))
    if n >= 2:
        pos[1] = pos[0]  # coincident particles are neighbours
    ps = W.ParticleSet(np.ascontiguousarray(pos), (0, 0, 0), (1, 1, 1), 0.3, 0.3, f"tiny{n}")
    got = run(ctx, ps)
    if n == 0:
        assert got[0].tolist() == [0] and got[1].size == 0
        return
    want = oracle.search_ps(ps, brute=True)
    for x, y in zip(got[:2], want[:2]):
        np.testing.assert_array_equal(x, y)


def test_allpairs_errors(ctx):
    lib = nnps.load()
    import ctypes
    pos = torch.tensor([[0.1, 0.1], [0.2, 0.2], [1.5, 0.5]], dtype=torch.float64, device="cuda")
    rp = torch.empty(4, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64(0)
    prob = nnps.make_problem(2, 3, (0, 0), (1, 1), 0.5, 0.5)
    code = lib.nnps_allpairs_search(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), None, None, 0,
                                    ctypes.byref(nnz), None)
    assert code == nnps.NNPS_EDOMAIN
    pos[2, 0] = 0.3
    code = lib.nnps_allpairs_search(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), None, None, 0,
                                    ctypes.byref(nnz), None)
    assert code == nnps.NNPS_ECAPACITY and nnz.value == 6
    # count then fill: the fill needs the count's problem, positions and row pointers
    col = torch.empty(6, dtype=torch.int32, device="cuda")
    dist = torch.empty(6, dtype=torch.float32, device="cuda")
    assert lib.nnps_allpairs_count(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), ctypes.byref(nnz),
                                   None) == nnps.NNPS_OK and nnz.value == 6
    rp2 = torch.empty(4, dtype=torch.int64, device="cuda")
    assert lib.nnps_allpairs_fill(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp2), nnps._ptr(col),
                                  nnps._ptr(dist), 6, None) == nnps.NNPS_EORDER
    assert lib.nnps_allpairs_fill(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), nnps._ptr(col),
                                  nnps._ptr(dist), 5, None) == nnps.NNPS_ECAPACITY
    assert lib.nnps_allpairs_fill(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), nnps._ptr(col),
                                  nnps._ptr(dist), 6, None) == nnps.NNPS_OK
    torch.cuda.synchronize()
    assert rp.cpu().tolist() == [0, 2, 4, 6] and col.cpu().tolist() == [1, 2, 0, 2, 0, 1]
    # a count that fails leaves nothing to fill
    pos[2, 0] = 1.5
    assert lib.nnps_allpairs_count(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), ctypes.byref(nnz),
                                   None) == nnps.NNPS_EDOMAIN
    assert lib.nnps_allpairs_fill(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp), nnps._ptr(col),
                                  nnps._ptr(dist), 6, None) == nnps.NNPS_EORDER
    big = nnps.make_problem(2, 65537, (0, 0), (1, 1), 0.5, 0.5)
    code = lib.nnps_allpairs_search(ctx._ctx, ctypes.byref(big), nnps._ptr(pos), nnps._ptr(rp), None, None, 0,
                                    ctypes.byref(nnz), None)
    assert code == nnps.NNPS_EINVAL


def test_allpairs_fill_stays_in_its_rows_when_counts_are_stale(ctx):
    """The fill writes row i only inside [row_ptr[i], min(row_ptr[i+1], capacity)). Row
    pointers that no longer match the count (rows shortened, or moved past the capacity,
    after the count) leave every entry outside those bounds untouched, and nnps_ctx_check
    reports the mismatch once."""
    import ctypes
    ps = W.uniform(3, 3000, seed=4)
    pos = torch.from_numpy(ps.pos).cuda()
    prob = nnps.make_problem(3, ps.n, ps.lo, ps.hi, ps.radius, ps.radius, nnps.MODE_FP64_BASELINE)
    rp = torch.empty(ps.n + 1, dtype=torch.int64, device="cuda")
    nnz = ctypes.c_int64(0)
    lib = ctx._lib
    assert lib.nnps_allpairs_count(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp),
                                   ctypes.byref(nnz), None) == nnps.NNPS_OK
    assert ctx.check() == nnps.NNPS_OK
    ref_rp = rp.cpu().numpy()
    nz = int(nnz.value)
    assert nz > 1000
    lens = np.diff(ref_rp)
    short = ref_rp.copy()
    short[1:] = np.maximum.accumulate(ref_rp[1:] - lens // 2)   # every row shorter than counted
    shifted = ref_rp + 100                                        # the last rows run past nz
    for name, new_rp in (("short", short), ("shifted", shifted)):
        rp.copy_(torch.from_numpy(new_rp))
        col = torch.full((nz + 200,), -7, dtype=torch.int32, device="cuda")
        dist = torch.full((nz + 200,), -1.0, dtype=torch.float32, device="cuda")
        assert lib.nnps_allpairs_fill(ctx._ctx, ctypes.byref(prob), nnps._ptr(pos), nnps._ptr(rp),
                                      nnps._ptr(col), nnps._ptr(dist), nz, None) == nnps.NNPS_OK, name
        torch.cuda.synchronize()
        c = col.cpu().numpy()
        assert np.all(c[nz:] == -7), name                       # nothing at or past the capacity
        inside = np.zeros(nz + 200, bool)
        for i in range(ps.n):
            inside[new_rp[i]:min(new_rp[i + 1], nz)] = True
        assert np.all(c[~inside] == -7), name                   # nothing outside the rows
        assert ctx.check() == nnps.NNPS_EORDER, name
        assert ctx.check() == nnps.NNPS_OK, name
