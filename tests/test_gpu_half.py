"""Half lists (nnps_cells_set_half): row i keeps only neighbours j > i. Checked against the
oracle's full neighbour lists restricted to j > i, on every path (block, dense-cell, long
rows), every mode, batches and graph replays; the half nnz is exactly half the full one
(the relation is symmetric)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2401_08586_amd import nnps
from paper_2401_08586_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = (nnps.MODE_FP16_RCLL, nnps.MODE_FP64_BASELINE, nnps.MODE_RECHECK_ALL, nnps.MODE_FP32_RCLL)


@pytest.fixture(scope="module")
def ctx():
    c = nnps.Context(0)
    yield c
    c.close()


def upper(rp, col, dist):
    """The oracle's CSR restricted to entries j > i."""
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    keep = col > rows
    hrp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows[keep], minlength=n), out=hrp[1:])
    return hrp, col[keep], dist[keep]


def check(got, want, mode, name):
    rp, col, dist = (t.cpu().numpy() for t in got)
    wrp, wcol, wdist = want
    np.testing.assert_array_equal(rp, wrp, err_msg=f"{name} row_ptr")
    np.testing.assert_array_equal(col, wcol, err_msg=f"{name} col")
    if mode in (nnps.MODE_FP64_BASELINE, nnps.MODE_FP32_RCLL):
        np.testing.assert_array_equal(dist.view(np.uint32), wdist.view(np.uint32), err_msg=f"{name} dist")
    else:
        wd = wdist.astype(np.float64)
        assert np.all(np.abs(dist.astype(np.float64) - wd) <= 1e-6 * wd), name


def half_search(ctx, ps, mode):
    cells = ctx.cells()
    cells.set_half(True)
    pos = torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda()
    rp, col, dist, _ = nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, mode=mode, ctx=ctx, cells=cells)
    st = cells.stats()
    torch.cuda.synchronize()
    cells.close()
    return (rp, col, dist), st


CASES = [
    lambda: W.c0(),
    lambda: W.lattice(3, 30, 1 / 30, 0.1, seed=3, name="lat3d_30"),
    lambda: W.uniform(2, 20000, seed=1),
    lambda: W.uniform(3, 20000, seed=2),
    lambda: W.clustered(8000, 5, dim=3),
    lambda: W.clustered(8000, 6, dim=2),
    lambda: W.ring_pairs(2000, 0.05, seed=8, dim=3),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("mode", MODES)
def test_half_lists_match_the_oracle(ctx, case, mode):
    ps = CASES[case]()
    print(f"[gpu] half {ps.name} mode={mode}", flush=True)
    full = oracle.search_ps(ps)
    want = upper(*full)
    got, _ = half_search(ctx, ps, mode)
    check(got, want, mode, ps.name)
    assert 2 * int(want[0][-1]) == int(full[0][-1])


@pytest.mark.parametrize("dense", [-1, 1])
def test_half_lists_on_the_dense_and_long_row_paths(ctx, dense):
    """dense = 1: every window through the dense-cell path; -1: block and long-row paths."""
    rng = np.random.default_rng(6)
    pos = np.clip(np.concatenate([rng.normal(0.5, 0.01, size=(3000, 3)), rng.uniform(0, 1, size=(3000, 3))]), 0, 1)
    ps = W.ParticleSet(pos, (0, 0, 0), (1, 1, 1), 0.05, 0.05, "half_long_rows")
    want = upper(*oracle.search_ps(ps))
    ctx.set_tuning(dense_min_union=dense)
    try:
        for mode in MODES:
            got, st = half_search(ctx, ps, mode)
            check(got, want, mode, f"{ps.name}_d{dense}_m{mode}")
            if dense == 1:
                assert st["dense_rows"] > 0
            else:
                assert st["heavy_rows"] > 0
    finally:
        ctx.set_tuning()


def test_half_lists_in_a_graph_replayed_batch(ctx):
    pss = [W.uniform(3, 5000, seed=s) for s in range(3)] + [W.clustered(4000, 9, dim=3)]
    sets = [(torch.from_numpy(p.pos).cuda(), p.lo, p.hi, p.cell_size, p.radius) for p in pss]
    wants = [upper(*oracle.search_ps(p)) for p in pss]
    cells = ctx.cells()
    cells.set_half(True)
    cells.set_graphs(True)
    rps = [torch.empty(p.n + 1, dtype=torch.int64, device="cuda") for p in pss]
    cols = [torch.empty(int(w[0][-1]) + 16, dtype=torch.int32, device="cuda") for w in wants]
    dists = [torch.empty(int(w[0][-1]) + 16, dtype=torch.float32, device="cuda") for w in wants]
    stream = torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(stream):
            cells.batch_step(sets, rps, cols, dists, stream=stream)
        nnz = cells.batch_nnz(stream=stream)
        for s, (w, k) in enumerate(zip(wants, nnz)):
            assert k == int(w[0][-1])
            check((rps[s], cols[s][:k], dists[s][:k]), w, nnps.MODE_FP16_RCLL, f"batch{s}_rep{rep}")
    # back to full lists on the same structure
    cells.set_half(False)
    full = oracle.search_ps(pss[0])
    with torch.cuda.stream(stream):
        cells.batch_build(sets[:1])
        rp = torch.empty(pss[0].n + 1, dtype=torch.int64, device="cuda")
        assert cells.batch_count([rp], sync=True)[0] == int(full[0][-1])
    cells.close()
