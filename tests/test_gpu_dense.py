"""GPU parity of the dense-cell path (stencil unions sorted by original index, staged
per chunk for all targets of a cell): element by element against the CPU oracle at
thresholds that send every occupied cell, some cells or no cell through it; its FP16
statistics equal to the block path's; the fallback when the union lists exceed their
capacity; batches and graph replays."""
import numpy as np
import pytest

import oracle
from paper_2401_08586_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2401_08586_amd import nnps  # noqa: E402

STAT_KEYS = ("nnz", "candidates", "band_pairs", "fp16_false_pos", "fp16_false_neg", "outside_band_disagree")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nnps.Context(0)
    yield c
    c.set_tuning()
    c.close()


def run(ctx, ps, mode, **tuning):
    ctx.set_tuning(**tuning)
    try:
        cells = ctx.cells()
        rp, col, dist, _ = nnps.search(torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda(), ps.lo, ps.hi,
                                       ps.cell_size, ps.radius, mode=mode, ctx=ctx, cells=cells)
        st = cells.stats()
        cells.close()
    finally:
        ctx.set_tuning()
    return rp.cpu().numpy(), col.cpu().numpy(), dist.cpu().numpy(), st


def check(got, want, mode, name):
    rp, col, dist, _ = got
    wrp, wcol, wdist = want
    np.testing.assert_array_equal(rp, wrp, err_msg=f"{name} row_ptr")
    np.testing.assert_array_equal(col, wcol, err_msg=f"{name} col")
    if mode in (nnps.MODE_FP64_BASELINE, nnps.MODE_FP32_RCLL):
        np.testing.assert_array_equal(dist.view(np.uint32), wdist.view(np.uint32), err_msg=f"{name} dist")
    else:
        wd = wdist.astype(np.float64)
        assert np.all(np.abs(dist - wd) <= 1e-6 * wd), name
        assert np.all(dist[wdist == 0] == 0), name


def cases():
    rng = np.random.default_rng(31)
    ball = np.clip(np.concatenate([rng.normal(0.5, 0.02, size=(4000, 3)), rng.uniform(0, 1, size=(1500, 3))]), 0, 1)
    disc = np.clip(np.concatenate([rng.normal(0.3, 0.01, size=(3000, 2)), rng.uniform(0, 1, size=(2000, 2))]), 0, 1)
    dup = np.repeat(rng.uniform(0, 1, size=(300, 3)), 4, axis=0)  # coincident particles
    return [
        W.clustered(30000, 41, dim=3),
        W.clustered(20000, 42, dim=2),
        W.ParticleSet(ball, (0, 0, 0), (1, 1, 1), 0.05, 0.05, "ball3d"),
        W.ParticleSet(disc, (0, 0), (1, 1), 0.02, 0.02, "disc2d"),
        W.ParticleSet(dup, (0, 0, 0), (1, 1, 1), 0.08, 0.08, "duplicates3d"),
        W.ParticleSet(ball, (0, 0, 0), (1, 1, 1), 0.3, 0.02, "small_radius3d"),  # T_lo = 0
        W.lattice(3, 18, 1 / 18, 0.1, seed=3),
        W.ring_pairs(400, 0.05, seed=5, dim=3),
    ]


@pytest.mark.parametrize("mode", [nnps.MODE_FP16_RCLL, nnps.MODE_FP64_BASELINE, nnps.MODE_RECHECK_ALL,
                                  nnps.MODE_FP32_RCLL],
                         ids=["fp16", "fp64", "recheck_all", "fp32"])
def test_dense_path_parity(ctx, mode):
    for ps in cases():
        want = oracle.search_ps(ps)
        ref = None
        for thr in (-1, 1, 40, 0):
            name = f"{ps.name}_m{mode}_t{thr}"
            print(f"[gpu] dense {name} n={ps.n}", flush=True)
            got = run(ctx, ps, mode, dense_min_union=thr)
            check(got, want, mode, name)
            st = got[3]
            if thr == 1:
                # every particle with a neighbour has a stencil of two or more: a dense row
                with_nb = int(np.count_nonzero(np.diff(want[0])))
                assert with_nb <= st["dense_rows"] <= ps.n and st["heavy_rows"] == 0, name
            if thr == -1:
                assert st["dense_rows"] == 0, name
                ref = st
            elif mode != nnps.MODE_FP32_RCLL:  # FP32 mode decides dense cells in FP64 (no band statistics)
                for k in STAT_KEYS:
                    assert st[k] == ref[k], (name, k, st[k], ref[k])
            assert st["outside_band_disagree"] == 0


def test_dense_capacity_fallback(ctx):
    """Union lists larger than their capacity: the build falls back to the block and
    long-row paths, with the same result."""
    ps = cases()[2]
    want = oracle.search_ps(ps)
    got = run(ctx, ps, nnps.MODE_FP16_RCLL, dense_min_union=1, dense_max_entries=1000)
    check(got, want, 0, "fallback")
    assert got[3]["dense_rows"] == 0 and got[3]["dense_entries"] == 0
    got = run(ctx, ps, nnps.MODE_FP16_RCLL, dense_min_union=1)
    assert got[3]["dense_entries"] > 1000


@pytest.mark.parametrize("grid", [1, 7, 4096])
def test_dense_grid_sizes(ctx, grid):
    ps = cases()[0]
    got = run(ctx, ps, nnps.MODE_FP16_RCLL, dense_min_union=1, dense_grid=grid)
    check(got, oracle.search_ps(ps), 0, f"grid{grid}")


def test_dense_batch_and_graph_replays(ctx):
    pss = [W.clustered(int(n), 50 + i, dim=3) for i, n in enumerate([3000, 25000, 800, 12000])]
    pss.insert(2, W.ParticleSet(np.zeros((0, 3)), (0, 0, 0), (1, 1, 1), 0.1, 0.1, "empty"))
    sets = [(torch.from_numpy(p.pos).cuda(), p.lo, p.hi, p.cell_size, p.radius) for p in pss]
    wants = [oracle.search_ps(p) for p in pss]
    ctx.set_tuning(dense_min_union=100)
    try:
        cells = ctx.cells()
        res, _ = nnps.search_batch(sets, ctx=ctx, cells=cells)
        assert cells.stats()["dense_rows"] > 0
        for r, w, p in zip(res, wants, pss):
            check(tuple(t.cpu().numpy() for t in r) + ({},), w, 0, p.name)
        gcells = ctx.cells()
        gcells.set_graphs(True)
        rps = [torch.empty_like(r[0]) for r in res]
        cols = [torch.empty(max(r[1].numel(), 1), dtype=torch.int32, device="cuda") for r in res]
        dists = [torch.empty(max(r[1].numel(), 1), dtype=torch.float32, device="cuda") for r in res]
        stream = torch.cuda.Stream()
        for rep in range(3):
            print(f"[gpu] dense graph replay {rep}", flush=True)
            with torch.cuda.stream(stream):
                gcells.batch_step(sets, rps, cols, dists, stream=stream)
            stream.synchronize()
            nnz = gcells.batch_nnz(stream=stream)
            for s, r in enumerate(res):
                k = r[1].numel()
                assert nnz[s] == k
                assert torch.equal(rps[s], r[0])
                assert torch.equal(cols[s][:k], r[1]) and torch.equal(dists[s][:k], r[2])
            torch.cuda.synchronize()
            _ = (sets[1][0] * 2).sum().item()
        cells.close()
        gcells.close()
    finally:
        ctx.set_tuning()


def upper(rp, col, dist):
    """The oracle's CSR restricted to entries j > i (half lists)."""
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    keep = col > rows
    hrp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows[keep], minlength=n), out=hrp[1:])
    return hrp, col[keep], dist[keep]


@pytest.mark.parametrize("mode", [nnps.MODE_FP16_RCLL, nnps.MODE_RECHECK_ALL], ids=["fp16", "recheck_all"])
@pytest.mark.parametrize("half", [False, True], ids=["full", "half"])
def test_dense_kept_bits(ctx, mode, half):
    """The FP16 dense count keeps its accepted bits for the fill once a call that
    synchronised has sized the scratch: on one structure the first search tests again in
    the fill (no scratch yet) and the second takes the kept bits; a bound too small for
    them (1 MiB, for a structure of several MiB) and the bits switched off (-1) test
    again. Every result is the oracle's, with the same statistics."""
    ps = W.clustered(60000, 43, dim=3)
    want = oracle.search_ps(ps)
    if half:
        want = upper(*want)
    pos = torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda()
    ref = None
    for mib in (0, 1, -1):
        ctx.set_tuning(dense_min_union=1, dense_bits_mib=mib)
        try:
            cells = ctx.cells()
            cells.set_half(half)
            for rep in range(3):
                name = f"bits{mib}_rep{rep}_m{mode}_h{int(half)}"
                print(f"[gpu] dense kept bits {name}", flush=True)
                rp, col, dist, _ = nnps.search(pos, ps.lo, ps.hi, ps.cell_size, ps.radius, mode=mode, ctx=ctx,
                                               cells=cells)
                check((rp.cpu().numpy(), col.cpu().numpy(), dist.cpu().numpy(), None), want, mode, name)
                st = cells.stats()
                assert st["dense_rows"] > 0 and st["outside_band_disagree"] == 0, name
                if ref is None:
                    ref = st
                for k in STAT_KEYS:
                    assert st[k] == ref[k], (name, k, st[k], ref[k])
            cells.close()
        finally:
            ctx.set_tuning()
