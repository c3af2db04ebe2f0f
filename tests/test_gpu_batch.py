"""GPU parity for batches: many uneven particle sets searched in one launch per pass,
the graph-captured step and its replays, and the long-row path (chunked sort + merge),
each set checked element by element against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2401_08586_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2401_08586_amd import nnps  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = nnps.Context(0)
    yield c
    c.close()


def as_sets(pss):
    return [(torch.from_numpy(np.ascontiguousarray(ps.pos)).cuda(), ps.lo, ps.hi, ps.cell_size, ps.radius)
            for ps in pss]


def check(got, ps, mode, name):
    rp, col, dist = (t.cpu().numpy() for t in got)
    wrp, wcol, wdist = oracle.search_ps(ps)
    np.testing.assert_array_equal(rp, wrp, err_msg=f"{name} row_ptr")
    np.testing.assert_array_equal(col, wcol, err_msg=f"{name} col")
    if mode in (nnps.MODE_FP64_BASELINE, nnps.MODE_FP32_RCLL):
        np.testing.assert_array_equal(dist.view(np.uint32), wdist.view(np.uint32), err_msg=f"{name} dist")
    else:
        wd = wdist.astype(np.float64)
        assert np.all(np.abs(dist - wd) <= 1e-6 * wd), name
        assert np.all(dist[wdist == 0] == 0)


def uneven_batch(dim=3, seed=0, k=7):
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(300), np.log(12000), size=k))).astype(int)
    sets = [W.clustered(int(n), seed * 100 + i, dim=dim) for i, n in enumerate(sizes)]
    sets.append(W.lattice(dim, 14 if dim == 3 else 60, 1 / (14 if dim == 3 else 60), 0.1, seed=seed))
    return sets


@pytest.mark.parametrize("mode", [nnps.MODE_FP16_RCLL, nnps.MODE_FP64_BASELINE, nnps.MODE_RECHECK_ALL,
                                  nnps.MODE_FP32_RCLL], ids=["fp16", "fp64", "recheck_all", "fp32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_batch_parity(ctx, dim, mode):
    pss = uneven_batch(dim, seed=dim)
    print(f"[gpu] batch dim={dim} mode={mode} sizes={[p.n for p in pss]}", flush=True)
    cells = ctx.cells()
    res, _ = nnps.search_batch(as_sets(pss), mode=mode, ctx=ctx, cells=cells)
    st = cells.stats()
    for got, ps in zip(res, pss):
        check(got, ps, mode, ps.name)
    assert st["nnz"] == sum(int(r[0][-1]) for r in res)
    assert st["outside_band_disagree"] == 0
    cells.close()


def test_batch_with_empty_and_tiny_sets(ctx):
    rng = np.random.default_rng(3)
    pss = [W.ParticleSet(np.zeros((0, 3)), (0, 0, 0), (1, 1, 1), 0.1, 0.1, "empty"),
           W.ParticleSet(rng.uniform(0, 1, (1, 3)), (0, 0, 0), (1, 1, 1), 0.1, 0.1, "one"),
           W.clustered(3000, 5, dim=3),
           W.ParticleSet(np.zeros((0, 3)), (0, 0, 0), (2, 2, 2), 0.2, 0.2, "empty2"),
           W.uniform(3, 5000, seed=6)]
    print("[gpu] batch with empty sets", flush=True)
    cells = ctx.cells()
    res, _ = nnps.search_batch(as_sets(pss), ctx=ctx, cells=cells)
    for got, ps in zip(res, pss):
        check(got, ps, 0, ps.name)
    cells.close()


def test_single_equals_batch(ctx):
    """A set's result is the same alone and inside a batch."""
    pss = uneven_batch(3, seed=9, k=5)
    cells = ctx.cells()
    res, _ = nnps.search_batch(as_sets(pss), ctx=ctx, cells=cells)
    for got, ps in zip(res, pss):
        alone = nnps.search(torch.from_numpy(ps.pos).cuda(), ps.lo, ps.hi, ps.cell_size, ps.radius, ctx=ctx)[:3]
        for x, y in zip(got, alone):
            assert torch.equal(x, y), ps.name
    cells.close()


@pytest.mark.parametrize("mode", [nnps.MODE_FP16_RCLL, nnps.MODE_FP32_RCLL], ids=["fp16", "fp32"])
def test_graph_step_replays(ctx, mode):
    """The captured step gives the eager result on every replay, also after the
    positions move (same sizes: the graph is replayed with the new pointers)."""
    pss = uneven_batch(3, seed=4, k=4)
    sets = as_sets(pss)
    eager_cells = ctx.cells()
    ref, _ = nnps.search_batch(sets, mode=mode, ctx=ctx, cells=eager_cells)
    cells = ctx.cells()
    cells.set_graphs(True)
    rps = [torch.empty_like(r[0]) for r in ref]
    cols = [torch.empty(r[1].numel() + 64, dtype=torch.int32, device="cuda") for r in ref]
    dists = [torch.empty(r[2].numel() + 64, dtype=torch.float32, device="cuda") for r in ref]
    stream = torch.cuda.Stream()
    print(f"[gpu] graph replays mode={mode}", flush=True)
    for rep in range(4):
        with torch.cuda.stream(stream):
            cells.batch_step(sets, rps, cols, dists, mode=mode, stream=stream)
        cells.batch_nnz_enqueue(stream=stream)
        nnz = cells.batch_nnz_fetch()
        assert nnz == cells.batch_nnz(stream=stream)
        for s, (r, k) in enumerate(zip(ref, nnz)):
            assert k == r[1].numel()
            assert torch.equal(rps[s], r[0])
            assert torch.equal(cols[s][:k], r[1])
            assert torch.equal(dists[s][:k], r[2])
        # eager work between replays
        torch.cuda.synchronize()
        _ = (sets[0][0] * 2.0).sum().item()
    # move the particles (same sizes): replay reads the new positions
    moved = [W.ParticleSet(W.step_displacement(ps, 1, seed=7), ps.lo, ps.hi, ps.cell_size, ps.radius, ps.name)
             for ps in pss]
    msets = as_sets(moved)
    nnz_new = None
    for rep in range(2):
        with torch.cuda.stream(stream):
            mrps = [torch.empty_like(r) for r in rps]
            big = [torch.empty(c.numel() + 20000, dtype=torch.int32, device="cuda") for c in cols]
            bigd = [torch.empty(c.numel() + 20000, dtype=torch.float32, device="cuda") for c in cols]
            cells.batch_step(msets, mrps, big, bigd, mode=mode, stream=stream)
        stream.synchronize()
        nnz_new = cells.batch_nnz(stream=stream)
        for s, ps in enumerate(moved):
            check((mrps[s], big[s][:nnz_new[s]], bigd[s][:nnz_new[s]]), ps, mode, ps.name + "_moved")
    cells.close()
    eager_cells.close()


def test_long_rows_chunked_merge(ctx):
    """Rows far longer than the LDS sort chunk: chunks sorted, then merged pairwise."""
    rng = np.random.default_rng(8)
    pos = np.clip(np.concatenate([rng.normal(0.5, 0.015, size=(2500, 3)), rng.uniform(0, 1, size=(500, 3))]), 0, 1)
    ps = W.ParticleSet(pos, (0, 0, 0), (1, 1, 1), 0.06, 0.06, "dense_ball")
    for keys in (64, 256, 0):
        ctx.set_tuning(block_target=56, long_rows_grid=256, long_rows_keys=keys, dense_min_union=-1)
        print(f"[gpu] long rows keys={keys}", flush=True)
        for mode in (nnps.MODE_FP16_RCLL, nnps.MODE_FP64_BASELINE, nnps.MODE_FP32_RCLL):
            cells = ctx.cells()
            rp, col, dist, _ = nnps.search(torch.from_numpy(ps.pos).cuda(), ps.lo, ps.hi, ps.cell_size, ps.radius,
                                           mode=mode, ctx=ctx, cells=cells)
            st = cells.stats()
            assert st["heavy_rows"] > 0
            check((rp, col, dist), ps, mode, f"{ps.name}_k{keys}_m{mode}")
            cells.close()
    ctx.set_tuning()


@pytest.mark.parametrize("bt", [16, 32, 64, 128])
def test_block_target_tuning_keeps_results(ctx, bt):
    ps = W.lattice(3, 20, 1 / 20, 0.1, seed=2)
    ctx.set_tuning(block_target=bt)
    print(f"[gpu] block_target={bt}", flush=True)
    rp, col, dist, _ = nnps.search(torch.from_numpy(ps.pos).cuda(), ps.lo, ps.hi, ps.cell_size, ps.radius, ctx=ctx)
    check((rp, col, dist), ps, 0, f"bt{bt}")
    ctx.set_tuning()


def test_batch_global_indices_past_the_packed_key_range(ctx):
    """A batch whose global particle indices pass 2^22: the fill ranks a block's union
    by original index with a 32-bit key holding the index above the union position. The
    first set (4.5M uniform points in random order) has unions whose index range does not
    fit that key (sampled rows + properties of the whole CSR); the second lies past 2^22
    in the global index space (checked whole)."""
    big = W.uniform(3, 4_500_000, seed=21, radius_factor=1.8)
    small = W.clustered(20000, 22, dim=3)
    print("[gpu] batch past 2^22 global indices", flush=True)
    cells = ctx.cells()
    res, _ = nnps.search_batch(as_sets([big, small]), ctx=ctx, cells=cells)
    check(res[1], small, 0, "small_after_big")
    rp, col, dist = res[0]
    rpc = rp.cpu().numpy()
    rows = np.random.default_rng(5).choice(big.n, size=3000, replace=False)
    wrp, wcol, wdist = oracle.search_rows(big.pos, big.lo, big.hi, big.cell_size, big.radius, rows)
    np.testing.assert_array_equal(np.diff(rpc)[rows], np.diff(wrp))
    got = np.concatenate([col[int(rpc[r]):int(rpc[r + 1])].cpu().numpy() for r in rows])
    np.testing.assert_array_equal(got, wcol)
    assert int(col.min()) >= 0 and int(col.max()) < big.n
    down = torch.nonzero(col[1:] <= col[:-1]).flatten().cpu().numpy() + 1
    lens = np.diff(rpc)
    assert set(down.tolist()) <= set(rpc[1:-1][lens[1:] > 0].tolist())
    cells.close()


def test_autotune_on_the_gpu(ctx, tmp_path):
    """The autotuner on a small clustered batch: coordinate descent over a reduced space
    times real graph-free steps on the GPU, leaves its choice on the context, and the
    search with the chosen shapes gives the oracle's lists; a second call with the same
    cache file takes the cached choice without timing anything."""
    from paper_2401_08586_amd import autotune as A
    pss = [W.clustered(n, 70 + i, dim=3) for i, n in enumerate([4000, 12000, 30000])]
    sets = as_sets(pss)
    space = {"block_target": [48, 80], "dense_min_union": [1, 512, -1], "dense_grid": [256, 2048]}
    path = str(tmp_path / "tune.json")
    try:
        print("[gpu] autotune", flush=True)
        best, ms, evals = A.tune(ctx, sets, pss, nnps.MODE_FP16_RCLL, steps=2, warmup=1, space=space,
                                 cache=A.Cache(path), sweeps=1)
        assert evals >= 2 and ms > 0
        for k, vals in space.items():
            assert best[k] in vals or best[k] == A.DEFAULTS[k]
            assert ctx.get_tuning()[k] == best[k]
        res, _ = nnps.search_batch(sets, ctx=ctx)
        for r, p in zip(res, pss):
            check(r, p, nnps.MODE_FP16_RCLL, f"tuned_{p.name}")
        best2, ms2, evals2 = A.tune(ctx, sets, pss, nnps.MODE_FP16_RCLL, space=space, cache=A.Cache(path))
        assert best2 == best and evals2 == 0 and ms2 is None
    finally:
        ctx.set_tuning()
